// D2Q9 contexts of the MCLG library (host side).
//
// Collision rules (Sec. "A D2Q9 implementation", classes numbered as the
// lambda_c of Eq. (D2Q9MOmega)); see mclg.h for the full statement.  Every
// site runs the literal sub-collision loop on the device; the host builds
// the integer rule table, the layout and the Poisson start laws.
#include "d2q9.h"

#include <algorithm>
#include <cstring>
#include <numeric>

#include "tables.h"

namespace mclg {
namespace {

constexpr int kVx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kVy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr uint64_t kW1296[9] = {576, 144, 144, 144, 144, 36, 36, 36, 36};  // 1296 w_i
constexpr uint64_t kPad = 128;
constexpr uint32_t kTile = 256;
constexpr uint32_t kPoisCap9 = 1024;

inline uint64_t up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// Class (1..9) of the swap of {i, j} for {k, l}, two different pairs of one
// total momentum p: by |p|^2, then by whether a rest particle takes part,
// then (p = 0) by the kinds of the two pairs.
int swap_class(int i, int j, int k, int l) {
  const int px = kVx[i] + kVx[j], py = kVy[i] + kVy[j];
  switch (px * px + py * py) {
    case 2: return 1;
    case 4: return 9;
    case 1: return (i == 0 || j == 0 || k == 0 || l == 0) ? 7 : 8;
    default: break;
  }
  // zero momentum: {0,0}, an axis pair {v, -v} or a diagonal pair
  auto kind = [](int v) { return v == 0 ? 0 : (v <= 4 ? 1 : 2); };
  static constexpr int table[3][3] = {{0, 2, 3}, {2, 5, 4}, {3, 4, 6}};
  return table[kind(i)][kind(k)];
}

}  // namespace

bool build_rules9(const uint32_t *lam, std::vector<uint32_t> &rules, uint32_t &D) {
  if (!lam) return false;
  uint64_t L = 1;
  for (int c = 0; c < 9; ++c) {
    const uint64_t num = lam[2 * c], den = lam[2 * c + 1];
    if (den == 0 || num > den) return false;
    L = std::lcm(L, den);
    if (L >= (1u << 25)) return false;
  }
  const uint64_t D64 = L * 128;
  D = (uint32_t)D64;
  constexpr uint32_t kNoChange = 0x2492492u;  // 2 in each of the nine 3-bit fields
  rules.assign(81 * kRule9Words, 0u);
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      uint32_t *e = &rules[(i * 9 + j) * kRule9Words];
      for (int q = 0; q < 4; ++q) e[q] = (uint32_t)D64;
      for (int q = 0; q < 5; ++q) e[4 + q] = kNoChange;
      const uint64_t mA = i == j ? 1 : 2;
      uint64_t cum = 0;
      int nt = 0;
      for (int k = 0; k < 9; ++k)
        for (int l = k; l < 9; ++l) {
          if (kVx[k] + kVx[l] != kVx[i] + kVx[j] || kVy[k] + kVy[l] != kVy[i] + kVy[j]) continue;
          if ((k == i && l == j) || (k == j && l == i)) continue;
          const int c = swap_class(i, j, k, l);
          const uint64_t mB = k == l ? 1 : 2;
          const uint64_t to = mB * kW1296[k] * kW1296[l], from = mA * kW1296[i] * kW1296[j];
          const uint64_t base = D64 / lam[2 * c - 1] * lam[2 * c - 2];  // D lambda_c
          // the weight ratio is a power of two, at least 2^-7, so this is exact
          const uint64_t w = to >= from ? base : base * to / from;
          if (nt >= 4) return false;
          cum += w;
          e[nt] = (uint32_t)cum;
          int delta[9] = {2, 2, 2, 2, 2, 2, 2, 2, 2};
          delta[i] -= 1;
          delta[j] -= 1;
          delta[k] += 1;
          delta[l] += 1;
          uint32_t packed = 0;
          for (int v = 0; v < 9; ++v) packed |= (uint32_t)delta[v] << (3 * v);
          e[4 + nt] = packed;
          ++nt;
        }
      if (cum > D64) return false;
    }
  return true;
}

std::vector<uint32_t> device_rules9(const std::vector<uint32_t> &rules) {
  std::vector<uint32_t> dev(81 * kRule9DevWords, 0u);
  for (int p = 0; p < 81; ++p) {
    const uint32_t *e = &rules[p * kRule9Words];
    uint32_t *o = &dev[p * kRule9DevWords];
    for (int q = 0; q < 4; ++q) o[q] = e[q];
    for (int q = 0; q < 5; ++q) {
      int32_t K = 0;
      uint16_t dk[8];
      for (int j = 0; j < 8; ++j) {
        K += (int32_t)((e[4 + q] >> (3 * j)) & 7u) - 2;
        dk[j] = (uint16_t)K;
      }
      for (int m = 0; m < 4; ++m) o[4 + 4 * q + m] = dk[2 * m] | (uint32_t)dk[2 * m + 1] << 16;
    }
  }
  return dev;
}

int d2q9_layout(const mclg_config *cfg, D2Ctx &d) {
  if (!cfg->Ly || !cfg->lambda9 || cfg->C < 0 || cfg->C > 4096) return MCLG_E_INVAL;
  if (cfg->flags & ~(uint32_t)MCLG_FLAG_NO_STREAM) return MCLG_E_INVAL;
  if (!build_rules9(cfg->lambda9, d.rules, d.D)) return MCLG_E_INVAL;
  d.rules_dev = device_rules9(d.rules);
  d.n = cfg->n_replicas;
  d.flags = cfg->flags;
  d.C = cfg->C;
  d.seed = cfg->seed;
  d.Lx.assign(cfg->L, cfg->L + d.n);
  d.Ly.assign(cfg->Ly, cfg->Ly + d.n);
  d.rid.resize(d.n);
  d.dense.resize(d.n);
  d.reps.resize(d.n);
  d.tiles.clear();
  uint64_t elems = 0, dense = 0;
  for (uint32_t r = 0; r < d.n; ++r) {
    const uint64_t Lx = d.Lx[r], Ly = d.Ly[r];
    if (!Lx || !Ly || Lx * Ly > (1ull << 28)) return MCLG_E_INVAL;
    if (cfg->replica_id && cfg->replica_id[r] >= (1ull << 32)) return MCLG_E_INVAL;
    d.rid[r] = cfg->replica_id ? cfg->replica_id[r] : r;
    const uint64_t S = Lx * Ly, stride = up(S, kPad);
    Rep9 &rp = d.reps[r];
    rp.off = elems;
    rp.Lx = (uint32_t)Lx;
    rp.Ly = (uint32_t)Ly;
    rp.S = (uint32_t)S;
    rp.stride = (uint32_t)stride;
    rp.rid = (uint32_t)d.rid[r];
    rp.pad = 0;
    d.dense[r] = dense;
    elems += 9 * stride;
    dense += 9 * S;
    for (uint64_t s0 = 0; s0 < S; s0 += kTile) d.tiles.push_back(Tile9{r, (uint32_t)s0});
  }
  d.state_bytes = elems * sizeof(uint16_t);
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o = up(o + bytes, 256);
    return at;
  };
  d.o_err = take(256);
  d.o_reps = take(sizeof(Rep9) * d.n);
  d.o_tiles = take(sizeof(Tile9) * d.tiles.size());
  d.o_rules = take(sizeof(uint32_t) * d.rules_dev.size());
  {
    std::vector<uint32_t> ids(d.n);
    std::vector<uint64_t> S(d.n);
    for (uint32_t r = 0; r < d.n; ++r) {
      ids[r] = r;
      S[r] = d.Lx[r] * d.Ly[r];
    }
    d.mplan = plan_moments(ids.data(), S.data(), d.n);
  }
  d.o_mseg = take(sizeof(MomSeg) * d.mplan.segs.size());
  d.o_mrun = take(sizeof(uint32_t) * d.mplan.run_seg.size());
  d.o_mslot = take(sizeof(uint32_t) * d.mplan.run_slot.size());
  d.o_mpart = take(sizeof(uint64_t) * kMom9Rec * d.mplan.segs.size());
  d.o_mout = take(sizeof(uint64_t) * kMom9Out * d.n);
  d.o_pdesc = take(sizeof(PoisDesc) * 9 * d.n);
  d.o_pool = take(sizeof(uint32_t) * kPoisCap9 * 9 * d.n);
  d.o_dense = take(sizeof(uint64_t) * d.n);
  d.ws_bytes = o;
  return MCLG_OK;
}

static int hip_rc(D2Ctx &d, hipError_t e) {
  if (e == hipSuccess) return MCLG_OK;
  d.last_hip = (int)e;
  return MCLG_E_HIP;
}

int d2q9_init(D2Ctx &d, const mclg_config *cfg, const mclg_init_spec *init) {
  d.state = static_cast<uint16_t *>(cfg->state);
  d.ws = static_cast<uint8_t *>(cfg->workspace);
  d.stream = reinterpret_cast<hipStream_t>(cfg->stream);
  if (cfg->state_bytes < d.state_bytes || cfg->workspace_bytes < d.ws_bytes) return MCLG_E_INVAL;
  std::vector<PoisDesc> pdesc(9 * d.n);
  std::vector<uint32_t> pool;
  if (init->kind == MCLG_INIT_POISSON) {
    if (!init->rho || !init->u0) return MCLG_E_INVAL;
    pool.assign((size_t)kPoisCap9 * 9 * d.n, 0u);
    for (uint32_t r = 0; r < d.n; ++r) {
      const double rho = init->rho[r], ux = init->u0[r], uy = init->u0y ? init->u0y[r] : 0.0;
      if (!(rho >= 0.0) || !(ux >= -1.0 && ux <= 1.0) || !(uy >= -1.0 && uy <= 1.0))
        return MCLG_E_INVAL;
      // Eq. (D2Q9eqdist) as (rho Fx[vx]) Fy[vy], F the unit-density D1Q3 law
      double fx[3], fy[3];
      feq(1.0, ux, fx);
      feq(1.0, uy, fy);
      for (int i = 0; i < 9; ++i) {
        const double mu = (rho * fx[kVx[i] + 1]) * fy[kVy[i] + 1];
        uint32_t k_lo = 0;
        std::vector<uint64_t> full;
        if (!poisson_full(mu, k_lo, full)) return MCLG_E_INVAL;
        CompactLaw cl = compact(k_lo, full);
        if (cl.thr.size() > kPoisCap9) return MCLG_E_INVAL;
        PoisDesc &pd = pdesc[9 * r + i];
        pd.off = (uint32_t)((9 * r + i) * kPoisCap9);
        pd.k_first = cl.k_first;
        pd.nthr = (uint32_t)cl.thr.size();
        pd.pad = 0;
        std::copy(cl.thr.begin(), cl.thr.end(), pool.begin() + pd.off);
      }
    }
  } else if (init->kind != MCLG_INIT_COUNTS || !init->counts) {
    return MCLG_E_INVAL;
  }
  auto put = [&](uint64_t off, const void *src, size_t bytes) {
    return bytes ? hipMemcpyAsync(d.ws + off, src, bytes, hipMemcpyHostToDevice, d.stream)
                 : hipSuccess;
  };
  std::vector<uint32_t> zero(64, 0u);
  hipError_t e = put(d.o_err, zero.data(), 256);
  if (!e) e = put(d.o_reps, d.reps.data(), sizeof(Rep9) * d.n);
  if (!e) e = put(d.o_tiles, d.tiles.data(), sizeof(Tile9) * d.tiles.size());
  if (!e) e = put(d.o_rules, d.rules_dev.data(), sizeof(uint32_t) * d.rules_dev.size());
  if (!e) e = put(d.o_dense, d.dense.data(), sizeof(uint64_t) * d.n);
  if (!e) e = put(d.o_mseg, d.mplan.segs.data(), sizeof(MomSeg) * d.mplan.segs.size());
  if (!e) e = put(d.o_mrun, d.mplan.run_seg.data(), sizeof(uint32_t) * d.mplan.run_seg.size());
  if (!e) e = put(d.o_mslot, d.mplan.run_slot.data(), sizeof(uint32_t) * d.mplan.run_slot.size());
  if (!e && !pool.empty()) e = put(d.o_pdesc, pdesc.data(), sizeof(PoisDesc) * pdesc.size());
  if (!e && !pool.empty()) e = put(d.o_pool, pool.data(), sizeof(uint32_t) * pool.size());
  const Rep9 *reps = reinterpret_cast<const Rep9 *>(d.ws + d.o_reps);
  const Tile9 *tiles = reinterpret_cast<const Tile9 *>(d.ws + d.o_tiles);
  if (!e && init->kind == MCLG_INIT_POISSON)
    e = launch_init9_poisson(d.stream, d.state, reps, tiles, (uint32_t)d.tiles.size(),
                             reinterpret_cast<const PoisDesc *>(d.ws + d.o_pdesc),
                             reinterpret_cast<const uint32_t *>(d.ws + d.o_pool), d.seed,
                             reinterpret_cast<uint32_t *>(d.ws + d.o_err));
  if (!e && init->kind == MCLG_INIT_COUNTS)
    e = launch_init9_counts(d.stream, d.state, reps, tiles, (uint32_t)d.tiles.size(),
                            reinterpret_cast<const uint64_t *>(d.ws + d.o_dense), init->counts);
  // the host vectors above must outlive the copies
  if (!e) e = hipStreamSynchronize(d.stream);
  d.t = 0;
  return hip_rc(d, e);
}

int d2q9_step(D2Ctx &d, uint64_t n_steps) {
  Step9 a{};
  a.state = d.state;
  a.reps = reinterpret_cast<const Rep9 *>(d.ws + d.o_reps);
  a.tiles = reinterpret_cast<const Tile9 *>(d.ws + d.o_tiles);
  a.rules = reinterpret_cast<const uint32_t *>(d.ws + d.o_rules);
  a.err = reinterpret_cast<uint32_t *>(d.ws + d.o_err);
  a.seed = d.seed;
  a.D = d.D;
  a.no_stream = (d.flags & MCLG_FLAG_NO_STREAM) ? 1u : 0u;
  a.C = d.C;
  for (uint64_t i = 0; i < n_steps; ++i) {
    a.t = (uint64_t)d.t;
    hipError_t e = launch_step9(d.stream, a, (uint32_t)d.tiles.size());
    if (e) return hip_rc(d, e);
    ++d.t;
  }
  return MCLG_OK;
}

int d2q9_histogram(D2Ctx &d, uint32_t n_bins, uint64_t *hist) {
  // 9 * n_bins uint32 of LDS per block: at most 36 KB
  const hipError_t e = launch_histogram9(
      d.stream, d.state, reinterpret_cast<const Rep9 *>(d.ws + d.o_reps),
      reinterpret_cast<const Tile9 *>(d.ws + d.o_tiles), (uint32_t)d.tiles.size(), n_bins,
      reinterpret_cast<unsigned long long *>(hist));
  return hip_rc(d, e);
}

int d2q9_check(D2Ctx &d) {
  uint32_t err = 0;
  hipError_t e = hipMemcpyAsync(&err, d.ws + d.o_err, sizeof(err), hipMemcpyDeviceToHost, d.stream);
  if (!e) e = hipStreamSynchronize(d.stream);
  if (e) return hip_rc(d, e);
  return err ? MCLG_E_RANGE : MCLG_OK;
}

int d2q9_get_counts(D2Ctx &d, uint32_t r, uint16_t *out) {
  if (r >= d.n || !out) return MCLG_E_INVAL;
  const Rep9 &rp = d.reps[r];
  std::vector<uint16_t> raw((size_t)9 * rp.stride);
  hipError_t e = hipMemcpyAsync(raw.data(), d.state + rp.off, raw.size() * 2,
                                hipMemcpyDeviceToHost, d.stream);
  if (!e) e = hipStreamSynchronize(d.stream);
  if (e) return hip_rc(d, e);
  const bool ns = (d.flags & MCLG_FLAG_NO_STREAM) != 0;
  const uint64_t tx = ns ? 0 : (uint64_t)d.t % rp.Lx, ty = ns ? 0 : (uint64_t)d.t % rp.Ly;
  for (int i = 0; i < 9; ++i)
    for (uint64_t y = 0; y < rp.Ly; ++y)
      for (uint64_t x = 0; x < rp.Lx; ++x) {
        // logical (x, y) sits at ((x - vx t) mod Lx, (y - vy t) mod Ly)
        int64_t px = ((int64_t)x - kVx[i] * (int64_t)tx) % (int64_t)rp.Lx;
        int64_t py = ((int64_t)y - kVy[i] * (int64_t)ty) % (int64_t)rp.Ly;
        px += px < 0 ? rp.Lx : 0;
        py += py < 0 ? rp.Ly : 0;
        out[(uint64_t)i * rp.S + y * rp.Lx + x] =
            raw[(uint64_t)i * rp.stride + (uint64_t)py * rp.Lx + (uint64_t)px];
      }
  return d2q9_check(d);
}

int d2q9_moments(D2Ctx &d, mclg_moments9_t *out) {
  if (!out) return MCLG_E_INVAL;
  static_assert(sizeof(mclg_moments9_t) == kMom9Out * sizeof(int64_t), "result layout");
  MomArgs m;
  m.state = d.state;
  m.reps = reinterpret_cast<const Rep9 *>(d.ws + d.o_reps);
  m.t9 = (uint64_t)d.t;
  m.no_stream = (d.flags & MCLG_FLAG_NO_STREAM) ? 1u : 0u;
  m.segs = reinterpret_cast<const MomSeg *>(d.ws + d.o_mseg);
  m.n_segs = (uint32_t)d.mplan.segs.size();
  m.run_seg = reinterpret_cast<const uint32_t *>(d.ws + d.o_mrun);
  m.run_slot = reinterpret_cast<const uint32_t *>(d.ws + d.o_mslot);
  m.n_runs = d.n;
  m.partial = reinterpret_cast<unsigned long long *>(d.ws + d.o_mpart);
  m.out = reinterpret_cast<long long *>(d.ws + d.o_mout);
  hipError_t e = launch_moments9(d.stream, m);
  if (!e) e = hipMemcpyAsync(out, d.ws + d.o_mout, sizeof(mclg_moments9_t) * d.n,
                             hipMemcpyDeviceToHost, d.stream);
  if (!e) e = hipStreamSynchronize(d.stream);
  if (e) return hip_rc(d, e);
  return d2q9_check(d);
}

}  // namespace mclg
