// Exact collision and Poisson tables (host side of the MCLG library).
//
// Collision law (Sec. "The Monte Carlo Lattice Gas algorithm", Eq. (select),
// Eq. (omega), and the D1Q3 transition table of Sec. "A D1Q3
// implementation"): on the fiber of fixed N and J a site is described by its
// rest count n0 (a = n_-1, c = n_+1).  One sub-collision picks an ordered
// pair of distinct particles; a {-1,+1} pair comes to rest with probability
// lambda, a {0,0} pair leaves as {-1,1} or {1,-1} with lambda/16 each.  With
// lambda = p/q and the common denominator D1 = 8 q N (N-1) the one-step
// transition weights are the integers
//     n0 -> n0 + 2 : 16 p a c
//     n0 -> n0 - 2 : p n0 (n0 - 1)
//     n0 -> n0     : D1 - (the two above)
// and C sub-collisions are the C-th power (entries are exact multiprecision
// integers, each row sums to D1^C).  For C = infinity the law is the fiber's
// stationary distribution, proportional to 4^n0 N!/(a! n0! c!) by detailed
// balance (Eq. (transprob)).  Thresholds are floor(2^32 * cumulative).
//
// Galilean-invariant acceptance (the remark after Eq. (D1Q3relax)): lambda
// = lambda~ / sqrt(1 + 3 U^2) with the site's own U = J / N, which is
// lambda~ N / sqrt(N^2 + 3 J^2).  It is irrational in general, so each fiber
// uses it rounded down to 32 fractional bits in two exact integer steps,
//     g = floor(2^32 N / sqrt(N^2 + 3 J^2)),   p = floor(g num / den),
// and then lambda = p / 2^32 exactly (q = 2^32 in the weights above).
#include "tables.h"

#include "device.h"  // kFixedStride

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>

namespace mclg {
namespace {

// ---------------------------------------------------------------------------
// Unsigned multiprecision integer, 64-bit limbs, little endian.
// ---------------------------------------------------------------------------
constexpr int kMaxLimbs = 72;  // 4608 bits

struct Big {
  int n = 0;                   // limbs in use
  uint64_t w[kMaxLimbs];
};

using u128 = unsigned __int128;

inline void big_set(Big &a, uint64_t v) {
  a.n = v ? 1 : 0;
  a.w[0] = v;
}
inline void big_norm(Big &a) {
  while (a.n && a.w[a.n - 1] == 0) --a.n;
}
// acc += x * m  (m < 2^64); returns false on overflow of the fixed width
inline bool big_fma(Big &acc, const Big &x, uint64_t m) {
  if (!m || !x.n) return true;
  int top = std::max(acc.n, x.n + 1);
  if (top > kMaxLimbs) return false;
  for (int i = acc.n; i < top; ++i) acc.w[i] = 0;
  uint64_t carry = 0;
  int i = 0;
  for (; i < x.n; ++i) {
    u128 t = (u128)x.w[i] * m + acc.w[i] + carry;
    acc.w[i] = (uint64_t)t;
    carry = (uint64_t)(t >> 64);
  }
  for (; carry; ++i) {
    if (i >= kMaxLimbs) return false;
    if (i >= top) { acc.w[i] = 0; top = i + 1; }
    u128 t = (u128)acc.w[i] + carry;
    acc.w[i] = (uint64_t)t;
    carry = (uint64_t)(t >> 64);
  }
  acc.n = std::max(top, i);
  big_norm(acc);
  return true;
}
inline bool big_mul(Big &a, uint64_t m) {
  Big r;
  r.n = 0;
  if (!big_fma(r, a, m)) return false;
  a = r;
  return true;
}
inline bool big_add(Big &a, const Big &b) {
  int top = std::max(a.n, b.n);
  for (int i = a.n; i < top; ++i) a.w[i] = 0;
  uint64_t carry = 0;
  for (int i = 0; i < top; ++i) {
    u128 t = (u128)a.w[i] + (i < b.n ? b.w[i] : 0) + carry;
    a.w[i] = (uint64_t)t;
    carry = (uint64_t)(t >> 64);
  }
  a.n = top;
  if (carry) {
    if (top >= kMaxLimbs) return false;
    a.w[a.n++] = carry;
  }
  return true;
}
// a /= d (exact, small d)
inline void big_div_small(Big &a, uint64_t d) {
  u128 rem = 0;
  for (int i = a.n - 1; i >= 0; --i) {
    u128 cur = (rem << 64) | a.w[i];
    a.w[i] = (uint64_t)(cur / d);
    rem = cur % d;
  }
  big_norm(a);
}
inline int big_cmp(const Big &a, const Big &b) {
  if (a.n != b.n) return a.n < b.n ? -1 : 1;
  for (int i = a.n - 1; i >= 0; --i)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
  return 0;
}
inline int big_bits(const Big &a) {
  if (!a.n) return 0;
  return 64 * (a.n - 1) + (64 - __builtin_clzll(a.w[a.n - 1]));
}
// Top 64 bits of a (as if a were shifted right so its bit length is <= 64 +
// extra), i.e. floor(a / 2^sh) for the given shift.
inline uint64_t big_shr64(const Big &a, int sh) {
  int limb = sh / 64, bit = sh % 64;
  auto get = [&](int i) -> uint64_t { return i < a.n && i >= 0 ? a.w[i] : 0; };
  uint64_t lo = get(limb), hi = get(limb + 1);
  return bit ? (lo >> bit) | (hi << (64 - bit)) : lo;
}
// compare q * d with s * 2^32 exactly
inline int cmp_qd_s32(uint64_t q, const Big &d, const Big &s) {
  Big lhs;
  lhs.n = 0;
  big_fma(lhs, d, q);
  Big rhs;
  rhs.n = 0;
  big_fma(rhs, s, (uint64_t)1 << 32);
  return big_cmp(lhs, rhs);
}
// floor(2^32 s / d), 0 <= s <= d: a 64-bit estimate from the leading bits,
// corrected by exact multiprecision comparison.
uint64_t quantise(const Big &s, const Big &d) {
  if (!s.n) return 0;
  int c = big_cmp(s, d);
  if (c == 0) return (uint64_t)1 << 32;
  int db = big_bits(d);
  int sh = db > 62 ? db - 62 : 0;
  uint64_t dt = big_shr64(d, sh);          // d / 2^sh, in [2^61, 2^62)
  uint64_t st = big_shr64(s, sh);          // s / 2^sh
  uint64_t q = (uint64_t)(((u128)st << 32) / (dt ? dt : 1));
  if (q > ((uint64_t)1 << 32)) q = (uint64_t)1 << 32;
  while (q > 0 && cmp_qd_s32(q, d, s) > 0) --q;
  while (cmp_qd_s32(q + 1, d, s) <= 0) ++q;
  return q;
}

struct Fiber {
  uint32_t N, absJ, m, par;
  uint64_t n0(uint32_t k) const { return par + 2ull * k; }
  uint64_t a(uint32_t k) const { return (N - n0(k) - absJ) / 2; }
  uint64_t c(uint32_t k) const { return (N - n0(k) + absJ) / 2; }
};

inline Fiber fiber(uint32_t N, uint32_t absJ) {
  Fiber f;
  f.N = N;
  f.absJ = absJ;
  f.m = (N - absJ) / 2 + 1;
  f.par = (N - absJ) & 1u;
  return f;
}

// Full-fiber quantised thresholds of one row (m - 1 values).
// Finite C: band-limited propagation of e_{k0} through the weight matrix.
bool row_finite(const Fiber &f, int32_t C, uint64_t p, uint64_t q, uint32_t k0,
                std::vector<uint64_t> &out, std::vector<Big> &va, std::vector<Big> &vb) {
  const uint32_t m = f.m;
  out.assign(m ? m - 1 : 0, 0);
  if (m <= 1) return true;
  const uint64_t D1 = 8ull * q * f.N * (f.N - 1ull);
  const uint32_t lo_lim = k0 > (uint32_t)C ? k0 - (uint32_t)C : 0;
  const uint32_t hi_lim = std::min<uint64_t>(m - 1, (uint64_t)k0 + (uint64_t)C);
  const uint32_t W = hi_lim - lo_lim + 1;
  va.resize(W);
  vb.resize(W);
  for (auto &b : va) b.n = 0;
  big_set(va[k0 - lo_lim], 1);
  uint32_t lo = k0, hi = k0;  // current support
  for (int32_t s = 0; s < C; ++s) {
    uint32_t nlo = lo > lo_lim ? lo - 1 : lo;
    uint32_t nhi = hi < hi_lim ? hi + 1 : hi;
    for (uint32_t k = nlo; k <= nhi; ++k) vb[k - lo_lim].n = 0;
    for (uint32_t k = lo; k <= hi; ++k) {
      const Big &x = va[k - lo_lim];
      if (!x.n) continue;
      uint64_t up = 16ull * p * f.a(k) * f.c(k);
      uint64_t n0 = f.n0(k);
      uint64_t dn = n0 >= 2 ? p * n0 * (n0 - 1) : 0;
      if (!big_fma(vb[k - lo_lim], x, D1 - up - dn)) return false;
      if (up && !big_fma(vb[k + 1 - lo_lim], x, up)) return false;
      if (dn && !big_fma(vb[k - 1 - lo_lim], x, dn)) return false;
    }
    std::swap(va, vb);
    lo = nlo;
    hi = nhi;
  }
  Big total;
  big_set(total, 1);
  for (int32_t s = 0; s < C; ++s)
    if (!big_mul(total, D1)) return false;
  Big cum;
  cum.n = 0;
  for (uint32_t k = 0; k + 1 < m; ++k) {
    if (k < lo) { out[k] = 0; continue; }
    if (k > hi) { out[k] = (uint64_t)1 << 32; continue; }
    if (!big_add(cum, va[k - lo_lim])) return false;
    out[k] = quantise(cum, total);
  }
  return true;
}

bool row_equilibrium(const Fiber &f, std::vector<uint64_t> &out) {
  const uint32_t m = f.m;
  out.assign(m ? m - 1 : 0, 0);
  if (m <= 1) return true;
  // weights 4^n0 N! / (a! n0! c!) = 4^n0 * binom(N, a) * binom(N - a, c)
  std::vector<Big> w(m);
  Big total;
  total.n = 0;
  for (uint32_t k = 0; k < m; ++k) {
    uint64_t a = f.a(k), c = f.c(k), n0 = f.n0(k);
    Big &b = w[k];
    big_set(b, 1);
    for (uint64_t i = 0; i < a; ++i) {  // binom(N, a)
      if (!big_mul(b, f.N - i)) return false;
      big_div_small(b, i + 1);
    }
    for (uint64_t i = 0; i < c; ++i) {  // binom(N - a, c)
      if (!big_mul(b, f.N - a - i)) return false;
      big_div_small(b, i + 1);
    }
    for (uint64_t i = 0; i < n0; i += 16) {
      uint64_t e = std::min<uint64_t>(16, n0 - i);
      if (!big_mul(b, (uint64_t)1 << (2 * e))) return false;
    }
    if (!big_add(total, b)) return false;
  }
  Big cum;
  cum.n = 0;
  for (uint32_t k = 0; k + 1 < m; ++k) {
    if (!big_add(cum, w[k])) return false;
    out[k] = quantise(cum, total);
  }
  return true;
}

std::mutex g_cache_mu;
std::map<std::tuple<int32_t, uint32_t, uint32_t, uint32_t, bool>,
         std::shared_ptr<const CollisionTables>>
    g_cache;

}  // namespace

uint64_t galilean_lambda_q(uint32_t num, uint32_t den, uint32_t N, uint32_t absJ) {
  uint64_t g = (uint64_t)1 << 32;
  if (absJ && N) {
    const u128 n2 = (u128)N * N;
    const uint64_t x = (uint64_t)((n2 << 64) / (n2 + 3 * (u128)absJ * absJ));  // < 2^64
    uint64_t r = (uint64_t)std::sqrt((double)x);                            // within +-1
    while ((u128)r * r > x) --r;
    while ((u128)(r + 1) * (r + 1) <= x) ++r;
    g = r;
  }
  return (uint64_t)((u128)g * num / den);
}

bool params_ok(int32_t C, uint32_t lam_p, uint32_t lam_q, uint32_t n_max, bool galilean) {
  if (lam_q == 0 || lam_p == 0 || lam_p > lam_q || lam_q >= (1u << 28)) return false;
  if (C < -1 || C > 4096 || n_max > 1023) return false;
  if (C > 0) {
    // bits of D1^C must fit the fixed width
    const double q = galilean ? 4294967296.0 : (double)lam_q;
    double bits = std::log2(8.0 * q * (double)n_max * (double)n_max + 1.0) + 1.0;
    if (bits * C + 64 > 64.0 * (kMaxLimbs - 1)) return false;
  }
  return true;
}

bool collision_row_full(int32_t C, uint32_t lam_p, uint32_t lam_q, bool galilean, uint32_t N,
                        uint32_t absJ, uint32_t n0, std::vector<uint64_t> &thr) {
  if (!params_ok(C, lam_p, lam_q, N, galilean) || absJ > N || n0 > N - absJ ||
      ((N - absJ - n0) & 1u))
    return false;
  Fiber f = fiber(N, absJ);
  if (N < 2 || C == 0) {
    thr.assign(f.m - 1, 0);
    for (uint32_t k = 0; k + 1 < f.m; ++k) thr[k] = k < (n0 - f.par) / 2 ? 0 : (uint64_t)1 << 32;
    return true;
  }
  if (C == -1) return row_equilibrium(f, thr);
  std::vector<Big> va, vb;
  if (galilean)
    return row_finite(f, C, galilean_lambda_q(lam_p, lam_q, N, absJ), (uint64_t)1 << 32,
                      (n0 - f.par) / 2, thr, va, vb);
  return row_finite(f, C, lam_p, lam_q, (n0 - f.par) / 2, thr, va, vb);
}

CompactLaw compact(uint32_t k_lo, const std::vector<uint64_t> &full) {
  // bins: width_j = full[j] - full[j-1], full[-1] = 0, full[m-1] = 2^32
  const size_t m = full.size() + 1;
  auto edge = [&](long j) -> uint64_t {
    if (j < 0) return 0;
    if ((size_t)j >= m - 1) return (uint64_t)1 << 32;
    return full[j];
  };
  size_t first = 0;
  while (first < m && edge((long)first) == edge((long)first - 1)) ++first;
  size_t last = m - 1;
  while (last > first && edge((long)last) == edge((long)last - 1)) --last;
  CompactLaw c;
  c.k_first = k_lo + (uint32_t)first;
  for (size_t j = first; j < last; ++j) c.thr.push_back((uint32_t)full[j]);
  return c;
}

std::shared_ptr<const CollisionTables> collision_tables(int32_t C, uint32_t lam_p,
                                                        uint32_t lam_q, uint32_t n_max,
                                                        bool galilean) {
  if (!params_ok(C, lam_p, lam_q, n_max, galilean)) return nullptr;
  auto key = std::make_tuple(C, lam_p, lam_q, n_max, galilean);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) return it->second;
  }
  // Per-N pieces built in parallel, then concatenated in N order.
  struct Piece {
    std::vector<uint32_t> rowdesc_rel;  // offsets relative to the piece
    std::vector<uint32_t> thr;
    uint32_t rows = 0, max_q = 0;
    bool ok = true;
  };
  std::vector<Piece> pieces(n_max + 1);
  std::atomic<int> next((int)n_max);
  auto work = [&]() {
    std::vector<Big> va, vb;
    std::vector<uint64_t> full;
    for (;;) {
      int N = next.fetch_sub(1);
      if (N < 0) break;
      Piece &pc = pieces[N];
      for (uint32_t absJ = 0; absJ <= (uint32_t)N && pc.ok; ++absJ) {
        Fiber f = fiber((uint32_t)N, absJ);
        uint32_t shared_off = 0, shared_q = 0, shared_first = 0;
        for (uint32_t k = 0; k < f.m; ++k) {
          bool ok = true;
          if (N < 2 || C == 0) {
            pc.rowdesc_rel.push_back((uint32_t)pc.thr.size());
            pc.rowdesc_rel.push_back(k | (1u << 16));
            pc.max_q = std::max(pc.max_q, 1u);
            continue;
          }
          if (C == -1) {
            if (k == 0) {
              ok = row_equilibrium(f, full);
              CompactLaw cl = compact(0, full);
              shared_off = (uint32_t)pc.thr.size();
              shared_first = cl.k_first;
              shared_q = (uint32_t)cl.thr.size() + 1;
              pc.thr.insert(pc.thr.end(), cl.thr.begin(), cl.thr.end());
            }
            pc.rowdesc_rel.push_back(shared_off);
            pc.rowdesc_rel.push_back(shared_first | (shared_q << 16));
            pc.max_q = std::max(pc.max_q, shared_q);
          } else {
            ok = galilean ? row_finite(f, C, galilean_lambda_q(lam_p, lam_q, (uint32_t)N, absJ),
                                       (uint64_t)1 << 32, k, full, va, vb)
                          : row_finite(f, C, lam_p, lam_q, k, full, va, vb);
            CompactLaw cl = compact(0, full);
            uint32_t qn = (uint32_t)cl.thr.size() + 1;
            pc.rowdesc_rel.push_back((uint32_t)pc.thr.size());
            pc.rowdesc_rel.push_back(cl.k_first | (qn << 16));
            pc.thr.insert(pc.thr.end(), cl.thr.begin(), cl.thr.end());
            pc.max_q = std::max(pc.max_q, qn);
          }
          if (!ok) { pc.ok = false; break; }
        }
        pc.rows += f.m;
      }
    }
  };
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned i = 0; i < nt; ++i) th.emplace_back(work);
  for (auto &t : th) t.join();

  auto tab = std::make_shared<CollisionTables>();
  tab->C = C;
  tab->lam_p = lam_p;
  tab->lam_q = lam_q;
  tab->galilean = galilean;
  tab->n_max = n_max;
  tab->rowbase.resize((size_t)(n_max + 1) * (n_max + 2) / 2);
  uint64_t rows = 0, thr_total = 0;
  for (uint32_t N = 0; N <= n_max; ++N) {
    if (!pieces[N].ok) return nullptr;
    rows += pieces[N].rows;
    thr_total += pieces[N].thr.size();
  }
  if (thr_total >= (1ull << 32) || rows >= (1ull << 32)) return nullptr;
  tab->rowdesc.reserve(2 * rows);
  tab->thr.reserve(thr_total);
  uint32_t row = 0;
  for (uint32_t N = 0; N <= n_max; ++N) {
    const Piece &pc = pieces[N];
    uint32_t thr_base = (uint32_t)tab->thr.size();
    uint32_t r = 0;
    for (uint32_t absJ = 0; absJ <= N; ++absJ) {
      tab->rowbase[(size_t)N * (N + 1) / 2 + absJ] = row + r;
      r += (N - absJ) / 2 + 1;
    }
    for (size_t i = 0; i < pc.rowdesc_rel.size(); i += 2) {
      tab->rowdesc.push_back(pc.rowdesc_rel[i] + thr_base);
      tab->rowdesc.push_back(pc.rowdesc_rel[i + 1]);
    }
    tab->thr.insert(tab->thr.end(), pc.thr.begin(), pc.thr.end());
    tab->max_q = std::max(tab->max_q, pc.max_q);
    row += pc.rows;
  }
  const size_t nrows = tab->rowdesc.size() / 2;
  if (tab->max_q <= kFixedStride && (uint64_t)nrows * kFixedStride * 4 < (1ull << 31)) {
    tab->fixed.assign(nrows * kFixedStride, 0u);
    for (size_t r = 0; r < nrows; ++r) {
      uint32_t *row = &tab->fixed[r * kFixedStride];
      const uint32_t off = tab->rowdesc[2 * r], hdr = tab->rowdesc[2 * r + 1];
      row[0] = hdr;
      for (uint32_t j = 0; j + 1 < (hdr >> 16); ++j) row[1 + j] = tab->thr[off + j];
    }
  }
  if (tab->max_q <= kRow16 - 1 && (uint64_t)nrows * kRow16 * 2 < (1ull << 31)) {
    tab->row16.assign(nrows * kRow16, (uint16_t)0xFFFF);
    for (size_t r = 0; r < nrows; ++r) {
      uint16_t *row = &tab->row16[r * kRow16];
      const uint32_t off = tab->rowdesc[2 * r], hdr = tab->rowdesc[2 * r + 1];
      row[0] = (uint16_t)(hdr & 0xFFFFu);  // k_first
      row[1] = (uint16_t)(hdr >> 16);      // q
      for (uint32_t j = 0; j + 1 < (hdr >> 16); ++j) row[2 + j] = (uint16_t)(tab->thr[off + j] >> 16);
    }
  }
  std::shared_ptr<const CollisionTables> res = tab;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache[key] = res;
  return res;
}

std::vector<uint8_t> LdsImage::blob() const {
  std::vector<uint8_t> out(dir_bytes() + records.size() * 2, 0);
  std::memcpy(out.data(), dir.data(), dir.size() * 2);
  std::memcpy(out.data() + dir_bytes(), records.data(), records.size() * 2);
  return out;
}

namespace {
// Poisson pmf in double (only steers what the image holds).
std::vector<double> pois_pmf(double mu, uint32_t kmax) {
  std::vector<double> p(kmax + 1, 0.0);
  if (!(mu > 0.0)) { p[0] = 1.0; return p; }
  for (uint32_t k = 0; k <= kmax; ++k)
    p[k] = std::exp(-mu + k * std::log(mu) - std::lgamma((double)k + 1.0));
  return p;
}

// Full-fiber threshold j of a compact row (k_first, thr[]), as uint64.
inline uint64_t full_thr(const uint32_t *thr, uint32_t k_first, uint32_t q, long j) {
  if (j < (long)k_first) return 0;
  if (j >= (long)(k_first + q - 1)) return (uint64_t)1 << 32;
  return thr[j - k_first];
}
inline uint16_t top16(uint64_t v) { return (uint16_t)std::min<uint64_t>(v >> 16, 0xFFFF); }
// ceil(v / 2^16), clamped to 0xFFFF (no draw reaches it: the upper bound is
// at most 0xFFFF and strict)
inline uint16_t top16_up(uint64_t v) {
  return (uint16_t)std::min<uint64_t>((v + 0xFFFF) >> 16, 0xFFFF);
}
}  // namespace

LdsImage build_image(const CollisionTables &tab, double rho, double u, uint32_t budget) {
  LdsImage im;
  // directory of (dim_a + 1) x (dim_c + 1) entries, then (np + 1) rows of
  // nb + 1 records (the last row and the last record of every row: never)
  auto image_bytes = [](uint32_t da, uint32_t dc, uint32_t np, uint32_t nb) {
    return (uint64_t)((da + 1) * (dc + 1) * 2 + 15) / 16 * 16 + (uint64_t)(np + 1) * (nb + 1) * 16;
  };
  uint32_t dim_a = 0, dim_c = 0, best_lo = 0, best_nb = 1, best_np = 0;
  std::vector<double> pb;
  struct Pair { uint32_t a, c; double p; };
  std::vector<Pair> pairs;
  if (tab.C != 0 && budget >= 256) {
    double f[3];
    feq(rho, std::max(-1.0, std::min(1.0, u)), f);
    const uint32_t kmax = std::min<uint32_t>(tab.n_max, 1023);
    auto pa = pois_pmf(f[0], kmax), pc = pois_pmf(f[2], kmax);
    pb = pois_pmf(f[1], kmax);
    // (a', c') pair masses
    for (uint32_t a = 0; a <= kmax; ++a)
      for (uint32_t c = a; c <= kmax; ++c) {
        double p = pa[a] * pc[c] + (a != c ? pa[c] * pc[a] : 0.0);
        if (p > 1e-12) pairs.push_back({a, c, p});
      }
    std::sort(pairs.begin(), pairs.end(), [](const Pair &x, const Pair &y) { return x.p > y.p; });
    std::vector<double> pair_cum(pairs.size() + 1, 0.0);
    for (size_t i = 0; i < pairs.size(); ++i) pair_cum[i + 1] = pair_cum[i] + pairs[i].p;
    // b ranges: grow a central interval around the mode, keep the best split
    uint32_t mode = (uint32_t)std::floor(f[1]);
    if (mode > kmax) mode = kmax;
    double best = -1.0;
    uint32_t lo = mode, hi = mode;
    double pbr = pb[mode];
    for (;;) {
      const uint32_t nb = hi - lo + 1;
      // directory size is bounded by the pairs' extent; reserve it generously
      const long room = (long)budget - 2048 - 16 * (long)(nb + 1);
      const uint32_t np =
          room > 0 ? (uint32_t)std::min<size_t>(pairs.size(), room / (16 * (nb + 1))) : 0;
      if (np == 0) break;
      const double cov = pbr * pair_cum[np];
      if (cov > best) { best = cov; best_lo = lo; best_nb = nb; best_np = np; }
      if (lo == 0 && hi == kmax) break;
      const bool left = lo > 0 && (hi == kmax || pb[lo - 1] >= pb[hi + 1]);
      if (left) { --lo; pbr += pb[lo]; } else { ++hi; pbr += pb[hi]; }
    }
    if (best_np == 0) best_nb = 1;
    auto extent = [&](uint32_t np) {
      dim_a = dim_c = 0;
      for (uint32_t i = 0; i < np; ++i) {
        dim_a = std::max(dim_a, pairs[i].a + 1);
        dim_c = std::max(dim_c, pairs[i].c + 1);
      }
    };
    extent(best_np);
    // shrink the pair count until directory + records fit the budget and
    // every directory byte offset and record index (in 16-byte units from
    // the image start) fits 16 bits
    auto fits = [&](uint32_t np) {
      const uint64_t bytes = image_bytes(dim_a, dim_c, np, best_nb);
      return bytes <= budget && (uint64_t)(dim_a + 1) * (dim_c + 1) * 2 <= 0xFFFF &&
             bytes / 16 <= 0xFFFF;
    };
    while (best_np > 0 && !fits(best_np)) extent(--best_np);
    if (best_np == 0) {
      best_nb = 1;
      best_lo = 0;
      dim_a = dim_c = 0;
    }
  }
  const uint32_t np = best_np, nb = best_nb, rs = nb + 1;
  im.dim_a = dim_a;
  im.dim_c = dim_c;
  im.b_lo = best_lo;
  im.nb = nb;
  // directory entries are record indices in 16-byte units from the image
  // start; absent pairs and the clamped row and column: the never row
  const uint32_t rec0 = im.dir_bytes() / 16;
  im.dir.assign((size_t)(dim_a + 1) * (dim_c + 1), (uint16_t)(rec0 + np * rs));
  im.records.assign((size_t)(np + 1) * rs * 8, 0);
  auto set_never = [&](size_t rec) {  // lower bound 0xFFFF, upper 0: no draw
    uint16_t *r = &im.records[rec * 8];
    std::fill(r, r + 8, (uint16_t)0);
    r[1] = 0xFFFF;
  };
  for (size_t k = 0; k < (size_t)(np + 1) * rs; ++k) set_never(k);
  double covered = 0.0;
  for (uint32_t pi = 0; pi < np; ++pi) {
    const Pair &pr = pairs[pi];
    im.dir[(size_t)pr.a * (dim_c + 1) + pr.c] = (uint16_t)(rec0 + pi * rs);
    for (uint32_t bi = 0; bi < nb; ++bi) {
      const uint32_t b = best_lo + bi;
      uint16_t *rec = &im.records[((size_t)pi * rs + bi) * 8];
      const uint32_t N = pr.a + b + pr.c, absJ = pr.c - pr.a;
      if (N < 2) {  // no collision: move 0 for every draw below 0xFFFF << 16
        rec[0] = 0;
        rec[1] = 0;
        for (int j = 2; j < 8; ++j) rec[j] = 0xFFFF;
        covered += pr.p * pb[b];
        continue;
      }
      if (N > tab.n_max) continue;  // never decided here
      const uint32_t par = (N - absJ) & 1u;
      const uint32_t m = (N - absJ) / 2 + 1;
      const uint32_t row = tab.rowbase[(size_t)N * (N + 1) / 2 + absJ] + (b - par) / 2;
      const uint32_t off = tab.rowdesc[2 * (size_t)row];
      const uint32_t kf = tab.rowdesc[2 * (size_t)row + 1] & 0xFFFF;
      const uint32_t q = tab.rowdesc[2 * (size_t)row + 1] >> 16;
      const uint32_t *thr = tab.thr.data() + off;
      // window start with the most mass
      long best_ks = 0;
      uint64_t best_w = 0;
      const long ks_hi = m > 6 ? (long)m - 6 : 0;
      for (long ks = 0; ks <= ks_hi; ++ks) {
        const uint64_t w = full_thr(thr, kf, q, ks + 5) - full_thr(thr, kf, q, ks - 1);
        if (ks == 0 || w > best_w) { best_w = w; best_ks = ks; }
      }
      // the kernel's move for the window's first state: (b >> 1) - k_s
      rec[0] = (uint16_t)(int16_t)((long)(b >> 1) - best_ks);
      rec[1] = top16_up(full_thr(thr, kf, q, best_ks - 1));
      for (int j = 1; j < 7; ++j) rec[1 + j] = top16(full_thr(thr, kf, q, best_ks - 1 + j));
      covered += pr.p * pb[b] * (double)best_w / 4294967296.0;
    }
  }
  im.coverage = covered;
  return im;
}

// Eq. (D1Q3equil), component form, evaluated in this exact order.
void feq(double rho, double u, double out[3]) {
  const double uu = u * u;
  const double three_uu = 3.0 * uu;
  const double s = std::sqrt(1.0 + three_uu);
  const double two_s = 2.0 * s;
  const double r6 = rho / 6.0;
  out[0] = r6 * ((-1.0 - 3.0 * u) + two_s);
  out[1] = ((2.0 * rho) / 3.0) * (2.0 - s);
  out[2] = r6 * ((-1.0 + 3.0 * u) + two_s);
}

// Poisson law of Eq. (poisson): weights relative to the mode m = floor(mu),
// w_m = 1, w_{k+1} = (w_k mu)/(k+1) upward and w_{k-1} = (w_k k)/mu downward
// while the new weight is >= 2^-60; S = ascending sum; thresholds
// floor(2^32 * (ascending running sum) / S) for all outcomes but the last.
bool poisson_full(double mu, uint32_t &k_lo, std::vector<uint64_t> &thr) {
  thr.clear();
  if (!(mu > 0.0)) { k_lo = 0; return true; }
  if (mu > 1.0e6) return false;
  const double cut = std::ldexp(1.0, -60);
  const uint32_t mode = (uint32_t)std::floor(mu);
  std::vector<double> up{1.0}, down;  // up[i] = w_{mode+i}, down[i] = w_{mode-1-i}
  for (uint32_t k = mode;; ++k) {
    double w = (up.back() * mu) / (double)(k + 1);
    if (w < cut) break;
    up.push_back(w);
  }
  double prev = 1.0;
  for (uint32_t k = mode; k > 0; --k) {
    double w = (prev * (double)k) / mu;
    if (w < cut) break;
    down.push_back(w);
    prev = w;
  }
  k_lo = mode - (uint32_t)down.size();
  std::vector<double> w(down.rbegin(), down.rend());
  w.insert(w.end(), up.begin(), up.end());
  double S = 0.0;
  for (double v : w) S += v;
  double run = 0.0;
  thr.resize(w.size() - 1);
  for (size_t i = 0; i + 1 < w.size(); ++i) {
    run += w[i];
    thr[i] = (uint64_t)std::floor(std::ldexp(run / S, 32));
  }
  return true;
}

}  // namespace mclg
