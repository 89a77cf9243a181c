// C ABI of the MCLG library: configuration, layout, context and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstring>
#include <map>
#include <thread>
#include <memory>
#include <new>
#include <vector>

#include "../../include/mclg.h"
#include "d2q9.h"
#include "device.h"
#include "moments.h"
#include "tables.h"

using namespace mclg;

namespace {

constexpr uint32_t kPadElems = 128;     // array stride granularity (256 B)
constexpr uint32_t kMinTileSites = 512; // chunk of the step kernel
constexpr uint32_t kPoisCap = 1024;     // thresholds per initial Poisson law
constexpr uint32_t kMaxImage = 160 * 1024; // largest LDS collision image

inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

struct Layout {
  uint64_t state_bytes = 0;
  std::vector<uint64_t> off, stride, dense;
  uint64_t total_sites = 0, max_tiles = 0;
  // workspace byte offsets
  uint64_t o_ctrl, o_slots, o_tslot, o_tiles, o_list, o_pdesc, o_pool, o_idesc, o_over, o_ipool,
      o_rowbase, o_rowdesc, o_thr, o_fixed, o_row16, ws_bytes;
  // moment kernels: segments, runs (one per slot), partial records, results
  MomPlan mplan;
  uint64_t o_mseg, o_mrun, o_mslot, o_mpart, o_mout;
};

bool compute_layout(uint32_t n, const uint64_t *L, const CollisionTables *tab, Layout &lay) {
  lay.off.resize(n);
  lay.stride.resize(n);
  lay.dense.resize(n);
  uint64_t elems = 0, dense = 0, tiles = 0;
  for (uint32_t r = 0; r < n; ++r) {
    lay.stride[r] = align_up(L[r], kPadElems);
    lay.off[r] = elems;
    lay.dense[r] = dense;
    elems += 3 * lay.stride[r];
    dense += L[r];
    tiles += (L[r] + kMinTileSites - 1) / kMinTileSites;
  }
  lay.state_bytes = elems * sizeof(uint16_t);
  lay.total_sites = dense;
  lay.max_tiles = tiles;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  lay.o_ctrl = take(256);
  lay.o_slots = take(sizeof(SlotDev) * n);
  lay.o_tslot = take(sizeof(uint32_t) * n);
  lay.o_tiles = take(sizeof(TileDev) * tiles);
  lay.o_list = take(sizeof(uint32_t) * n);
  {
    std::vector<uint32_t> ids(n);
    for (uint32_t r = 0; r < n; ++r) ids[r] = r;
    lay.mplan = plan_moments(ids.data(), L, n);
  }
  lay.o_mseg = take(sizeof(MomSeg) * lay.mplan.segs.size());
  lay.o_mrun = take(sizeof(uint32_t) * lay.mplan.run_seg.size());
  lay.o_mslot = take(sizeof(uint32_t) * lay.mplan.run_slot.size());
  lay.o_mpart = take(sizeof(uint64_t) * kMom3Rec * lay.mplan.segs.size());
  lay.o_mout = take(sizeof(uint64_t) * kMom3Out * n);
  lay.o_pdesc = take(sizeof(PoisDesc) * 3 * n);
  lay.o_pool = take(sizeof(uint32_t) * kPoisCap * 3 * n);
  lay.o_idesc = take(sizeof(ImageDesc) * n);
  lay.o_over = take(kOverflowBytes);
  lay.o_ipool = take((uint64_t)kMaxImage * n);
  lay.o_rowbase = take(sizeof(uint32_t) * tab->rowbase.size());
  lay.o_rowdesc = take(sizeof(uint32_t) * tab->rowdesc.size());
  lay.o_thr = take(sizeof(uint32_t) * (tab->thr.size() + 16));  // +16: see count_le_16
  lay.o_fixed = take(sizeof(uint32_t) * tab->fixed.size());
  lay.o_row16 = take(sizeof(uint16_t) * tab->row16.size());
  lay.ws_bytes = o;
  return true;
}

// The density and velocity a replica's LDS image is built for: its own
// (rho, |u|).  The image depends on u only through |u| (its directory is over
// min(a, c) and max(a, c)), so replicas at u and -u share one image.
std::pair<double, double> image_key(double rho, double u) { return {rho, std::fabs(u)}; }

int validate(const mclg_config *cfg) {
  if (!cfg || cfg->abi_version != MCLG_ABI_VERSION) return MCLG_E_INVAL;
  if (cfg->lattice != MCLG_D1Q3) return MCLG_E_INVAL;
  if (cfg->n_replicas == 0 || !cfg->L) return MCLG_E_INVAL;
  if (cfg->flags & ~(uint32_t)(MCLG_FLAG_NO_STREAM | MCLG_FLAG_GALILEAN)) return MCLG_E_INVAL;
  for (uint32_t r = 0; r < cfg->n_replicas; ++r) {
    if (cfg->L[r] == 0 || cfg->L[r] > kMaxSites) return MCLG_E_INVAL;
    if (cfg->replica_id && cfg->replica_id[r] >= (1ull << 32)) return MCLG_E_INVAL;
  }
  if (!params_ok(cfg->C, cfg->lambda_num, cfg->lambda_den, cfg->n_max,
                 (cfg->flags & MCLG_FLAG_GALILEAN) != 0))
    return MCLG_E_INVAL;
  return MCLG_OK;
}

}  // namespace

struct mclg_ctx {
  std::unique_ptr<D2Ctx> d2;  // set for a D2Q9 context; then nothing below is used
  uint32_t n = 0, flags = 0;
  uint64_t seed = 0;
  int32_t C = 0;
  uint32_t lam_p = 1, lam_q = 1, n_max = 0;
  std::vector<uint64_t> L, rid;
  hipStream_t stream = nullptr;
  uint16_t *state = nullptr;
  uint8_t *ws = nullptr;
  Layout lay;
  std::shared_ptr<const CollisionTables> tab;
  std::vector<int64_t> t;
  // steps of every slot launched (with t_off) but not yet added to tslot on
  // the device; flushed by flush_t() before anything else reads tslot
  uint32_t t_pending = 0;
  Schedule sch;
  std::vector<TileDev> tiles;
  std::vector<uint32_t> tile_begin, tile_end;
  int last_hip = 0;
  std::map<uint64_t, hipGraphExec_t> graphs;
  std::vector<hipGraph_t> graph_defs;
  // LDS collision images (a cache in front of the exact global rows)
  std::vector<double> est_rho, est_u;   // density and velocity each image targets
  std::vector<ImageDesc> img_desc;
  std::vector<SlotDev> slot_host;  // the device's slot descriptors
  std::vector<uint8_t> img_pool;
  uint32_t lds_bytes = 0, max_blocks = 1, lds_limit = 64 * 1024, n_cu = 1;
  uint32_t grid_limit = 0;  // 0: occupancy-derived grid
  // several steps per launch (mclg_set_blocked): geometry, grid, caller's
  // scratch; tb.steps <= 1 means one step per launch
  TbLaunch tb;
  uint32_t tb_grid = 0;
  uint32_t tb_arrivals = 0;  // blocks of every blocked launch so far (the barrier's count)
  uint32_t drain_policy = MCLG_DRAIN_AUTO;
  // the device address of this device's static scratch area (moments.hip),
  // looked up in mclg_init with the context's device current
  unsigned long long *scratch = nullptr;
  double coverage = 0.0;                // expected LDS hit fraction (site-weighted)
  bool use_row16 = false;               // resolve misses from the 64-byte rows

  uint32_t *err() { return reinterpret_cast<uint32_t *>(ws + lay.o_ctrl); }
  uint32_t *ticket() { return reinterpret_cast<uint32_t *>(ws + lay.o_ctrl) + 1; }
  uint32_t *barrier() { return reinterpret_cast<uint32_t *>(ws + lay.o_ctrl) + 2; }
  // One launch of tb.steps steps (temporal blocking) at step t + t_pending.
  hipError_t launch_blocked(TbLaunch b) {
    b.bar = barrier();
    b.bar_target = tb_arrivals + tb_grid;
    hipError_t e = launch_step_blocked(sch, stream,
                                       launch_args(0, (uint32_t)tiles.size(), 0, n, t_pending), b,
                                       tb_grid);
    // (the replicas' kernel has no barrier)
    if (!e && !b.reps) tb_arrivals += b.n_logs ? 2u * tb_grid : tb_grid;
    return e;
  }
  SlotDev *slots() { return reinterpret_cast<SlotDev *>(ws + lay.o_slots); }
  uint32_t *tslot() { return reinterpret_cast<uint32_t *>(ws + lay.o_tslot); }
  hipError_t flush_t() {
    if (!t_pending) return hipSuccess;
    hipError_t e = launch_add_t(stream, tslot(), 0, n, t_pending);
    if (!e) t_pending = 0;
    return e;
  }
  TileDev *tiles_dev() { return reinterpret_cast<TileDev *>(ws + lay.o_tiles); }
  // The moment kernels' arguments; partial records and results go to
  // `partial` and `out` (device).
  MomArgs mom_args(unsigned long long *partial, long long *out) {
    MomArgs m;
    m.state = state;
    m.slots = slots();
    m.tslot = tslot();
    m.no_stream = (flags & MCLG_FLAG_NO_STREAM) ? 1u : 0u;
    m.segs = reinterpret_cast<const MomSeg *>(ws + lay.o_mseg);
    m.n_segs = (uint32_t)lay.mplan.segs.size();
    m.run_seg = reinterpret_cast<const uint32_t *>(ws + lay.o_mrun);
    m.run_slot = reinterpret_cast<const uint32_t *>(ws + lay.o_mslot);
    m.n_runs = n;
    m.partial = partial;
    m.out = out;
    return m;
  }
  TableDev table() {
    TableDev d;
    d.rowbase = reinterpret_cast<const uint32_t *>(ws + lay.o_rowbase);
    d.rowdesc = reinterpret_cast<const uint2 *>(ws + lay.o_rowdesc);
    d.thr = reinterpret_cast<const uint32_t *>(ws + lay.o_thr);
    d.fixed = tab->fixed.empty() ? nullptr : reinterpret_cast<const uint4 *>(ws + lay.o_fixed);
    d.row16 = tab->row16.empty() ? nullptr : reinterpret_cast<const uint4 *>(ws + lay.o_row16);
    return d;
  }
  StepParams params() const {
    StepParams p;
    p.seed = seed;
    p.C = C;
    p.lam_p = lam_p;
    p.lam_q = lam_q;
    p.n_max = n_max;
    p.no_stream = (flags & MCLG_FLAG_NO_STREAM) ? 1u : 0u;
    p.galilean = (flags & MCLG_FLAG_GALILEAN) ? 1u : 0u;
    p.tile_sites = sch.tile_sites();
    return p;
  }
  int hip(hipError_t e) {
    if (e == hipSuccess) return MCLG_OK;
    last_hip = (int)e;
    return MCLG_E_HIP;
  }
  // (Replicas stay in their given order in the tile list: grouping replicas
  // of equal images, so that blocks keep an image across segments, measured
  // slower on the 1024-replica batch -- 477 against 465 us per step -- since
  // the blocks that get the densest replicas then finish last.)
  void build_tiles() {
    tiles.clear();
    tile_begin.assign(n, 0);
    tile_end.assign(n, 0);
    const uint32_t ts = sch.tile_sites();
    for (uint32_t r = 0; r < n; ++r) {
      tile_begin[r] = (uint32_t)tiles.size();
      const uint32_t next = tile_begin[r] + (uint32_t)((L[r] + ts - 1) / ts);
      for (uint64_t x0 = 0; x0 < L[r]; x0 += ts) tiles.push_back(TileDev{r, (uint32_t)x0, next, 0});
      tile_end[r] = (uint32_t)tiles.size();
    }
  }
  ImageDesc *img_desc_dev() { return reinterpret_cast<ImageDesc *>(ws + lay.o_idesc); }
  StepLaunch launch_args(uint32_t tile_lo, uint32_t tile_hi, uint32_t slot_first,
                         uint32_t n_slots, uint32_t t_off) {
    StepLaunch a{};
    a.state = state;
    a.slots = slots();
    a.tslot = tslot();
    a.tiles = tiles_dev() + tile_lo;
    a.n_tiles = tile_hi - tile_lo;
    a.slot_list = nullptr;
    a.slot_first = slot_first;
    a.n_slots = n_slots;
    a.ticket = nullptr;  // the host advances tslot (launch_add_t)
    a.t_off = t_off;
    // one slot whose tiles are exactly the launch's: descriptors by value
    a.single = (n_slots == 1 && tile_lo == tile_begin[slot_first] &&
                tile_hi == tile_end[slot_first]) ? 1u : 0u;
    if (a.single) {
      a.im1 = img_desc[slot_first];
      a.sl1 = slot_host[slot_first];
    }
    a.err = err();
    a.tab = table();
    if (!use_row16) a.tab.row16 = nullptr;
    a.p = params();
    uint64_t bytes = 0;  // state the launch streams: 6 bytes per site
    for (uint32_t s = slot_first; s < slot_first + n_slots; ++s) bytes += 6ull * L[s];
    a.p.drain = drain_policy == MCLG_DRAIN_AUTO ? auto_drain(bytes) : drain_policy - 1u;
    a.images = img_desc_dev();
    a.image_pool = ws + lay.o_ipool;
    a.overflow = reinterpret_cast<uint4 *>(ws + lay.o_over);
    a.lds_bytes = lds_bytes;
    a.max_blocks = grid_limit ? std::min(max_blocks, grid_limit) : max_blocks;
    return a;
  }
  // (Re)build the images for the current budget, upload them, and size the
  // persistent grid from the runtime's occupancy for that LDS footprint.
  hipError_t prepare_images() {
    const uint32_t queues = (sch.threads / 64u) * kWaveLdsBytes;
    const uint32_t room = lds_limit > queues ? lds_limit - queues : 0u;
    const uint32_t budget = std::min(sch.lds_budget, std::min(kMaxImage, room)) / 16u * 16u;
    std::map<std::pair<double, double>, uint32_t> uniq;
    std::vector<uint32_t> which(n);
    std::vector<std::pair<double, double>> keys;
    for (uint32_t r = 0; r < n; ++r) {
      auto k = image_key(est_rho[r], est_u[r]);
      auto it = uniq.find(k);
      if (it == uniq.end()) { it = uniq.emplace(k, (uint32_t)keys.size()).first; keys.push_back(k); }
      which[r] = it->second;
    }
    std::vector<LdsImage> ims(keys.size());
    std::atomic<size_t> next(0);
    auto work = [&]() {
      for (size_t i; (i = next.fetch_add(1)) < keys.size();)
        ims[i] = build_image(*tab, keys[i].first, keys[i].second, budget);
    };
    std::vector<std::thread> th;
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    for (unsigned i = 0; i < nt; ++i) th.emplace_back(work);
    for (auto &x : th) x.join();
    img_pool.clear();
    img_desc.assign(n, ImageDesc{});
    std::vector<uint64_t> at(ims.size());
    lds_bytes = 16;
    for (size_t i = 0; i < ims.size(); ++i) {
      at[i] = img_pool.size();
      auto b = ims[i].blob();
      img_pool.insert(img_pool.end(), b.begin(), b.end());
      img_pool.resize((img_pool.size() + 15) / 16 * 16, 0);
      lds_bytes = std::max<uint32_t>(lds_bytes, (uint32_t)(b.size() + 15) / 16 * 16);
    }
    double cov = 0.0, sites = 0.0;
    for (uint32_t r = 0; r < n; ++r) {
      const LdsImage &im = ims[which[r]];
      ImageDesc &d = img_desc[r];
      d.off = at[which[r]];
      d.bytes = (uint32_t)im.blob().size();
      d.dir_bytes = im.dir_bytes();
      d.dim_a = im.dim_a;
      d.dim_c = im.dim_c;
      d.b_lo = im.b_lo;
      d.nb = im.nb;
      cov += im.coverage * (double)L[r];
      sites += (double)L[r];
    }
    coverage = sites > 0 ? cov / sites : 0.0;
    use_row16 = use_compact_rows(1.0 - coverage, (uint32_t)ims.size());
    if (img_pool.size() > (uint64_t)kMaxImage * n) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    if (!img_pool.empty())
      e = hipMemcpyAsync(ws + lay.o_ipool, img_pool.data(), img_pool.size(), hipMemcpyHostToDevice, stream);
    if (!e) e = hipMemcpyAsync(img_desc_dev(), img_desc.data(), sizeof(ImageDesc) * n,
                               hipMemcpyHostToDevice, stream);
    if (!e) e = hipStreamSynchronize(stream);
    if (!e) e = step_occupancy(sch, lds_bytes, n_cu, max_blocks);
    return e;
  }
  void drop_graphs() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
    for (auto &g : graph_defs) (void)hipGraphDestroy(g);
    graphs.clear();
    graph_defs.clear();
  }
};

extern "C" {

int mclg_sizes(const mclg_config *cfg, uint64_t *state_bytes, uint64_t *workspace_bytes) {
  if (cfg && cfg->abi_version == MCLG_ABI_VERSION && cfg->lattice == MCLG_D2Q9) {
    if (cfg->n_replicas == 0 || !cfg->L) return MCLG_E_INVAL;
    D2Ctx d;
    int rc = d2q9_layout(cfg, d);
    if (rc) return rc;
    if (state_bytes) *state_bytes = d.state_bytes;
    if (workspace_bytes) *workspace_bytes = d.ws_bytes;
    return MCLG_OK;
  }
  int rc = validate(cfg);
  if (rc) return rc;
  auto tab = collision_tables(cfg->C, cfg->lambda_num, cfg->lambda_den, cfg->n_max,
                              (cfg->flags & MCLG_FLAG_GALILEAN) != 0);
  if (!tab) return MCLG_E_INVAL;
  Layout lay;
  compute_layout(cfg->n_replicas, cfg->L, tab.get(), lay);
  if (state_bytes) *state_bytes = lay.state_bytes;
  if (workspace_bytes) *workspace_bytes = lay.ws_bytes;
  return MCLG_OK;
}

int mclg_init(const mclg_config *cfg, const mclg_init_spec *init, mclg_ctx **out) {
  if (!out || !init) return MCLG_E_INVAL;
  if (cfg && cfg->abi_version == MCLG_ABI_VERSION && cfg->lattice == MCLG_D2Q9) {
    if (cfg->n_replicas == 0 || !cfg->L || !cfg->state || !cfg->workspace) return MCLG_E_INVAL;
    std::unique_ptr<mclg_ctx> c(new (std::nothrow) mclg_ctx());
    if (!c) return MCLG_E_NOMEM;
    c->d2.reset(new (std::nothrow) D2Ctx());
    if (!c->d2) return MCLG_E_NOMEM;
    int rc = d2q9_layout(cfg, *c->d2);
    if (!rc) rc = d2q9_init(*c->d2, cfg, init);
    if (rc) return rc;
    *out = c.release();
    return MCLG_OK;
  }
  int rc = validate(cfg);
  if (rc) return rc;
  if (!cfg->state || !cfg->workspace) return MCLG_E_INVAL;
  auto tab = collision_tables(cfg->C, cfg->lambda_num, cfg->lambda_den, cfg->n_max,
                              (cfg->flags & MCLG_FLAG_GALILEAN) != 0);
  if (!tab) return MCLG_E_INVAL;
  std::unique_ptr<mclg_ctx> c(new (std::nothrow) mclg_ctx());
  if (!c) return MCLG_E_NOMEM;
  c->n = cfg->n_replicas;
  c->flags = cfg->flags;
  c->seed = cfg->seed;
  c->C = cfg->C;
  c->lam_p = cfg->lambda_num;
  c->lam_q = cfg->lambda_den;
  c->n_max = cfg->n_max;
  c->L.assign(cfg->L, cfg->L + c->n);
  c->rid.resize(c->n);
  for (uint32_t r = 0; r < c->n; ++r) c->rid[r] = cfg->replica_id ? cfg->replica_id[r] : r;
  c->stream = reinterpret_cast<hipStream_t>(cfg->stream);
  c->state = reinterpret_cast<uint16_t *>(cfg->state);
  c->ws = reinterpret_cast<uint8_t *>(cfg->workspace);
  c->tab = tab;
  compute_layout(c->n, cfg->L, tab.get(), c->lay);
  if (cfg->state_bytes < c->lay.state_bytes || cfg->workspace_bytes < c->lay.ws_bytes)
    return MCLG_E_INVAL;
  c->t.assign(c->n, 0);
  c->build_tiles();

  const Layout &lay = c->lay;
  hipStream_t s = c->stream;
  std::vector<SlotDev> slots(c->n);
  std::vector<uint32_t> list(c->n);
  for (uint32_t r = 0; r < c->n; ++r) {
    slots[r].off = lay.off[r];
    slots[r].dense = lay.dense[r];
    slots[r].L = (uint32_t)c->L[r];
    slots[r].stride = (uint32_t)lay.stride[r];
    slots[r].rid = (uint32_t)c->rid[r];
    slots[r].pad = 0;
    list[r] = r;
  }
  std::vector<uint32_t> ctrl(64, 0), tz(c->n, 0);
  // Poisson laws (host) for the initial state
  std::vector<PoisDesc> pdesc(3 * c->n);
  std::vector<uint32_t> pool;
  if (init->kind == MCLG_INIT_POISSON) {
    if (!init->rho || !init->u0) return MCLG_E_INVAL;
    pool.assign((size_t)kPoisCap * 3 * c->n, 0);
    for (uint32_t r = 0; r < c->n; ++r) {
      if (!(init->rho[r] >= 0.0) || !(init->u0[r] >= -1.0 && init->u0[r] <= 1.0))
        return MCLG_E_INVAL;
      double mu[3];
      feq(init->rho[r], init->u0[r], mu);
      for (int i = 0; i < 3; ++i) {
        uint32_t k_lo = 0;
        std::vector<uint64_t> full;
        if (!poisson_full(mu[i], k_lo, full)) return MCLG_E_INVAL;
        CompactLaw cl = compact(k_lo, full);
        if (cl.thr.size() > kPoisCap) return MCLG_E_INVAL;
        PoisDesc &d = pdesc[3 * r + i];
        d.off = (uint32_t)((3 * r + i) * kPoisCap);
        d.k_first = cl.k_first;
        d.nthr = (uint32_t)cl.thr.size();
        d.pad = 0;
        std::copy(cl.thr.begin(), cl.thr.end(), pool.begin() + d.off);
      }
    }
  } else if (init->kind != MCLG_INIT_COUNTS || !init->counts) {
    return MCLG_E_INVAL;
  }
  auto up = [&](uint64_t off, const void *src, size_t bytes) {
    return bytes ? hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  hipError_t e = hipSuccess;
  if (!e) e = up(lay.o_ctrl, ctrl.data(), 256);
  c->slot_host = slots;
  if (!e) e = up(lay.o_slots, slots.data(), sizeof(SlotDev) * c->n);
  if (!e) e = up(lay.o_tslot, tz.data(), sizeof(uint32_t) * c->n);
  if (!e) e = up(lay.o_tiles, c->tiles.data(), sizeof(TileDev) * c->tiles.size());
  if (!e) e = up(lay.o_list, list.data(), sizeof(uint32_t) * c->n);
  if (!e) e = up(lay.o_mseg, lay.mplan.segs.data(), sizeof(MomSeg) * lay.mplan.segs.size());
  if (!e) e = up(lay.o_mrun, lay.mplan.run_seg.data(), sizeof(uint32_t) * lay.mplan.run_seg.size());
  if (!e) e = up(lay.o_mslot, lay.mplan.run_slot.data(), sizeof(uint32_t) * lay.mplan.run_slot.size());
  if (!e) e = up(lay.o_rowbase, tab->rowbase.data(), sizeof(uint32_t) * tab->rowbase.size());
  if (!e) e = up(lay.o_rowdesc, tab->rowdesc.data(), sizeof(uint32_t) * tab->rowdesc.size());
  if (!e) e = up(lay.o_thr, tab->thr.data(), sizeof(uint32_t) * tab->thr.size());
  if (!e && !tab->fixed.empty()) e = up(lay.o_fixed, tab->fixed.data(), sizeof(uint32_t) * tab->fixed.size());
  if (!e && !tab->row16.empty()) e = up(lay.o_row16, tab->row16.data(), sizeof(uint16_t) * tab->row16.size());
  const uint32_t ts = c->sch.tile_sites();
  if (init->kind == MCLG_INIT_POISSON) {
    if (!e) e = up(lay.o_pdesc, pdesc.data(), sizeof(PoisDesc) * pdesc.size());
    if (!e) e = up(lay.o_pool, pool.data(), sizeof(uint32_t) * pool.size());
    if (!e)
      e = launch_init_poisson(s, c->state, c->slots(), c->tslot(), c->tiles_dev(),
                              (uint32_t)c->tiles.size(), ts,
                              reinterpret_cast<const PoisDesc *>(c->ws + lay.o_pdesc),
                              reinterpret_cast<const uint32_t *>(c->ws + lay.o_pool), c->seed,
                              c->err());
  } else {
    if (!e)
      e = launch_init_counts(s, c->state, c->slots(), c->tiles_dev(), (uint32_t)c->tiles.size(),
                             ts, init->counts);
  }
  if (!e) e = hipStreamSynchronize(s);
  if (e) return c->hip(e);
  // device limits for the LDS images
  int dev = 0, v = 0;
  e = hipGetDevice(&dev);
  if (!e) e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (!e) c->lds_limit = (uint32_t)std::max(0, v - 64);  // the block's two counters
  if (!e) e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
  if (!e) c->n_cu = (uint32_t)std::max(1, v);
  if (e) return c->hip(e);
  if (c->n_cu > 256) return MCLG_E_UNSUPPORTED;  // overflow region sized for 256 CUs
  e = moments_scratch(&c->scratch);
  if (e) return c->hip(e);
  // what density and velocity each replica's image should target
  c->est_rho.assign(c->n, 0.0);
  c->est_u.assign(c->n, 0.0);
  if (init->kind == MCLG_INIT_POISSON) {
    for (uint32_t r = 0; r < c->n; ++r) { c->est_rho[r] = init->rho[r]; c->est_u[r] = init->u0[r]; }
  } else {
    std::vector<mclg_moments_t> m(c->n);
    int rc2 = mclg_moments(c.get(), nullptr, 0, 0, m.data());
    if (rc2 && rc2 != MCLG_E_RANGE) return rc2;
    for (uint32_t r = 0; r < c->n; ++r) {
      c->est_rho[r] = (double)m[r].sum_N / (double)c->L[r];
      c->est_u[r] = m[r].sum_N ? (double)m[r].sum_J / (double)m[r].sum_N : 0.0;
    }
  }
  e = c->prepare_images();
  if (e) return c->hip(e);
  uint32_t err = 0;
  e = hipMemcpy(&err, c->err(), sizeof(err), hipMemcpyDeviceToHost);
  if (e) return c->hip(e);
  *out = c.release();
  return (err & 4u) ? MCLG_E_INTERNAL : err ? MCLG_E_RANGE : MCLG_OK;
}

// One step of the slots [slot_first, slot_first + n_slots) (their tiles are
// tile_lo .. tile_hi), whose step is tslot + t_off on the device.
static int step_range(mclg_ctx *c, uint32_t tile_lo, uint32_t tile_hi, uint32_t slot_first,
                      uint32_t n_slots, uint32_t t_off) {
  hipError_t e = launch_step(c->sch, c->stream,
                             c->launch_args(tile_lo, tile_hi, slot_first, n_slots, t_off));
  return c->hip(e);
}

// The geometry of `steps` steps per launch for the context's one lattice:
// every block of the grid resident at once, R owned sites per block (a
// multiple of 8), kh = steps rounded up to 8 extra sites on each side.
// Whole regions: each block's copy holds its R + 2 kh sites; tiles: copies
// of `tile` sites, T = tile - 2 kh of them the tile's own (tile = 0 picks
// whole regions while all copies fit kTbCachedCopies bytes, else tiles of
// kTbTileSites).  The scratch holds the blocks' areas, then the partial
// records of up to `steps` logs per launch (records_at bytes in).
constexpr uint64_t kTbCachedCopies = 128ull << 20;
constexpr uint32_t kTbTileSites = 65536;  // 128 chunks of 512: 100 MB of copies in all
static int blocked_geometry(mclg_ctx *c, uint32_t steps, uint32_t tile, TbLaunch &tb,
                            uint32_t &grid, uint64_t &bytes, uint64_t &records_at) {
  if (c->d2) return MCLG_E_UNSUPPORTED;
  if (steps < 2 || steps > kTbMaxSteps) return MCLG_E_INVAL;
  if (c->sch.threads != 1024) return MCLG_E_UNSUPPORTED;
  uint32_t g = 0;
  hipError_t e = step_blocked_occupancy(c->sch, c->lds_bytes, c->n_cu, g);
  if (e) return c->hip(e);
  g = std::min(g, kOverflowWaves / (c->sch.threads / 64u));  // waves with an overflow area
  if (c->n > 1) {
    // replicas: each block copies whole replicas, so its copy area holds
    // the largest; then the blocks' replica lists (records_at: where)
    if (tile > 1) return MCLG_E_INVAL;
    const uint64_t maxL = *std::max_element(c->L.begin(), c->L.end());
    TbLaunch t;
    t.steps = steps;
    t.reps = 1;
    t.stride = (uint32_t)align_up(maxL + 8u, 64);
    t.bstride = 3ull * t.stride;
    if (6ull * t.stride >= (1ull << 31)) return MCLG_E_UNSUPPORTED;
    tb = t;
    grid = g;
    records_at = align_up((uint64_t)g * t.bstride * sizeof(uint16_t), 256);
    bytes = records_at + sizeof(uint32_t) * ((uint64_t)c->n + g + 1u);
    return MCLG_OK;
  }
  if (c->L[0] % 8 != 0) return MCLG_E_UNSUPPORTED;
  const uint64_t L = c->L[0];
  TbLaunch t;
  t.R = (uint32_t)(((L + g - 1) / g + 7) / 8 * 8);
  t.kh = (steps + 7u) / 8u * 8u;
  t.steps = steps;
  if (tile == 0)
    tile = (uint64_t)g * (t.R + 2u * t.kh) * 6u > kTbCachedCopies ? kTbTileSites : 1u;
  if (tile == 1) {
    t.es = t.R + 2u * t.kh;
    t.stride = (t.es + 63u) / 64u * 64u;
    t.bstride = 3ull * t.stride;
  } else {
    if (tile % 8u != 0 || tile <= 2u * t.kh || tile > (1u << 20)) return MCLG_E_INVAL;
    t.T = tile - 2u * t.kh;
    t.es = tile;
    t.stride = (t.es + 63u) / 64u * 64u;
    t.bstride = align_up(3ull * t.stride + 18ull * t.kh, 128);
    if (2ull * t.bstride * g >= (1ull << 31)) return MCLG_E_UNSUPPORTED;
  }
  // the copy's random-number keys wrap around the lattice at most once
  if ((uint64_t)t.es + 512u > L) return MCLG_E_UNSUPPORTED;
  tb = t;
  grid = g;
  records_at = align_up((uint64_t)g * t.bstride * sizeof(uint16_t), 256);
  bytes = records_at + (uint64_t)steps * g * kMom3Rec * sizeof(uint64_t);
  return MCLG_OK;
}

int mclg_blocked_bytes(mclg_ctx *c, uint32_t steps, uint32_t tile, uint64_t *scratch_bytes) {
  if (!c || !scratch_bytes) return MCLG_E_INVAL;
  TbLaunch tb;
  uint32_t grid = 0;
  uint64_t records_at = 0;
  return blocked_geometry(c, steps, tile, tb, grid, *scratch_bytes, records_at);
}

int mclg_set_blocked(mclg_ctx *c, uint32_t steps, uint32_t tile, void *scratch,
                     uint64_t scratch_bytes) {
  if (!c) return MCLG_E_INVAL;
  if (c->d2) return MCLG_E_UNSUPPORTED;
  if (steps <= 1) {
    c->tb = TbLaunch{};
    c->tb_grid = 0;
    return MCLG_OK;
  }
  TbLaunch tb;
  uint32_t grid = 0;
  uint64_t need = 0, records_at = 0;
  int rc = blocked_geometry(c, steps, tile, tb, grid, need, records_at);
  if (rc) return rc;
  if (!scratch || scratch_bytes < need) return MCLG_E_INVAL;
  tb.scratch = static_cast<uint16_t *>(scratch);
  if (tb.reps) {
    // each block's replicas: the longest-work-first greedy assignment, with a
    // replica's work per step taken as its chunks of 512 sites plus 10 (a
    // step's fixed cost, about ten chunks')
    std::vector<uint32_t> order(c->n);
    for (uint32_t r = 0; r < c->n; ++r) order[r] = r;
    auto work = [&](uint32_t r) { return (c->L[r] + 511u) / 512u + 10u; };
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return work(x) > work(y); });
    std::vector<std::vector<uint32_t>> lists(grid);
    std::vector<std::pair<uint64_t, uint32_t>> heap;  // (work, block), min-heap
    for (uint32_t b = 0; b < grid; ++b) heap.push_back({0, b});
    auto cmp = [](const std::pair<uint64_t, uint32_t> &x, const std::pair<uint64_t, uint32_t> &y) {
      return x > y;
    };
    std::make_heap(heap.begin(), heap.end(), cmp);
    for (uint32_t r : order) {
      std::pop_heap(heap.begin(), heap.end(), cmp);
      heap.back().first += work(r);
      lists[heap.back().second].push_back(r);
      std::push_heap(heap.begin(), heap.end(), cmp);
    }
    std::vector<uint32_t> first(grid + 1u, 0), items;
    for (uint32_t b = 0; b < grid; ++b) {
      first[b] = (uint32_t)items.size();
      items.insert(items.end(), lists[b].begin(), lists[b].end());
    }
    first[grid] = (uint32_t)items.size();
    uint32_t *lst = reinterpret_cast<uint32_t *>(static_cast<uint8_t *>(scratch) + records_at);
    hipError_t e = hipMemcpyAsync(lst, items.data(), sizeof(uint32_t) * items.size(),
                                  hipMemcpyHostToDevice, c->stream);
    if (!e) e = hipMemcpyAsync(lst + items.size(), first.data(), sizeof(uint32_t) * first.size(),
                               hipMemcpyHostToDevice, c->stream);
    if (!e) e = hipStreamSynchronize(c->stream);
    if (e) return c->hip(e);
    tb.items = lst;
    tb.item_first = lst + items.size();
  } else {
    tb.records =
        reinterpret_cast<unsigned long long *>(static_cast<uint8_t *>(scratch) + records_at);
  }
  c->tb = tb;
  c->tb_grid = grid;
  return MCLG_OK;
}

int mclg_step(mclg_ctx *c, uint64_t n_steps) {
  if (!c) return MCLG_E_INVAL;
  if (c->d2) return d2q9_step(*c->d2, n_steps);
  // whole blocks of tb.steps steps first
  const uint32_t K = c->tb.steps;
  if (K > 1) {
    for (; n_steps >= K; n_steps -= K) {
      if (c->t_pending >= (1u << 30)) {
        hipError_t e = c->flush_t();
        if (e) return c->hip(e);
      }
      hipError_t e = c->launch_blocked(c->tb);
      if (e) return c->hip(e);
      for (auto &t : c->t) t += K;  // (the launch advances the device counters itself)
    }
  }
  for (uint64_t i = 0; i < n_steps; ++i) {
    if (c->t_pending >= (1u << 30)) {
      hipError_t e = c->flush_t();
      if (e) return c->hip(e);
    }
    int rc = step_range(c, 0, (uint32_t)c->tiles.size(), 0, c->n, c->t_pending);
    if (rc) return rc;
    ++c->t_pending;
    for (auto &t : c->t) ++t;
  }
  return MCLG_OK;
}

int mclg_step_replica(mclg_ctx *c, uint32_t r, uint64_t n_steps) {
  if (c && c->d2) return MCLG_E_UNSUPPORTED;
  if (!c || r >= c->n) return MCLG_E_INVAL;
  hipError_t e = c->flush_t();
  if (e) return c->hip(e);
  for (uint64_t done = 0; done < n_steps;) {
    const uint32_t m = (uint32_t)std::min<uint64_t>(n_steps - done, 1u << 30);
    for (uint32_t i = 0; i < m; ++i) {
      int rc = step_range(c, c->tile_begin[r], c->tile_end[r], r, 1, i);
      if (rc) return rc;
      ++c->t[r];
    }
    e = launch_add_t(c->stream, c->tslot(), r, 1, m);
    if (e) return c->hip(e);
    done += m;
  }
  return MCLG_OK;
}

int mclg_step_graph(mclg_ctx *c, uint64_t n_steps) {
  if (c && c->d2) return MCLG_E_UNSUPPORTED;
  if (!c || !c->stream || n_steps == 0) return MCLG_E_INVAL;
  if (n_steps >= (1u << 30)) return MCLG_E_INVAL;
  hipError_t fe = c->flush_t();  // the graph's steps count from tslot itself
  if (fe) return c->hip(fe);
  auto it = c->graphs.find(n_steps);
  if (it == c->graphs.end()) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e) return c->hip(e);
    int rc = MCLG_OK;
    for (uint64_t i = 0; i < n_steps && !rc; ++i)
      rc = step_range(c, 0, (uint32_t)c->tiles.size(), 0, c->n, (uint32_t)i);
    if (!rc) rc = c->hip(launch_add_t(c->stream, c->tslot(), 0, c->n, (uint32_t)n_steps));
    e = hipStreamEndCapture(c->stream, &g);
    if (rc) return rc;
    if (e) return c->hip(e);
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e) { (void)hipGraphDestroy(g); return c->hip(e); }
    c->graph_defs.push_back(g);
    it = c->graphs.emplace(n_steps, ge).first;
  }
  hipError_t e = hipGraphLaunch(it->second, c->stream);
  if (e) return c->hip(e);
  for (auto &t : c->t) t += (int64_t)n_steps;
  return MCLG_OK;
}

static int read_err(mclg_ctx *c) {
  uint32_t err = 0;
  hipError_t e = hipMemcpyAsync(&err, c->err(), sizeof(err), hipMemcpyDeviceToHost, c->stream);
  if (!e) e = hipStreamSynchronize(c->stream);
  if (e) return c->hip(e);
  return (err & 4u) ? MCLG_E_INTERNAL : err ? MCLG_E_RANGE : MCLG_OK;
}

int mclg_check(mclg_ctx *c) {
  if (!c) return MCLG_E_INVAL;
  if (c->d2) return d2q9_check(*c->d2);
  return read_err(c);
}

int mclg_moments9(mclg_ctx *c, mclg_moments9_t *out) {
  if (!c || !out) return MCLG_E_INVAL;
  if (!c->d2) return MCLG_E_UNSUPPORTED;
  return d2q9_moments(*c->d2, out);
}

int mclg_moments(mclg_ctx *c, const int32_t *twiddle, uint32_t n_modes, uint32_t flags,
                 mclg_moments_t *out) {
  if (c && c->d2) return MCLG_E_UNSUPPORTED;
  if (!c || !out || n_modes > MCLG_MAX_MODES || (n_modes && !twiddle) ||
      (flags & ~(uint32_t)MCLG_MOMENTS_DIGEST))
    return MCLG_E_INVAL;
  static_assert(sizeof(mclg_moments_t) == kMom3Out * sizeof(int64_t), "result layout");
  hipStream_t s = c->stream;
  MomArgs m = c->mom_args(reinterpret_cast<unsigned long long *>(c->ws + c->lay.o_mpart),
                          reinterpret_cast<long long *>(c->ws + c->lay.o_mout));
  m.twiddle = twiddle;
  m.n_modes = n_modes;
  m.digest = (flags & MCLG_MOMENTS_DIGEST) ? 1u : 0u;
  hipError_t e = c->flush_t();
  if (!e) e = launch_moments3(s, m);
  if (!e) e = hipMemcpyAsync(out, c->ws + c->lay.o_mout, sizeof(mclg_moments_t) * c->n,
                             hipMemcpyDeviceToHost, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return c->hip(e);
  for (uint32_t r = 0; r < c->n; ++r) out[r].t = c->t[r];  // exact beyond 2^32 steps
  return read_err(c);
}

int mclg_moments_noalloc(mclg_ctx *c, const int32_t *twiddle, uint32_t n_modes, uint32_t flags,
                         mclg_moments_t *dev_out) {
  if (c && c->d2) return MCLG_E_UNSUPPORTED;
  if (!c || !dev_out || n_modes > MCLG_MAX_MODES || (n_modes && !twiddle) ||
      (flags & ~(uint32_t)MCLG_MOMENTS_DIGEST))
    return MCLG_E_INVAL;
  if ((uint64_t)c->lay.mplan.segs.size() * kMom3Rec * 8 > kMomScratchBytes) return MCLG_E_TOO_LARGE;
  if (!c->scratch) return MCLG_E_INTERNAL;
  MomArgs m = c->mom_args(c->scratch, reinterpret_cast<long long *>(dev_out));
  m.twiddle = twiddle;
  m.n_modes = n_modes;
  m.digest = (flags & MCLG_MOMENTS_DIGEST) ? 1u : 0u;
  hipError_t e = c->flush_t();
  if (!e) e = launch_moments3(c->stream, m);
  return c->hip(e);
}

int mclg_step_log(mclg_ctx *c, uint64_t every, uint64_t n_logs, const int32_t *twiddle,
                  uint32_t n_modes, uint32_t flags, mclg_moments_t *dev_out) {
  if (c && c->d2) return MCLG_E_UNSUPPORTED;
  if (!c || !dev_out || every == 0 || n_modes > MCLG_MAX_MODES || (n_modes && !twiddle) ||
      (flags & ~(uint32_t)MCLG_MOMENTS_DIGEST) || n_logs > (1ull << 62) / every)
    return MCLG_E_INVAL;
  const uint32_t dig = (flags & MCLG_MOMENTS_DIGEST) ? 1u : 0u;
  const uint32_t K = c->tb.steps;
  if (!(K > 1 && c->tb.T == 0 && !c->tb.reps && n_modes <= 2 && !(n_modes == 2 && dig))) {
    // steps, then the moment kernels, per log (partial sums in the workspace)
    unsigned long long *part = reinterpret_cast<unsigned long long *>(c->ws + c->lay.o_mpart);
    for (uint64_t j = 0; j < n_logs; ++j) {
      int rc = mclg_step(c, every);
      if (rc) return rc;
      MomArgs m = c->mom_args(part, reinterpret_cast<long long *>(dev_out + j * c->n));
      m.twiddle = twiddle;
      m.n_modes = n_modes;
      m.digest = dig;
      hipError_t e = c->flush_t();
      if (!e) e = launch_moments3(c->stream, m);
      if (e) return c->hip(e);
    }
    return MCLG_OK;
  }
  // launches of K steps (the last one shorter); each sums the logs that fall
  // in it, at steps every, 2 every, ... of the call.  With the digest or the
  // Galilean acceptance a launch also ends at each log (the kernel sums those
  // only as it writes the sites back).
  const bool at_end_only = dig || (c->flags & MCLG_FLAG_GALILEAN);
  const uint64_t total = every * n_logs;
  for (uint64_t c0 = 0; c0 < total;) {
    if (c->t_pending >= (1u << 30)) {
      hipError_t e = c->flush_t();
      if (e) return c->hip(e);
    }
    const uint64_t o1 = every - c0 % every;  // the first log after c0, relative
    const uint32_t S =
        (uint32_t)std::min<uint64_t>(std::min<uint64_t>(K, total - c0), at_end_only ? o1 : K);
    TbLaunch b = c->tb;
    b.steps = S;
    if (o1 <= S) {
      b.n_logs = (uint32_t)((S - o1) / every + 1u);
      b.log = 1u + 2u * n_modes + dig;
      b.log_first = (uint32_t)o1;
      b.log_every = (uint32_t)std::min<uint64_t>(every, K);  // (one log when every > K)
      b.tw = twiddle;
      b.out = reinterpret_cast<long long *>(dev_out + ((c0 + o1) / every - 1u) * c->n);
    }
    hipError_t e = c->launch_blocked(b);
    if (e) return c->hip(e);
    c->t[0] += S;
    c0 += S;
  }
  return MCLG_OK;
}

int mclg_histogram(mclg_ctx *c, uint32_t n_bins, uint64_t *hist) {
  if (!c || !hist || n_bins == 0 || n_bins > MCLG_MAX_HIST_BINS) return MCLG_E_INVAL;
  if (c->d2) return n_bins > 1024 ? MCLG_E_INVAL : d2q9_histogram(*c->d2, n_bins, hist);
  const hipError_t e =
      launch_histogram(c->stream, c->state, c->slots(), c->tiles_dev(), (uint32_t)c->tiles.size(),
                       c->sch.tile_sites(), n_bins, reinterpret_cast<unsigned long long *>(hist));
  return e ? c->hip(e) : MCLG_OK;
}

int mclg_get_counts(mclg_ctx *c, uint32_t r, uint16_t *out) {
  if (c && c->d2) return d2q9_get_counts(*c->d2, r, out);
  if (!c || !out || r >= c->n) return MCLG_E_INVAL;
  const uint64_t L = c->L[r], stride = c->lay.stride[r];
  std::vector<uint16_t> raw(3 * stride);
  hipError_t e = hipMemcpyAsync(raw.data(), c->state + c->lay.off[r], 3 * stride * 2,
                                hipMemcpyDeviceToHost, c->stream);
  if (!e) e = hipStreamSynchronize(c->stream);
  if (e) return c->hip(e);
  const uint64_t tm = (c->flags & MCLG_FLAG_NO_STREAM) ? 0 : (uint64_t)c->t[r] % L;
  for (uint64_t x = 0; x < L; ++x) {
    out[x] = raw[(x + tm) % L];
    out[L + x] = raw[stride + x];
    out[2 * L + x] = raw[2 * stride + (x + L - tm) % L];
  }
  return read_err(c);
}

int mclg_set_schedule(mclg_ctx *c, uint32_t groups, uint32_t threads, uint32_t lds_budget) {
  if (c && c->d2) return MCLG_E_UNSUPPORTED;
  if (!c) return MCLG_E_INVAL;
  if (groups != 1) return MCLG_E_INVAL;
  if (threads < 64 || threads > 1024 || threads % 64) return MCLG_E_INVAL;
  if (lds_budget > kMaxImage) return MCLG_E_INVAL;
  c->sch.groups = groups;
  c->sch.threads = threads;
  c->sch.lds_budget = lds_budget;
  c->tb = TbLaunch{};  // its geometry depends on the schedule: set it again
  c->tb_grid = 0;
  // graphs still in flight on the stream use the old tiles and images
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e) return c->hip(e);
  c->build_tiles();
  c->drop_graphs();
  e = hipMemcpyAsync(c->tiles_dev(), c->tiles.data(), sizeof(TileDev) * c->tiles.size(),
                                hipMemcpyHostToDevice, c->stream);
  if (!e) e = hipStreamSynchronize(c->stream);
  if (!e) e = c->prepare_images();
  return c->hip(e);
}

int mclg_set_grid_limit(mclg_ctx *c, uint32_t max_blocks) {
  if (c && c->d2) return MCLG_E_UNSUPPORTED;
  if (!c) return MCLG_E_INVAL;
  hipError_t e = hipStreamSynchronize(c->stream);
  c->grid_limit = max_blocks;
  c->drop_graphs();
  return c->hip(e);
}

int mclg_set_drain(mclg_ctx *c, uint32_t policy) {
  if (c && c->d2) return MCLG_E_UNSUPPORTED;
  if (!c || policy > MCLG_DRAIN_PATCH) return MCLG_E_INVAL;
  hipError_t e = hipStreamSynchronize(c->stream);  // captured graphs hold the old policy
  c->drain_policy = policy;
  c->drop_graphs();
  return c->hip(e);
}

int mclg_lds_coverage(const mclg_ctx *c, double *expected_fraction, uint32_t *lds_bytes) {
  if (c && c->d2) return MCLG_E_UNSUPPORTED;
  if (!c || !expected_fraction || !lds_bytes) return MCLG_E_INVAL;
  *expected_fraction = c->coverage;
  *lds_bytes = c->lds_bytes;
  return MCLG_OK;
}

int mclg_destroy(mclg_ctx *c) {
  if (!c) return MCLG_E_INVAL;
  if (c->d2) {
    if (c->d2->stream) (void)hipStreamSynchronize(c->d2->stream);
    delete c;
    return MCLG_OK;
  }
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  c->drop_graphs();
  delete c;
  return MCLG_OK;
}

const char *mclg_strerror(int code) {
  switch (code) {
    case MCLG_OK: return "ok";
    case MCLG_E_INVAL: return "invalid argument";
    case MCLG_E_RANGE: return "site occupation out of range";
    case MCLG_E_HIP: return "HIP runtime error";
    case MCLG_E_NOMEM: return "host out of memory";
    case MCLG_E_UNSUPPORTED: return "unsupported lattice or mode";
    case MCLG_E_FULL: return "server full";
    case MCLG_E_INTERNAL: return "internal consistency check failed";
    case MCLG_E_TOO_LARGE: return "input larger than the static scratch area";
    default: return "unknown error";
  }
}

int mclg_last_hip_error(const mclg_ctx *c) {
  return c ? (c->d2 ? c->d2->last_hip : c->last_hip) : 0;
}

int mclg_table_row(int32_t C, uint32_t p, uint32_t q, uint32_t flags, uint32_t N, uint32_t absJ,
                   uint32_t n0, uint64_t *thr, uint32_t cap, uint32_t *m_out) {
  if (!thr || !m_out || (flags & ~(uint32_t)MCLG_FLAG_GALILEAN)) return MCLG_E_INVAL;
  std::vector<uint64_t> full;
  if (!collision_row_full(C, p, q, (flags & MCLG_FLAG_GALILEAN) != 0, N, absJ, n0, full))
    return MCLG_E_INVAL;
  if (full.size() > cap) return MCLG_E_INVAL;
  std::copy(full.begin(), full.end(), thr);
  *m_out = (uint32_t)full.size() + 1;
  return MCLG_OK;
}

int mclg_galilean_lambda(uint32_t num, uint32_t den, uint32_t N, uint32_t absJ,
                         uint64_t *lambda_q) {
  if (!lambda_q || den == 0 || num == 0 || num > den || den >= (1u << 28) || absJ > N)
    return MCLG_E_INVAL;
  *lambda_q = galilean_lambda_q(num, den, N, absJ);
  return MCLG_OK;
}

int mclg_d2q9_rules(const uint32_t *lambda9, uint32_t *out, uint32_t *D) {
  if (!lambda9 || !out || !D) return MCLG_E_INVAL;
  std::vector<uint32_t> rules;
  if (!build_rules9(lambda9, rules, *D)) return MCLG_E_INVAL;
  std::copy(rules.begin(), rules.end(), out);
  return MCLG_OK;
}

int mclg_poisson_thresholds(double mu, uint32_t *k_lo, uint32_t *cnt, uint64_t *thr,
                            uint32_t cap) {
  if (!k_lo || !cnt || !thr) return MCLG_E_INVAL;
  std::vector<uint64_t> full;
  if (!poisson_full(mu, *k_lo, full)) return MCLG_E_INVAL;
  if (full.size() > cap) return MCLG_E_INVAL;
  std::copy(full.begin(), full.end(), thr);
  *cnt = (uint32_t)full.size() + 1;
  return MCLG_OK;
}

}  // extern "C"
