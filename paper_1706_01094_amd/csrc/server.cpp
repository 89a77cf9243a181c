// Continuous-batching server of MCLG simulation jobs.
//
// Jobs are queued on the host, admitted first-fit into a caller-owned device
// arena (their state stays resident until they finish), and advanced together
// by the batched stream+collide kernel: every launch covers the tiles of all
// resident jobs, each job at its own step t (per-slot step counters on the
// device).  A job's result depends only on (seed, job id, L, steps, rho, u0)
// and the collision parameters, never on what else is resident.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "../../include/mclg.h"
#include "device.h"
#include "moments.h"
#include "tables.h"

using namespace mclg;

namespace {

constexpr uint32_t kPad = 128;
constexpr uint32_t kPoisCap = 1024;
constexpr uint32_t kImage = 160 * 1024;  // LDS collision image budget per job (at most)
constexpr size_t kImageCacheMax = 4096;   // host images kept for reuse
inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

struct SrvLayout {
  uint64_t o_ctrl, o_slots, o_tslot, o_tiles, o_list, o_pdesc, o_pool, o_idesc, o_over, o_ipool,
      o_rowbase, o_rowdesc, o_thr, o_fixed, o_row16, bytes, max_tiles;
  // moments of retiring jobs: segments, runs, partial records, results
  uint64_t o_mseg, o_mrun, o_mslot, o_mpart, o_mout, max_mom_segs;
};

SrvLayout srv_layout(const mclg_server_config *cfg, const CollisionTables *tab,
                     uint32_t tile_sites) {
  SrvLayout l;
  uint64_t o = 0;
  auto take = [&](uint64_t b) {
    uint64_t at = o;
    o = align_up(o + b, 256);
    return at;
  };
  const uint64_t n = cfg->max_slots;
  // every resident site occupies 6 arena bytes; each slot adds one partial tile
  l.max_tiles = cfg->arena_bytes / (6ull * tile_sites) + n + 1;
  l.o_ctrl = take(256);
  l.o_slots = take(sizeof(SlotDev) * n);
  l.o_tslot = take(sizeof(uint32_t) * n);
  l.o_tiles = take(sizeof(TileDev) * l.max_tiles);
  l.o_list = take(sizeof(uint32_t) * n);
  l.max_mom_segs = max_mom_segs((uint32_t)n, cfg->arena_bytes / 6u);
  l.o_mseg = take(sizeof(MomSeg) * l.max_mom_segs);
  l.o_mrun = take(sizeof(uint32_t) * (n + 1));
  l.o_mslot = take(sizeof(uint32_t) * n);
  l.o_mpart = take(sizeof(uint64_t) * kMom3Rec * l.max_mom_segs);
  l.o_mout = take(sizeof(uint64_t) * kMom3Out * n);
  l.o_pdesc = take(sizeof(PoisDesc) * 3 * n);
  l.o_pool = take(sizeof(uint32_t) * kPoisCap * 3 * n);
  l.o_idesc = take(sizeof(ImageDesc) * n);
  l.o_over = take(kOverflowBytes);
  l.o_ipool = take((uint64_t)kImage * n);
  l.o_rowbase = take(sizeof(uint32_t) * tab->rowbase.size());
  l.o_rowdesc = take(sizeof(uint32_t) * tab->rowdesc.size());
  l.o_thr = take(sizeof(uint32_t) * (tab->thr.size() + 16));  // +16: see count_le_16
  l.o_fixed = take(sizeof(uint32_t) * tab->fixed.size());
  l.o_row16 = take(sizeof(uint16_t) * tab->row16.size());
  l.bytes = o;
  return l;
}

struct Resident {
  mclg_job job;
  uint64_t arena_off;   // bytes
  uint64_t bytes;
  uint64_t t = 0;
  bool active = false;
};

}  // namespace

struct mclg_server {
  mclg_server_config cfg;
  std::shared_ptr<const CollisionTables> tab;
  SrvLayout lay;
  Schedule sch;
  uint8_t *ws = nullptr;
  uint16_t *arena = nullptr;
  hipStream_t s = nullptr;
  std::deque<mclg_job> queue;
  std::vector<Resident> slot;
  std::map<uint64_t, uint64_t> free_spans;  // offset -> bytes
  uint64_t arena_used = 0;
  std::vector<mclg_job_result> done;
  // host mirrors of device tables (kept alive across async uploads)
  std::vector<SlotDev> h_slots;
  std::vector<TileDev> h_tiles;
  std::vector<uint32_t> h_list;
  std::vector<PoisDesc> h_pdesc;
  std::vector<uint32_t> h_pool;
  std::vector<ImageDesc> h_idesc;
  MomPlan h_mplan;  // segments of the jobs being retired
  // Host images by the (rho, |u0|) they are built for: jobs of equal density
  // and speed reuse one (the image depends on u0 only through |u0|), and the
  // cached bytes stay alive while their upload is in flight.
  struct CachedImage {
    std::vector<uint8_t> blob;
    uint32_t dir_bytes = 0, dim_a = 0, dim_c = 0, b_lo = 0, nb = 0;
  };
  std::map<std::pair<double, double>, CachedImage> image_cache;
  uint32_t n_tiles = 0, n_active = 0;
  uint32_t lds_bytes = 16, max_blocks = 1, image_budget = kImage, n_cu = 1;
  int last_hip = 0;

  uint32_t *err() { return reinterpret_cast<uint32_t *>(ws + lay.o_ctrl); }
  uint32_t *ticket() { return err() + 1; }
  SlotDev *d_slots() { return reinterpret_cast<SlotDev *>(ws + lay.o_slots); }
  uint32_t *d_tslot() { return reinterpret_cast<uint32_t *>(ws + lay.o_tslot); }
  TileDev *d_tiles() { return reinterpret_cast<TileDev *>(ws + lay.o_tiles); }
  uint32_t *d_list() { return reinterpret_cast<uint32_t *>(ws + lay.o_list); }
  TableDev table() {
    TableDev d;
    d.rowbase = reinterpret_cast<const uint32_t *>(ws + lay.o_rowbase);
    d.rowdesc = reinterpret_cast<const uint2 *>(ws + lay.o_rowdesc);
    d.thr = reinterpret_cast<const uint32_t *>(ws + lay.o_thr);
    d.fixed = tab->fixed.empty() ? nullptr : reinterpret_cast<const uint4 *>(ws + lay.o_fixed);
    d.row16 = tab->row16.empty() ? nullptr : reinterpret_cast<const uint4 *>(ws + lay.o_row16);
    return d;
  }
  int hip(hipError_t e) {
    if (e == hipSuccess) return MCLG_OK;
    last_hip = (int)e;
    return MCLG_E_HIP;
  }
  hipError_t up(void *dst, const void *src, size_t bytes) {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
  }

  bool alloc(uint64_t bytes, uint64_t &off) {
    for (auto it = free_spans.begin(); it != free_spans.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        uint64_t rest = it->second - bytes;
        free_spans.erase(it);
        if (rest) free_spans[off + bytes] = rest;
        arena_used += bytes;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    arena_used -= bytes;
    auto it = free_spans.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_spans.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_spans.erase(nx);
    }
    if (it != free_spans.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_spans.erase(it);
      }
    }
  }
  static uint64_t job_bytes(uint64_t L) { return 3 * align_up(L, kPad) * sizeof(uint16_t); }

  ImageDesc *d_idesc() { return reinterpret_cast<ImageDesc *>(ws + lay.o_idesc); }
  StepLaunch launch_args() {
    StepLaunch a{};
    a.state = arena;
    a.slots = d_slots();
    a.tslot = d_tslot();
    a.tiles = d_tiles();
    a.n_tiles = n_tiles;
    a.slot_list = d_list();
    a.slot_first = 0;
    a.n_slots = n_active;
    a.ticket = ticket();
    a.t_off = 0;
    a.single = 0;
    a.err = err();
    a.tab = table();
    a.p = params();
    a.p.drain = auto_drain(arena_used);  // by the resident jobs' state
    a.images = d_idesc();
    a.image_pool = ws + lay.o_ipool;
    a.overflow = reinterpret_cast<uint4 *>(ws + lay.o_over);
    a.lds_bytes = lds_bytes;
    a.max_blocks = max_blocks;
    return a;
  }
  StepParams params() const {
    StepParams p;
    p.seed = cfg.seed;
    p.C = cfg.C;
    p.lam_p = cfg.lambda_num;
    p.lam_q = cfg.lambda_den;
    p.n_max = cfg.n_max;
    p.no_stream = 0;
    p.galilean = 0;
    p.tile_sites = sch.tile_sites();
    return p;
  }

  // Rebuild the tile and slot lists of the resident jobs and upload them.
  hipError_t rebuild_lists() {
    h_tiles.clear();
    h_list.clear();
    const uint32_t ts = sch.tile_sites();
    for (uint32_t i = 0; i < slot.size(); ++i) {
      if (!slot[i].active) continue;
      h_list.push_back(i);
      const uint32_t next = (uint32_t)(h_tiles.size() + (slot[i].job.L + ts - 1) / ts);
      for (uint64_t x0 = 0; x0 < slot[i].job.L; x0 += ts) h_tiles.push_back(TileDev{i, (uint32_t)x0, next, 0});
    }
    if (h_tiles.size() > lay.max_tiles) return hipErrorInvalidValue;
    n_tiles = (uint32_t)h_tiles.size();
    n_active = (uint32_t)h_list.size();
    hipError_t e = up(d_tiles(), h_tiles.data(), sizeof(TileDev) * h_tiles.size());
    if (!e) e = up(d_list(), h_list.data(), sizeof(uint32_t) * h_list.size());
    return e;
  }

  // Admit queued jobs (FIFO, stop at the first that does not fit).
  int admit() {
    std::vector<uint32_t> fresh;
    while (!queue.empty()) {
      const mclg_job &j = queue.front();
      uint32_t free_slot = UINT32_MAX;
      for (uint32_t i = 0; i < slot.size(); ++i)
        if (!slot[i].active) { free_slot = i; break; }
      if (free_slot == UINT32_MAX) break;
      uint64_t bytes = job_bytes(j.L), off = 0;
      if (!alloc(bytes, off)) break;
      Resident &r = slot[free_slot];
      r.job = j;
      r.arena_off = off;
      r.bytes = bytes;
      r.t = 0;
      r.active = true;
      SlotDev &sd = h_slots[free_slot];
      sd.off = off / sizeof(uint16_t);
      sd.dense = 0;
      sd.L = (uint32_t)j.L;
      sd.stride = (uint32_t)align_up(j.L, kPad);
      sd.rid = (uint32_t)j.job_id;
      sd.pad = 0;
      double mu[3];
      feq(j.rho, j.u0, mu);
      for (int i = 0; i < 3; ++i) {
        uint32_t k_lo = 0;
        std::vector<uint64_t> full;
        poisson_full(mu[i], k_lo, full);
        CompactLaw cl = compact(k_lo, full);
        PoisDesc &d = h_pdesc[3 * free_slot + i];
        d.off = (3 * free_slot + i) * kPoisCap;
        d.k_first = cl.k_first;
        d.nthr = (uint32_t)cl.thr.size();
        std::copy(cl.thr.begin(), cl.thr.end(), h_pool.begin() + d.off);
      }
      // collision image for this job's density and speed (cached on the host)
      const auto key = std::make_pair(j.rho, std::fabs(j.u0));
      auto ci = image_cache.find(key);
      if (ci == image_cache.end()) {
        if (image_cache.size() >= kImageCacheMax) {
          hipError_t e = hipStreamSynchronize(s);  // no upload may still read them
          if (e) return hip(e);
          image_cache.clear();
        }
        LdsImage im = build_image(*tab, j.rho, std::fabs(j.u0), image_budget);
        CachedImage c;
        c.blob = im.blob();
        c.dir_bytes = im.dir_bytes();
        c.dim_a = im.dim_a;
        c.dim_c = im.dim_c;
        c.b_lo = im.b_lo;
        c.nb = im.nb;
        ci = image_cache.emplace(key, std::move(c)).first;
      }
      const CachedImage &img = ci->second;
      ImageDesc &idd = h_idesc[free_slot];
      idd.off = (uint64_t)free_slot * kImage;
      idd.bytes = (uint32_t)img.blob.size();
      idd.dir_bytes = img.dir_bytes;
      idd.dim_a = img.dim_a;
      idd.dim_c = img.dim_c;
      idd.b_lo = img.b_lo;
      idd.nb = img.nb;
      if (idd.bytes) {
        hipError_t e = hipMemcpyAsync(ws + lay.o_ipool + idd.off, img.blob.data(), img.blob.size(),
                                      hipMemcpyHostToDevice, s);
        if (e) return hip(e);
      }
      fresh.push_back(free_slot);
      queue.pop_front();
    }
    if (fresh.empty()) return MCLG_OK;
    // Upload the changed host mirrors; then initialise the new jobs only.
    std::vector<TileDev> init_tiles;
    const uint32_t ts = sch.tile_sites();
    for (uint32_t i : fresh)
      for (uint64_t x0 = 0; x0 < slot[i].job.L; x0 += ts) init_tiles.push_back(TileDev{i, (uint32_t)x0, 0, 0});
    if (init_tiles.size() > lay.max_tiles) return MCLG_E_INVAL;
    hipError_t e = hipSuccess;
    for (uint32_t i : fresh) {  // only the admitted slots' entries change
      if (!e) e = up(d_slots() + i, &h_slots[i], sizeof(SlotDev));
      if (!e) e = up(d_idesc() + i, &h_idesc[i], sizeof(ImageDesc));
      if (!e) e = up(ws + lay.o_pdesc + sizeof(PoisDesc) * 3 * i, &h_pdesc[3 * i], sizeof(PoisDesc) * 3);
      if (!e) e = up(ws + lay.o_pool + sizeof(uint32_t) * kPoisCap * 3 * i,
                     &h_pool[(size_t)kPoisCap * 3 * i], sizeof(uint32_t) * kPoisCap * 3);
    }
    // fresh slot ids and their tiles go through the list/tile areas, which
    // are rebuilt right after
    if (!e) e = up(d_list(), fresh.data(), sizeof(uint32_t) * fresh.size());
    if (!e) e = up(d_tiles(), init_tiles.data(), sizeof(TileDev) * init_tiles.size());
    if (!e) e = launch_set_t(s, d_tslot(), d_list(), (uint32_t)fresh.size(), 0u);
    if (!e)
      e = launch_init_poisson(s, arena, d_slots(), d_tslot(), d_tiles(), (uint32_t)init_tiles.size(),
                              ts, reinterpret_cast<const PoisDesc *>(ws + lay.o_pdesc),
                              reinterpret_cast<const uint32_t *>(ws + lay.o_pool), cfg.seed, err());
    if (!e) e = hipStreamSynchronize(s);
    if (!e) e = rebuild_lists();
    if (!e) e = hipStreamSynchronize(s);
    return hip(e);
  }

  // Moments (with the state digest) of finished jobs, then free their slots.
  int retire() {
    std::vector<uint32_t> fin;
    std::vector<uint64_t> sites;
    for (uint32_t i = 0; i < slot.size(); ++i)
      if (slot[i].active && slot[i].t >= slot[i].job.steps) {
        fin.push_back(i);
        sites.push_back(slot[i].job.L);
      }
    if (fin.empty()) return MCLG_OK;
    h_mplan = plan_moments(fin.data(), sites.data(), (uint32_t)fin.size());
    if (h_mplan.segs.size() > lay.max_mom_segs) return MCLG_E_INTERNAL;
    MomArgs m;
    m.state = arena;
    m.slots = d_slots();
    m.tslot = d_tslot();
    m.segs = reinterpret_cast<const MomSeg *>(ws + lay.o_mseg);
    m.n_segs = (uint32_t)h_mplan.segs.size();
    m.run_seg = reinterpret_cast<const uint32_t *>(ws + lay.o_mrun);
    m.run_slot = reinterpret_cast<const uint32_t *>(ws + lay.o_mslot);
    m.n_runs = (uint32_t)fin.size();
    m.digest = 1u;
    m.partial = reinterpret_cast<unsigned long long *>(ws + lay.o_mpart);
    m.out = reinterpret_cast<long long *>(ws + lay.o_mout);
    hipError_t e = up(ws + lay.o_mseg, h_mplan.segs.data(), sizeof(MomSeg) * h_mplan.segs.size());
    if (!e) e = up(ws + lay.o_mrun, h_mplan.run_seg.data(), 4 * h_mplan.run_seg.size());
    if (!e) e = up(ws + lay.o_mslot, h_mplan.run_slot.data(), 4 * h_mplan.run_slot.size());
    if (!e) e = launch_moments3(s, m);
    std::vector<mclg_moments_t> h(fin.size());
    if (!e) e = hipMemcpyAsync(h.data(), ws + lay.o_mout, sizeof(mclg_moments_t) * h.size(),
                               hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return hip(e);
    for (size_t k = 0; k < fin.size(); ++k) {
      const uint32_t i = fin[k];
      mclg_job_result res;
      std::memset(&res, 0, sizeof(res));
      res.job_id = slot[i].job.job_id;
      res.moments = h[k];
      res.moments.t = (int64_t)slot[i].t;
      done.push_back(res);
      slot[i].active = false;
      release(slot[i].arena_off, slot[i].bytes);
    }
    e = rebuild_lists();
    if (!e) e = hipStreamSynchronize(s);
    return hip(e);
  }
};

extern "C" {

int mclg_server_sizes(const mclg_server_config *cfg, uint64_t *workspace_bytes) {
  if (!cfg || cfg->abi_version != MCLG_ABI_VERSION || cfg->max_slots == 0 || !workspace_bytes)
    return MCLG_E_INVAL;
  if (!params_ok(cfg->C, cfg->lambda_num, cfg->lambda_den, cfg->n_max, false))
    return MCLG_E_INVAL;
  auto tab = collision_tables(cfg->C, cfg->lambda_num, cfg->lambda_den, cfg->n_max, false);
  if (!tab) return MCLG_E_INVAL;
  Schedule sch;
  *workspace_bytes = srv_layout(cfg, tab.get(), sch.tile_sites()).bytes;
  return MCLG_OK;
}

int mclg_server_create(const mclg_server_config *cfg, mclg_server **out) {
  uint64_t need = 0;
  int rc = mclg_server_sizes(cfg, &need);
  if (rc) return rc;
  if (!out || !cfg->arena || !cfg->workspace || cfg->workspace_bytes < need) return MCLG_E_INVAL;
  std::unique_ptr<mclg_server> sv(new (std::nothrow) mclg_server());
  if (!sv) return MCLG_E_NOMEM;
  sv->cfg = *cfg;
  sv->tab = collision_tables(cfg->C, cfg->lambda_num, cfg->lambda_den, cfg->n_max, false);
  sv->lay = srv_layout(cfg, sv->tab.get(), sv->sch.tile_sites());
  sv->ws = reinterpret_cast<uint8_t *>(cfg->workspace);
  sv->arena = reinterpret_cast<uint16_t *>(cfg->arena);
  sv->s = reinterpret_cast<hipStream_t>(cfg->stream);
  sv->slot.resize(cfg->max_slots);
  sv->h_slots.assign(cfg->max_slots, SlotDev{});
  sv->h_pdesc.assign(3ull * cfg->max_slots, PoisDesc{});
  sv->h_pool.assign((size_t)kPoisCap * 3 * cfg->max_slots, 0);
  sv->h_idesc.assign(cfg->max_slots, ImageDesc{});
  {
    int dev = 0, v = 0;
    hipError_t e = hipGetDevice(&dev);
    if (!e) e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    const uint32_t queues = (sv->sch.threads / 64u) * kWaveLdsBytes;
    if (!e) sv->image_budget = std::min<uint32_t>(kImage, (uint32_t)std::max(0, v - 1024 - (int)queues)) / 16u * 16u;
    if (!e) e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
    if (!e) sv->n_cu = (uint32_t)std::max(1, v);
    if (!e && sv->n_cu > 256) return MCLG_E_UNSUPPORTED;  // overflow region sized for 256 CUs
    sv->lds_bytes = std::max<uint32_t>(64, sv->image_budget);  // the smallest image is 48 bytes
    if (!e) e = step_occupancy(sv->sch, sv->lds_bytes, sv->n_cu, sv->max_blocks);
    if (e) return sv->hip(e);
  }
  uint64_t usable = cfg->arena_bytes / 256 * 256;
  if (usable) sv->free_spans[0] = usable;
  std::vector<uint32_t> ctrl(64, 0), tz(cfg->max_slots, 0);
  const CollisionTables &t = *sv->tab;
  hipError_t e = sv->up(sv->ws + sv->lay.o_ctrl, ctrl.data(), 256);
  if (!e) e = sv->up(sv->d_tslot(), tz.data(), 4 * tz.size());
  if (!e) e = sv->up(sv->ws + sv->lay.o_rowbase, t.rowbase.data(), 4 * t.rowbase.size());
  if (!e) e = sv->up(sv->ws + sv->lay.o_rowdesc, t.rowdesc.data(), 4 * t.rowdesc.size());
  if (!e) e = sv->up(sv->ws + sv->lay.o_thr, t.thr.data(), 4 * t.thr.size());
  if (!e && !t.fixed.empty()) e = sv->up(sv->ws + sv->lay.o_fixed, t.fixed.data(), 4 * t.fixed.size());
  if (!e && !t.row16.empty()) e = sv->up(sv->ws + sv->lay.o_row16, t.row16.data(), 2 * t.row16.size());
  if (!e) e = hipStreamSynchronize(sv->s);
  if (e) return sv->hip(e);
  *out = sv.release();
  return MCLG_OK;
}

int mclg_server_submit(mclg_server *sv, const mclg_job *job) {
  if (!sv || !job || job->L == 0 || job->L > kMaxSites || job->job_id >= (1ull << 32))
    return MCLG_E_INVAL;
  if (!(job->rho >= 0.0) || !(job->u0 >= -1.0 && job->u0 <= 1.0)) return MCLG_E_INVAL;
  if (mclg_server::job_bytes(job->L) > sv->cfg.arena_bytes / 256 * 256) return MCLG_E_INVAL;
  double mu[3];
  feq(job->rho, job->u0, mu);
  for (double m : mu) {
    uint32_t k_lo = 0;
    std::vector<uint64_t> full;
    if (!poisson_full(m, k_lo, full) || compact(k_lo, full).thr.size() > kPoisCap) return MCLG_E_INVAL;
  }
  sv->queue.push_back(*job);
  return MCLG_OK;
}

int mclg_server_tick(mclg_server *sv, uint32_t k) {
  if (!sv) return MCLG_E_INVAL;
  int rc = sv->admit();
  if (rc) return rc;
  uint32_t left = k;
  while (left > 0) {
    if (sv->n_active == 0) {
      rc = sv->admit();
      if (rc) return rc;
      if (sv->n_active == 0) break;
    }
    uint64_t chunk = left;
    for (auto &r : sv->slot)
      if (r.active) chunk = std::min<uint64_t>(chunk, r.job.steps - r.t);
    for (uint64_t i = 0; i < chunk; ++i) {
      hipError_t e = launch_step(sv->sch, sv->s, sv->launch_args());
      if (e) return sv->hip(e);
    }
    for (auto &r : sv->slot)
      if (r.active) r.t += chunk;
    left -= (uint32_t)chunk;
    rc = sv->retire();
    if (rc) return rc;
    rc = sv->admit();
    if (rc) return rc;
  }
  return MCLG_OK;
}

int mclg_server_poll(mclg_server *sv, mclg_job_result *out, uint32_t cap, uint32_t *n_out) {
  if (!sv || !n_out || (cap && !out)) return MCLG_E_INVAL;
  uint32_t n = (uint32_t)std::min<size_t>(cap, sv->done.size());
  std::copy(sv->done.begin(), sv->done.begin() + n, out);
  sv->done.erase(sv->done.begin(), sv->done.begin() + n);
  *n_out = n;
  uint32_t err = 0;
  hipError_t e = hipMemcpy(&err, sv->err(), sizeof(err), hipMemcpyDeviceToHost);
  if (e) return sv->hip(e);
  return (err & 4u) ? MCLG_E_INTERNAL : err ? MCLG_E_RANGE : MCLG_OK;
}

int mclg_server_stats(const mclg_server *sv, uint64_t *queued, uint64_t *resident,
                      uint64_t *arena_used) {
  if (!sv) return MCLG_E_INVAL;
  if (queued) *queued = sv->queue.size();
  if (resident) *resident = sv->n_active;
  if (arena_used) *arena_used = sv->arena_used;
  return MCLG_OK;
}

int mclg_server_destroy(mclg_server *sv) {
  if (!sv) return MCLG_E_INVAL;
  if (sv->s) (void)hipStreamSynchronize(sv->s);
  delete sv;
  return MCLG_OK;
}

}  // extern "C"
