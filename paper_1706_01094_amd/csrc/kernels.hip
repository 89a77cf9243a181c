// HIP kernels of the MCLG library for gfx950 (MI355X).
//
// The hot kernel fuses streaming and the Monte Carlo collision of the D1Q3
// integer lattice gas (Sec. "The Monte Carlo Lattice Gas algorithm" and
// "A D1Q3 implementation"): per site it loads n_-1, n_0, n_+1 (uint16) from
// the in-place shifted layout, draws the post-collision rest count from the
// exact C-sub-collision law with one Philox4x32-10 word, restores n_-1 and
// n_+1 from the conserved N and J, and stores the three counts back to the
// same three physical locations -- streaming is the shift of the layout.
// Algorithmic traffic: 6 B read + 6 B written per site update; there is no
// dense contraction, so no MFMA.
#include "device.h"

#include <algorithm>

namespace mclg {
namespace {

constexpr uint32_t kErrOverflow = 1u;   // a site with N > 65535
constexpr uint32_t kErrEqRange = 2u;    // C = infinity and N > n_max

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds, multipliers 0xD2511F53,
// 0xCD9E8D57, Weyl increments 0x9E3779B9, 0xBB67AE85.
__device__ __forceinline__ uint4 philox10(uint4 c, uint2 k) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    if (i) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    // one 32x32 -> 64-bit multiply per product (v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k.x, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k.y,
                   (uint32_t)p0);
  }
  return c;
}

__device__ __forceinline__ uint32_t word_of(const uint4 &w, uint32_t i) {
  return i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w;
}

// number of entries <= r in an ascending array (binary search)
__device__ __forceinline__ uint32_t count_le(const uint32_t *__restrict__ t, uint32_t n,
                                             uint32_t r) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (t[mid] <= r) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Random word stream of the literal sub-collision loop of one site:
// Philox blocks (x, t, replica, 2 | j << 2), j = 0, 1, ..., words in order.
struct WordStream {
  uint2 key;
  uint32_t x, t, rid, block, used;
  uint4 buf;
  __device__ uint32_t next() {
    if (used == 4) {
      buf = philox10(make_uint4(x, t, rid, 2u | (block << 2)), key);
      ++block;
      used = 0;
    }
    return word_of(buf, used++);
  }
  // exact uniform integer in [0, s): multiply-and-reject (Lemire, 2019)
  __device__ uint32_t uniform(uint32_t s) {
    uint64_t m = (uint64_t)next() * s;
    if ((uint32_t)m < s) {
      const uint32_t floor_ = (0u - s) % s;
      while ((uint32_t)m < floor_) m = (uint64_t)next() * s;
    }
    return (uint32_t)(m >> 32);
  }
};

// The paper's C sub-collisions one by one (Eq. (select), Eq. (omega)); used
// for sites with N > n_max.  Returns the new rest count.
__device__ __forceinline__ uint32_t collide_direct(uint32_t a, uint32_t b, uint32_t c,
                                                const StepParams &p, uint32_t x, uint32_t t,
                                                uint32_t rid) {
  WordStream ws;
  ws.key = make_uint2((uint32_t)p.seed, (uint32_t)(p.seed >> 32));
  ws.x = x; ws.t = t; ws.rid = rid; ws.block = 0; ws.used = 4;
  const uint32_t N = a + b + c;
  for (int32_t s = 0; s < p.C; ++s) {
    const uint32_t r1 = ws.uniform(N);
    uint32_t r2 = ws.uniform(N - 1);
    r2 += (r2 >= r1);
    const int v1 = r1 < a ? -1 : (r1 < a + b ? 0 : 1);
    const int v2 = r2 < a ? -1 : (r2 < a + b ? 0 : 1);
    if (v1 + v2 == 0 && v1 != 0) {
      if (ws.uniform(p.lam_q) < p.lam_p) { a -= 1; c -= 1; b += 2; }
    } else if (v1 == 0 && v2 == 0) {
      if (ws.uniform(8u * p.lam_q) < p.lam_p) { b -= 2; a += 1; c += 1; }
    }
  }
  return b;
}

// Exact row of the global tables: the number of thresholds <= r.
__device__ __forceinline__ uint32_t global_outcome(const TableDev &tab, uint32_t N, uint32_t absJ,
                                                   uint32_t b, uint32_t par, uint32_t r) {
  const uint32_t base = tab.rowbase[(N * (N + 1u) >> 1) + absJ];
  const uint2 d = tab.rowdesc[base + ((b - par) >> 1)];  // fiber states ascend in n0
  return (d.y & 0xffffu) + count_le(tab.thr + d.x, (d.y >> 16) - 1u, r);
}

// The slot's collision image in LDS: directory of (min(a,c), max(a,c)) pairs,
// then 16-byte records (k_s, top 16 bits of 7 thresholds).  Decides the
// outcome exactly whenever the top 16 bits of r fall strictly inside the
// record's window and differ from every stored value; returns false
// otherwise.
struct LdsView {
  const uint16_t *dir;
  const uint4 *rec;
  uint32_t dim_a, dim_c, b_lo, nb;
};

__device__ __forceinline__ bool lds_outcome(const LdsView &v, uint32_t a, uint32_t b, uint32_t c,
                                            uint32_t r, uint32_t &idx) {
  const uint32_t lo = min(a, c), hi = max(a, c), bi = b - v.b_lo;
  if (lo >= v.dim_a || hi >= v.dim_c || bi >= v.nb) return false;
  const uint32_t pidx = v.dir[lo * v.dim_c + hi];
  if (pidx == 0xFFFFu) return false;
  const uint4 q = v.rec[pidx * v.nb + bi];
  const uint32_t rh = r >> 16;
  const uint32_t t1 = q.x >> 16, t2 = q.y & 0xffffu, t3 = q.y >> 16, t4 = q.z & 0xffffu,
                 t5 = q.z >> 16, t6 = q.w & 0xffffu, t7 = q.w >> 16;
  const bool inside = (rh > t1) & (rh < t7);
  const bool tie = (rh == t2) | (rh == t3) | (rh == t4) | (rh == t5) | (rh == t6);
  idx = (q.x & 0xffffu) + (uint32_t)(t2 < rh) + (uint32_t)(t3 < rh) + (uint32_t)(t4 < rh) +
        (uint32_t)(t5 < rh) + (uint32_t)(t6 < rh);
  return inside & !tie;
}

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t get16(const uint32_t (&w)[4], int e) {
  return (e & 1) ? (w[e >> 1] >> 16) : (w[e >> 1] & 0xffffu);
}
__device__ __forceinline__ void set16(uint32_t (&w)[4], int e, uint32_t v) {
  if (e & 1) w[e >> 1] = (w[e >> 1] & 0xffffu) | (v << 16);
  else w[e >> 1] = (w[e >> 1] & 0xffff0000u) | (v & 0xffffu);
}
// out = elements [s, s + 8) of the sixteen uint16 of (lo ++ hi); s is
// wave-uniform, 0 <= s <= 8.
__device__ __forceinline__ void extract8(const uint32_t (&lo)[4], const uint32_t (&hi)[4],
                                         uint32_t s, uint32_t (&out)[4]) {
  const uint32_t w[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  const uint32_t sh = (s & 1u) * 2u;
  switch (s >> 1) {
#define MCLG_EXTRACT_CASE(K)                                                      \
  case K:                                                                         \
    for (int j = 0; j < 4; ++j)                                                   \
      out[j] = (K + j + 1 < 8) ? __builtin_amdgcn_alignbyte(w[(K + j + 1) & 7], w[K + j], sh) \
                               : w[K + j];                                        \
    break;
    MCLG_EXTRACT_CASE(0)
    MCLG_EXTRACT_CASE(1)
    MCLG_EXTRACT_CASE(2)
    MCLG_EXTRACT_CASE(3)
#undef MCLG_EXTRACT_CASE
    default:
      for (int j = 0; j < 4; ++j) out[j] = hi[j];
  }
}
__device__ __forceinline__ void shfl_down4(const uint32_t (&v)[4], uint32_t (&o)[4]) {
  for (int j = 0; j < 4; ++j) o[j] = __shfl_down(v[j], 1u);
}
__device__ __forceinline__ void shfl_up4(const uint32_t (&v)[4], uint32_t (&o)[4]) {
  for (int j = 0; j < 4; ++j) o[j] = __shfl_up(v[j], 1u);
}
__device__ __forceinline__ void load4(const uint16_t *p, uint32_t (&v)[4]) {
  const uint4 q = *reinterpret_cast<const uint4 *>(p);
  v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}
__device__ __forceinline__ void store4(uint16_t *p, const uint32_t (&v)[4]) {
  *reinterpret_cast<uint4 *>(p) = make_uint4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Eight consecutive elements [s, s + 8) of an array whose window of 512
// elements starting at s does not wrap: lane-aligned 16-byte loads, the next
// lane's vector by a shuffle (the last lane reads the vector after the
// window), and a byte-align by the wave-uniform misalignment s & 7.
__device__ __forceinline__ void load_window(const uint16_t *arr, uint32_t s, uint32_t lane,
                                            uint32_t (&out)[4]) {
  const uint32_t bmis = s & 7u, A = s - bmis;
  uint32_t v[4], nx[4];
  load4(arr + A + 8u * lane, v);
  if (bmis == 0u) {
    for (int j = 0; j < 4; ++j) out[j] = v[j];
    return;
  }
  uint32_t ext[4];
  load4(arr + A + 512u, ext);
  shfl_down4(v, nx);
  if (lane == 63u)
    for (int j = 0; j < 4; ++j) nx[j] = ext[j];
  extract8(v, nx, bmis, out);
}
// Inverse of load_window: lanes 1..63 store their aligned vector; lane 0
// and lane 63 store only the elements of the two boundary vectors this
// window owns (the rest belongs to the neighbouring windows).
__device__ __forceinline__ void store_window(uint16_t *arr, uint32_t s, uint32_t lane,
                                             const uint32_t (&o)[4]) {
  const uint32_t bmis = s & 7u, A = s - bmis;
  if (bmis == 0u) {
    store4(arr + A + 8u * lane, o);
    return;
  }
  uint32_t prev[4], al[4];
  shfl_up4(o, prev);
  extract8(prev, o, 8u - bmis, al);
  if (lane != 0u) {
    store4(arr + A + 8u * lane, al);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if ((uint32_t)e < 8u - bmis) arr[s + e] = (uint16_t)get16(o, e);
  }
  if (lane == 63u) {
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if ((uint32_t)e < bmis) arr[A + 512u + e] = (uint16_t)get16(o, 8 - (int)bmis + e);
  }
}

// Element k of a site triple gets rest count bn; n_-1 and n_+1 follow from
// the conserved N and J (Eq. (collcons)).
__device__ __forceinline__ void apply_outcome(uint32_t (&va)[4], uint32_t (&vb)[4],
                                              uint32_t (&vc)[4], int k, uint32_t bn) {
  const int32_t ea = (int32_t)get16(va, k), eb = (int32_t)get16(vb, k),
                ec = (int32_t)get16(vc, k);
  const int32_t N = ea + eb + ec, J = ec - ea;
  set16(va, k, (uint32_t)((N - (int32_t)bn - J) >> 1));
  set16(vb, k, bn);
  set16(vc, k, (uint32_t)((N - (int32_t)bn + J) >> 1));
}

// Per-wave queue of draws the LDS image could not decide (or sites with
// N > n_max); drained by all lanes at once.
constexpr uint32_t kQueue = kQueueBytesPerWave / 16;

// Exact outcome for a queued site: global row, or the literal loop.
__device__ __forceinline__ uint32_t resolve_queued(const uint4 e, const StepParams &p,
                                                const TableDev &tab, uint32_t t, uint32_t rid,
                                                uint32_t *err) {
  const uint32_t x = e.x, a = e.y & 0xffffu, b = e.y >> 16, c = e.z, r = e.w;
  const uint32_t N = a + b + c;
  if (N <= p.n_max) {
    const uint32_t absJ = (uint32_t)abs((int32_t)c - (int32_t)a);
    const uint32_t par = (N - absJ) & 1u;
    return par + 2u * global_outcome(tab, N, absJ, b, par, r);
  }
  if (p.C < 0) {
    atomicOr(err, kErrEqRange);
    return b;
  }
  return collide_direct(a, b, c, p, x, t, rid);
}

// Per-chunk state of one lane while its eight sites are decided.
struct ChunkCtx {
  uint32_t x8;     // first of the lane's eight sites
  uint4 w0, w1;    // Philox words of sites x8 .. x8 + 7
  uint32_t L;
  uint32_t qn;     // the wave's queue fill (wave-uniform)
};

// Where a slot's three arrays are and how they are shifted at step t.
struct SlotView {
  uint16_t *nm, *n0, *np;
  uint32_t L, tm, t, rid;
};

// Site K of the lane: decide from the LDS image, or queue it (all lanes
// place their queued sites by ballot order).  Branch-free apart from the
// queue: indices are clamped into the image and the outcome is selected.
// With b' drawn, n_-1 and n_+1 follow from the conserved N and J
// (Eq. (collcons)): a' = a + (b - b')/2, c' = c + (b - b')/2.
template <int K>
__device__ __forceinline__ void decide_site(ChunkCtx &cx, bool full, uint32_t (&va)[4],
                                            uint32_t (&vb)[4], uint32_t (&vc)[4],
                                            const LdsView &lv, uint4 *queue,
                                            const StepParams &p, const TableDev &tab, uint32_t t,
                                            uint32_t rid, uint32_t *err) {
  const uint4 &w = K < 4 ? cx.w0 : cx.w1;
  const uint32_t r = (K & 3) == 0 ? w.x : (K & 3) == 1 ? w.y : (K & 3) == 2 ? w.z : w.w;
  const uint32_t ea = get16(va, K), eb = get16(vb, K), ec = get16(vc, K);
  const uint32_t N = ea + eb + ec;
  const bool live = full | (cx.x8 + K < cx.L);
  if (live & (N > 65535u)) atomicOr(err, kErrOverflow);
  const bool collide = live & (N >= 2u) & (N <= 65535u) & (p.C != 0);
  // LDS image lookup with clamped indices
  const uint32_t lo = min(ea, ec), hi = max(ea, ec), bi = eb - lv.b_lo;
  const bool inbox = (lo < lv.dim_a) & (hi < lv.dim_c) & (bi < lv.nb) & (N <= p.n_max);
  const uint32_t pidx = lv.dir[inbox ? __umul24(lo, lv.dim_c) + hi : 0u];
  const bool have = inbox & (pidx != 0xFFFFu);
  const uint4 q = lv.rec[have ? __umul24(pidx, lv.nb) + bi : 0u];
  const uint32_t rh = r >> 16;
  const uint32_t t1 = q.x >> 16, t2 = q.y & 0xffffu, t3 = q.y >> 16, t4 = q.z & 0xffffu,
                 t5 = q.z >> 16, t6 = q.w & 0xffffu, t7 = q.w >> 16;
  const bool hit = have & (rh > t1) & (rh < t7) & (rh != t2) & (rh != t3) & (rh != t4) &
                   (rh != t5) & (rh != t6);
  const uint32_t idx = (q.x & 0xffffu) + (uint32_t)(t2 < rh) + (uint32_t)(t3 < rh) +
                       (uint32_t)(t4 < rh) + (uint32_t)(t5 < rh) + (uint32_t)(t6 < rh);
  const uint32_t par = eb & 1u;  // N - |J| = b + 2 min(a, c): the fiber's parity is b's
  const uint32_t bn = par + 2u * idx;
  const int32_t d = (collide & hit) ? ((int32_t)eb - (int32_t)bn) >> 1 : 0;
  set16(va, K, (uint32_t)((int32_t)ea + d));
  set16(vb, K, (uint32_t)((int32_t)eb - 2 * d));
  set16(vc, K, (uint32_t)((int32_t)ec + d));
  const bool miss = collide & !hit;
  const uint64_t bal = __ballot(miss);
  if (bal) {
    const uint32_t cnt = (uint32_t)__popcll(bal);
    const uint4 e = make_uint4(cx.x8 + K, ea | (eb << 16), ec, r);
    if (cx.qn + cnt <= kQueue) {
      // queued: the state keeps the pre-collision counts until the drain
      // writes the final ones
      if (miss) queue[cx.qn + lanes_below(bal)] = e;
      cx.qn += cnt;
    } else if (miss) {  // queue full: this lane resolves the site itself
      apply_outcome(va, vb, vc, K, resolve_queued(e, p, tab, t, rid, err));
    }
  }
}

// Resolve every queued draw of the wave (all lanes in parallel) and store
// the site's three final counts.  The wave first waits until all of its
// earlier memory operations have completed -- among them the stores that
// wrote the pre-collision counts of these sites -- so the final counts land
// after them.
__device__ __forceinline__ void drain_queue(uint4 *queue, uint32_t qn, uint32_t lane,
                                            const SlotView &v, const StepParams &p,
                                            const TableDev &tab, uint32_t *err) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0);  // vmcnt = expcnt = lgkmcnt = 0
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  for (uint32_t i = lane; i < qn; i += 64u) {
    const uint4 e = queue[i];
    const uint32_t x = e.x, ea = e.y & 0xffffu, eb = e.y >> 16, ec = e.z;
    const uint32_t bn = resolve_queued(e, p, tab, v.t, v.rid, err);
    const int32_t N = (int32_t)(ea + eb + ec), J = (int32_t)ec - (int32_t)ea;
    uint32_t pm = x + v.tm;
    pm -= (pm >= v.L) ? v.L : 0u;
    const uint32_t pp = x >= v.tm ? x - v.tm : x + v.L - v.tm;
    v.nm[pm] = (uint16_t)((N - (int32_t)bn - J) >> 1);
    v.n0[x] = (uint16_t)bn;
    v.np[pp] = (uint16_t)((N - (int32_t)bn + J) >> 1);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Fused stream + collide.  Persistent blocks: block i takes a contiguous run
// of tiles (so consecutive tiles mostly share a slot) and loads the slot's
// collision image into LDS whenever the slot changes.  A tile holds
// G chunks of 512 sites per wave; each lane owns 8 consecutive sites of a
// chunk (two Philox calls).  All state of a tile is loaded before any of it
// is stored: every physical element belongs to exactly one site per step.
template <int G>
__global__ void __launch_bounds__(1024) k_step(StepLaunch a) {
  extern __shared__ uint4 lds[];
  const StepParams &p = a.p;
  const uint2 key = make_uint2((uint32_t)p.seed, (uint32_t)(p.seed >> 32));
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  uint4 *const queue = lds + a.lds_bytes / 16u + wave * kQueue;
  const uint32_t per = (a.n_tiles + gridDim.x - 1) / gridDim.x;
  const uint32_t tb = blockIdx.x * per;
  const uint32_t te = min(a.n_tiles, tb + per);
  uint32_t cur = 0xFFFFFFFFu;
  uint32_t qn = 0;  // queued draws of this wave (wave-uniform), all of slot `cur`
  SlotView sv;
  sv.nm = sv.n0 = sv.np = nullptr;
  sv.L = 1; sv.tm = sv.t = sv.rid = 0;
  LdsView lv;
  lv.dir = reinterpret_cast<const uint16_t *>(lds);
  lv.rec = lds;
  lv.dim_a = lv.dim_c = lv.nb = lv.b_lo = 0;
  for (uint32_t ti = tb; ti < te; ++ti) {
    const TileDev tile = a.tiles[ti];
    if (tile.slot != cur) {
      if (qn) drain_queue(queue, qn, lane, sv, p, a.tab, a.err);
      qn = 0;
      cur = tile.slot;
      const ImageDesc im = a.images[cur];
      __syncthreads();  // previous image no longer in use
      const uint4 *src = reinterpret_cast<const uint4 *>(a.image_pool + im.off);
      for (uint32_t i = threadIdx.x; i < im.bytes / 16u; i += blockDim.x) lds[i] = src[i];
      __syncthreads();
      lv.dim_a = im.bytes ? im.dim_a : 0u;
      lv.dim_c = im.dim_c;
      lv.b_lo = im.b_lo;
      lv.nb = im.nb;
      lv.rec = lds + im.dir_bytes / 16u;
      const SlotDev sl = a.slots[cur];
      sv.t = a.tslot[cur];
      sv.L = sl.L;
      sv.tm = p.no_stream ? 0u : sv.t % sl.L;
      sv.rid = sl.rid;
      sv.nm = a.state + sl.off;
      sv.n0 = sv.nm + sl.stride;
      sv.np = sv.n0 + sl.stride;
    } else if (qn > kQueue - 64u) {
      drain_queue(queue, qn, lane, sv, p, a.tab, a.err);
      qn = 0;
    }
    const uint32_t L = sv.L, tm = sv.tm, t = sv.t;
    uint16_t *const nm = sv.nm;
    uint16_t *const n0 = sv.n0;
    uint16_t *const np = sv.np;

    // ---- load ----
    uint32_t va[G][4], vb[G][4], vc[G][4];
    uint32_t xs[G], sm[G], sp[G];
    bool fast[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      xs[g] = tile.x0 + ((uint32_t)g * nwaves + wave) * 512u;
      sm[g] = xs[g] + tm;
      sm[g] -= (sm[g] >= L) ? L : 0u;
      sp[g] = xs[g] >= tm ? xs[g] - tm : xs[g] + L - tm;
      fast[g] = (xs[g] + 512u <= L) & (sm[g] + 512u <= L) & (sp[g] + 512u <= L);
      if (fast[g]) {
        load_window(nm, sm[g], lane, va[g]);
        load4(n0 + xs[g] + 8u * lane, vb[g]);
        load_window(np, sp[g], lane, vc[g]);
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t x = xs[g] + 8u * lane + k;
          uint32_t ea = 0, eb = 0, ec = 0;
          if (x < L) {
            uint32_t pm = x + tm;
            pm -= (pm >= L) ? L : 0u;
            const uint32_t pp = x >= tm ? x - tm : x + L - tm;
            ea = nm[pm]; eb = n0[x]; ec = np[pp];
          }
          set16(va[g], k, ea); set16(vb[g], k, eb); set16(vc[g], k, ec);
        }
      }
    }

    // ---- collide: LDS image first, the rest into the wave's queue ----
#pragma unroll
    for (int g = 0; g < G; ++g) {
      ChunkCtx cx;
      cx.x8 = xs[g] + 8u * lane;
      cx.w0 = philox10(make_uint4(cx.x8 >> 2, t, sv.rid, 0u), key);
      cx.w1 = philox10(make_uint4((cx.x8 >> 2) + 1u, t, sv.rid, 0u), key);
      cx.L = L;
      cx.qn = qn;
      decide_site<0>(cx, fast[g], va[g], vb[g], vc[g], lv, queue, p, a.tab, t, sv.rid, a.err);
      decide_site<1>(cx, fast[g], va[g], vb[g], vc[g], lv, queue, p, a.tab, t, sv.rid, a.err);
      decide_site<2>(cx, fast[g], va[g], vb[g], vc[g], lv, queue, p, a.tab, t, sv.rid, a.err);
      decide_site<3>(cx, fast[g], va[g], vb[g], vc[g], lv, queue, p, a.tab, t, sv.rid, a.err);
      decide_site<4>(cx, fast[g], va[g], vb[g], vc[g], lv, queue, p, a.tab, t, sv.rid, a.err);
      decide_site<5>(cx, fast[g], va[g], vb[g], vc[g], lv, queue, p, a.tab, t, sv.rid, a.err);
      decide_site<6>(cx, fast[g], va[g], vb[g], vc[g], lv, queue, p, a.tab, t, sv.rid, a.err);
      decide_site<7>(cx, fast[g], va[g], vb[g], vc[g], lv, queue, p, a.tab, t, sv.rid, a.err);
      qn = cx.qn;
    }

    // ---- store ----
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (fast[g]) {
        store_window(nm, sm[g], lane, va[g]);
        store4(n0 + xs[g] + 8u * lane, vb[g]);
        store_window(np, sp[g], lane, vc[g]);
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t x = xs[g] + 8u * lane + k;
          if (x < L) {
            uint32_t pm = x + tm;
            pm -= (pm >= L) ? L : 0u;
            const uint32_t pp = x >= tm ? x - tm : x + L - tm;
            nm[pm] = (uint16_t)get16(va[g], k);
            n0[x] = (uint16_t)get16(vb[g], k);
            np[pp] = (uint16_t)get16(vc[g], k);
          }
        }
      }
    }
  }
  if (qn) drain_queue(queue, qn, lane, sv, p, a.tab, a.err);
  // The last block of the launch advances t of every slot in the launch.
  // Every block has consumed its loads of t before it takes its ticket (the
  // values shaped its work), so nothing reads the new value during this
  // launch; the next launch sees it through the kernel boundary.
  __shared__ uint32_t last;
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(a.ticket, 1u) == gridDim.x - 1u;
  __syncthreads();
  if (last) {
    for (uint32_t i = threadIdx.x; i < a.n_slots; i += blockDim.x) {
      const uint32_t s = a.slot_list ? a.slot_list[i] : a.slot_first + i;
      a.tslot[s] += 1u;
    }
    if (threadIdx.x == 0) atomicExch(a.ticket, 0u);
  }
}

// n_i(x, 0) ~ Poisson(f_i^eq): one Philox call per site (counter (x, 0,
// replica, 1)), words 0, 1, 2 for i = -1, 0, +1, inverse CDF over the host's
// quantised thresholds.  t must be 0, so physical = logical order.
__global__ void __launch_bounds__(256) k_init_poisson(
    uint16_t *__restrict__ state, const SlotDev *__restrict__ slots,
    const TileDev *__restrict__ tiles, uint32_t tile_sites, const PoisDesc *__restrict__ desc,
    const uint32_t *__restrict__ pool, uint64_t seed, uint32_t *err) {
  const TileDev tile = tiles[blockIdx.x];
  const SlotDev sl = slots[tile.slot];
  const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
  const uint32_t end = min(sl.L, tile.x0 + tile_sites);
  for (uint32_t x = tile.x0 + threadIdx.x; x < end; x += blockDim.x) {
    const uint4 w = philox10(make_uint4(x, 0u, sl.rid, 1u), key);
#pragma unroll
    for (uint32_t i = 0; i < 3; ++i) {
      const PoisDesc d = desc[3u * tile.slot + i];
      const uint32_t n = d.k_first + count_le(pool + d.off, d.nthr, word_of(w, i));
      if (n > 65535u) atomicOr(err, kErrOverflow);
      state[sl.off + (uint64_t)i * sl.stride + x] = (uint16_t)n;
    }
  }
}

__global__ void __launch_bounds__(256) k_init_counts(uint16_t *__restrict__ state,
                                                     const SlotDev *__restrict__ slots,
                                                     const TileDev *__restrict__ tiles,
                                                     uint32_t tile_sites,
                                                     const uint16_t *__restrict__ counts) {
  const TileDev tile = tiles[blockIdx.x];
  const SlotDev sl = slots[tile.slot];
  const uint32_t end = min(sl.L, tile.x0 + tile_sites);
  const uint16_t *src = counts + 3ull * sl.dense;
  for (uint32_t x = tile.x0 + threadIdx.x; x < end; x += blockDim.x)
#pragma unroll
    for (uint32_t i = 0; i < 3; ++i)
      state[sl.off + (uint64_t)i * sl.stride + x] = src[(uint64_t)i * sl.L + x];
}

__global__ void k_zero(unsigned long long *p, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_set_t(uint32_t *tslot, const uint32_t *slot_list, uint32_t n, uint32_t value) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) tslot[slot_list[i]] = value;
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)v, m);
  const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m);
  return ((unsigned long long)hi << 32) | lo;
}

constexpr int kMomVals = 14 + 2 * 8;

// Exact integer sums of one tile (logical site order), reduced over the
// wave with shuffles, over the block in LDS, then one atomic per value.
__global__ void __launch_bounds__(256) k_moments(
    const uint16_t *__restrict__ state, const SlotDev *__restrict__ slots,
    const uint32_t *__restrict__ tslot, const TileDev *__restrict__ tiles, uint32_t tile_sites,
    uint32_t no_stream, const int32_t *__restrict__ twiddle, uint32_t n_modes,
    MomDev *__restrict__ out) {
  const TileDev tile = tiles[blockIdx.x];
  const SlotDev sl = slots[tile.slot];
  const uint32_t L = sl.L;
  const uint32_t tm = no_stream ? 0u : tslot[tile.slot] % L;
  const uint16_t *nm = state + sl.off;
  const uint16_t *n0 = nm + sl.stride;
  const uint16_t *np = n0 + sl.stride;
  const int32_t *tw = twiddle ? twiddle + 2ull * n_modes * sl.dense : nullptr;
  unsigned long long v[kMomVals];
#pragma unroll
  for (int i = 0; i < kMomVals; ++i) v[i] = 0ull;
  const uint32_t end = min(L, tile.x0 + tile_sites);
  for (uint32_t x = tile.x0 + threadIdx.x; x < end; x += blockDim.x) {
    uint32_t pm = x + tm;
    pm -= (pm >= L) ? L : 0u;
    const uint32_t pp = x >= tm ? x - tm : x + L - tm;
    const unsigned long long a = nm[pm], b = n0[x], c = np[pp];
    const unsigned long long N = a + b + c;
    v[0] += a; v[1] += b; v[2] += c;
    v[3] += a * a; v[4] += b * b; v[5] += c * c;
    v[6] += a * b; v[7] += b * c; v[8] += a * c;
    v[9] += N;
    v[10] += c - a;
    v[11] += N * N;
    v[12] += b & 1ull;
    v[13] = v[13] > N ? v[13] : N;
    for (uint32_t m = 0; m < n_modes; ++m) {
      v[14 + 2 * m] += N * (unsigned long long)(long long)tw[(2ull * m) * L + x];
      v[15 + 2 * m] += N * (unsigned long long)(long long)tw[(2ull * m + 1) * L + x];
    }
  }
  __shared__ unsigned long long red[16][kMomVals];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kMomVals; ++i) {
    unsigned long long x = v[i];
    for (int m = 32; m >= 1; m >>= 1) {
      const unsigned long long y = shfl_xor_u64(x, m);
      x = (i == 13) ? (x > y ? x : y) : x + y;
    }
    if (lane == 0) red[wave][i] = x;
  }
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  if (threadIdx.x < kMomVals) {
    const int i = threadIdx.x;
    unsigned long long s = 0ull;
    for (int w = 0; w < nw; ++w) s = (i == 13) ? (s > red[w][i] ? s : red[w][i]) : s + red[w][i];
    if (i == 13) atomicMax(&out[tile.slot].v[13], s);
    else if (i < 14 + 2 * (int)n_modes) atomicAdd(&out[tile.slot].v[i], s);
  }
}

}  // namespace

template <int G>
static hipError_t occupancy_of(uint32_t threads, uint32_t lds, int &blocks) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_step<G>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_step<G>, (int)threads, lds);
}

uint32_t step_lds_bytes(const Schedule &sch, uint32_t image_bytes) {
  return (image_bytes + 15u) / 16u * 16u + (sch.threads / 64u) * kQueueBytesPerWave;
}

hipError_t step_occupancy(const Schedule &sch, uint32_t lds_bytes, uint32_t n_cu,
                          uint32_t &max_blocks) {
  int b = 0;
  hipError_t e;
  const uint32_t lds = step_lds_bytes(sch, lds_bytes);
  switch (sch.groups) {
    case 1: e = occupancy_of<1>(sch.threads, lds, b); break;
    case 2: e = occupancy_of<2>(sch.threads, lds, b); break;
    case 4: e = occupancy_of<4>(sch.threads, lds, b); break;
    default: return hipErrorInvalidValue;
  }
  if (e) return e;
  if (b < 1) return hipErrorInvalidConfiguration;
  max_blocks = (uint32_t)b * n_cu;
  return hipSuccess;
}

hipError_t launch_step(const Schedule &sch, hipStream_t s, const StepLaunch &a) {
  if (a.n_tiles == 0) return hipSuccess;
  dim3 grid(std::max<uint32_t>(1, std::min(a.n_tiles, a.max_blocks))), block(sch.threads);
  const uint32_t lds = step_lds_bytes(sch, a.lds_bytes);
  switch (sch.groups) {
    case 1: k_step<1><<<grid, block, lds, s>>>(a); break;
    case 2: k_step<2><<<grid, block, lds, s>>>(a); break;
    case 4: k_step<4><<<grid, block, lds, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_init_poisson(hipStream_t s, uint16_t *state, const SlotDev *slots,
                               const uint32_t *, const TileDev *tiles, uint32_t n_tiles,
                               uint32_t tile_sites, const PoisDesc *desc, const uint32_t *pool,
                               uint64_t seed, uint32_t *err) {
  if (n_tiles == 0) return hipSuccess;
  k_init_poisson<<<n_tiles, 256, 0, s>>>(state, slots, tiles, tile_sites, desc, pool, seed, err);
  return hipGetLastError();
}

hipError_t launch_init_counts(hipStream_t s, uint16_t *state, const SlotDev *slots,
                              const TileDev *tiles, uint32_t n_tiles, uint32_t tile_sites,
                              const uint16_t *counts) {
  if (n_tiles == 0) return hipSuccess;
  k_init_counts<<<n_tiles, 256, 0, s>>>(state, slots, tiles, tile_sites, counts);
  return hipGetLastError();
}

hipError_t launch_zero(hipStream_t s, unsigned long long *p, uint64_t n) {
  if (n == 0) return hipSuccess;
  uint32_t blocks = (uint32_t)std::min<uint64_t>((n + 255) / 256, 1024);
  k_zero<<<blocks, 256, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_moments(hipStream_t s, const uint16_t *state, const SlotDev *slots,
                          const uint32_t *tslot, const TileDev *tiles, uint32_t n_tiles,
                          uint32_t tile_sites, uint32_t no_stream, const int32_t *twiddle,
                          uint32_t n_modes, MomDev *out) {
  if (n_tiles == 0) return hipSuccess;
  k_moments<<<n_tiles, 256, 0, s>>>(state, slots, tslot, tiles, tile_sites, no_stream, twiddle,
                                    n_modes, out);
  return hipGetLastError();
}

hipError_t launch_set_t(hipStream_t s, uint32_t *tslot, const uint32_t *slot_list, uint32_t n,
                        uint32_t value) {
  if (n == 0) return hipSuccess;
  k_set_t<<<1, 256, 0, s>>>(tslot, slot_list, n, value);
  return hipGetLastError();
}

}  // namespace mclg
