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
#include "mom3_sum.h"
#include "rng.h"


#include <algorithm>

namespace mclg {
namespace {

// Galilean-invariant acceptance of fiber (N, |J|) as a numerator over 2^32:
// floor(g num / den) with g = floor(2^32 N / sqrt(N^2 + 3 J^2)), both exact:
// each is estimated in double and corrected by integer tests that use only
// products (g is the largest integer with g^2 (N^2 + 3 J^2) <= 2^64 N^2).
__device__ uint64_t galilean_lambda(uint32_t num, uint32_t den, uint32_t N, uint32_t absJ) {
  using u128 = unsigned __int128;
  uint64_t g = 1ull << 32;
  if (absJ) {
    const uint64_t n2 = (uint64_t)N * N, d = n2 + 3ull * absJ * absJ;
    const u128 bound = (u128)n2 << 64;
    uint64_t s = (uint64_t)(4294967296.0 * (double)N / __dsqrt_rn((double)d));
    while (s && (u128)s * s * d > bound) --s;
    while ((u128)(s + 1) * (s + 1) * d <= bound) ++s;
    g = s;
  }
  const uint64_t gn = g * num;  // < 2^61
  uint64_t q = (uint64_t)((double)gn / (double)den);
  while (q && (u128)q * den > gn) --q;
  while ((u128)(q + 1) * den <= gn) ++q;
  return q;
}

// The paper's C sub-collisions one by one (Eq. (select), Eq. (omega)); used
// for sites with N > n_max.  Returns the new rest count.  GAL selects the
// Galilean-invariant acceptance (its own kernel instantiation, so that the
// plain kernel carries none of its code).
template <bool GAL>
__device__ __forceinline__ uint32_t collide_direct(uint32_t a, uint32_t b, uint32_t c,
                                                const StepParams &p, uint32_t x, uint32_t t,
                                                uint32_t rid) {
  WordStream ws;
  ws.key = make_uint2((uint32_t)p.seed, (uint32_t)(p.seed >> 32));
  ws.x = x; ws.t = t; ws.rid = rid; ws.block = 0; ws.used = 4;
  const uint32_t N = a + b + c;
  if constexpr (GAL) {
    // lambda = lq / 2^32: a {-1,+1} pair is accepted when a word is below lq,
    // a {0,0} pair (lambda / 8) when a 35-bit uniform (w1 * 8 + w2 >> 29) is.
    const uint64_t lq = galilean_lambda(p.lam_p, p.lam_q, N, c > a ? c - a : a - c);
    for (int32_t s = 0; s < p.C; ++s) {
      const uint32_t r1 = ws.uniform(N);
      uint32_t r2 = ws.uniform(N - 1);
      r2 += (r2 >= r1);
      const int v1 = r1 < a ? -1 : (r1 < a + b ? 0 : 1);
      const int v2 = r2 < a ? -1 : (r2 < a + b ? 0 : 1);
      if (v1 + v2 == 0 && v1 != 0) {
        if ((uint64_t)ws.next() < lq) { a -= 1; c -= 1; b += 2; }
      } else if (v1 == 0 && v2 == 0) {
        const uint64_t w1 = ws.next();
        const uint32_t w2 = ws.next();
        if (((w1 << 3) | (w2 >> 29)) < lq) { b -= 2; a += 1; c += 1; }
      }
    }
    return b;
  }
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

// Index of the first row of fiber (N, |J|) in the global tables, in closed
// form: fibers are stored by N, then |J|, and fiber (N, j) holds
// floor((N - j) / 2) + 1 rows, so with S(M) = M + 1 + floor(M^2 / 4) rows in
// the fibers (M, 0..M) and T(K) = sum_{M <= K} floor(M^2 / 4), the base is
// N (N + 1) / 2 + T(N - 1) + S(N) - S(N - j).  (Saves a dependent load.)
__device__ __forceinline__ uint32_t fiber_base(uint32_t N, uint32_t absJ) {
  auto S = [](uint32_t M) { return M + 1u + ((M * M) >> 2); };
  uint32_t T = 0;
  if (N >= 1u) {
    const uint32_t K = N - 1u, i = K >> 1;
    T = (K & 1u) ? i * (i + 1u) * (4u * i + 5u) / 6u : i * (i + 1u) * (4u * i - 1u) / 6u;
  }
  return ((N * (N + 1u)) >> 1) + T + S(N) - S(N - absJ);
}

// Number of entries <= r of an ascending array of n values: probe seven
// evenly spaced pivots at once, then count the one bucket left (all its
// loads at once) -- two rounds of independent loads for n <= 64.
__device__ __forceinline__ uint32_t count_le_wide(const uint32_t *__restrict__ t, uint32_t n,
                                                  uint32_t r) {
  uint32_t lo = 0;
  while (n > 8u) {
    const uint32_t s = (n + 7u) >> 3;  // bucket width; pivots t[lo + j s - 1]
    uint32_t c = 0;
#pragma unroll
    for (uint32_t j = 1; j < 8; ++j)
      c += (j * s <= n && t[lo + j * s - 1u] <= r) ? 1u : 0u;
    lo += c * s;
    n = min(s, n - c * s);
  }
  uint32_t c = 0;
#pragma unroll
  for (uint32_t j = 0; j < 8; ++j) c += (j < n && t[lo + j] <= r) ? 1u : 0u;
  return lo + c;
}

// Exact row of the global tables: the number of thresholds <= r.
// Rows of up to 16 thresholds (every row of C <= 7, most of larger C) are
// counted from four 16-byte loads issued together; the threshold pool is
// padded by 16 values so that these loads stay inside it.
__device__ __forceinline__ uint32_t count_le_16(const uint32_t *t, uint32_t n, uint32_t r) {
  uint4 q[4];
  for (int j = 0; j < 4; ++j) __builtin_memcpy(&q[j], t + 4 * j, 16);  // 4-byte aligned
  uint32_t c = 0;
#pragma unroll
  for (uint32_t j = 0; j < 16; ++j) {
    const uint4 &v = q[j >> 2];
    const uint32_t x = (j & 3) == 0 ? v.x : (j & 3) == 1 ? v.y : (j & 3) == 2 ? v.z : v.w;
    c += (j < n && x <= r) ? 1u : 0u;
  }
  return c;
}

// Two 16-bit lanes of a 32-bit register.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t global_outcome(const TableDev &tab, uint32_t N, uint32_t absJ,
                                                   uint32_t b, uint32_t par, uint32_t r) {
  const uint32_t row = fiber_base(N, absJ) + ((b - par) >> 1);  // states ascend in n0
  if (tab.row16) {
    // one 64-byte row of 16-bit values: k_first, q, the thresholds' top 16
    // bits (0xFFFF padding); the outcome is k_first + #{t < rh} unless some
    // t equals rh, when only the full 32-bit threshold decides (the rows
    // below)
    const uint4 *q = tab.row16 + (size_t)row * (kRow16 / 8);
    const uint4 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
    const uint32_t w[16] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                            q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
    const uint32_t rr = (r >> 16) * 0x10001u;
    const u16x2 R = __builtin_bit_cast(u16x2, rr), one = {1, 1};
    u16x2 acc = {0, 0};
    uint32_t eq = 0;
#pragma unroll
    for (int j = 1; j < 16; ++j) {
      acc += __builtin_elementwise_min(__builtin_elementwise_sub_sat(R, __builtin_bit_cast(u16x2, w[j])),
                                       one);
      const uint32_t x = w[j] ^ rr;  // a zero half: that threshold's top bits equal rh
      eq |= (x - 0x00010001u) & ~x & 0x80008000u;
    }
    if (eq == 0u) return (w[0] & 0xffffu) + (uint32_t)acc.x + (uint32_t)acc.y;
  }
  if (tab.fixed) {
    // header and up to 19 thresholds, all five 16-byte pieces at once
    const uint4 *q = tab.fixed + (size_t)row * (kFixedStride / 4);
    const uint4 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4];
    const uint32_t w[20] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y,
                            q2.z, q2.w, q3.x, q3.y, q3.z, q3.w, q4.x, q4.y, q4.z, q4.w};
    const uint32_t n = (w[0] >> 16) - 1u;
    uint32_t c = 0;
#pragma unroll
    for (uint32_t j = 0; j < kFixedStride - 1; ++j) c += (j < n && w[1 + j] <= r) ? 1u : 0u;
    return (w[0] & 0xffffu) + c;
  }
  const uint2 d = tab.rowdesc[row];
  const uint32_t n = (d.y >> 16) - 1u;
  return (d.y & 0xffffu) +
         (n <= 16u ? count_le_16(tab.thr + d.x, n, r) : count_le_wide(tab.thr + d.x, n, r));
}

// The slot's collision image in LDS: a directory of (min(a,c), max(a,c))
// pairs whose last row and column stand for every pair out of range, then
// 16-byte records, nb + 1 per pair (the last one for every b out of range).
// A record decides the outcome exactly whenever the top 16 bits of r lie in
// its window and differ from every inner value.
// The image sits at LDS address 0 (the step kernel has no static LDS, so its
// dynamic LDS starts there) and is read by byte address.
struct LdsView {
  // dim_a, dim_c, dim_c + 1, b_lo and nb, each in both 16-bit halves
  uint32_t da2, dc2, w2, blo2, nb2;
};
typedef __attribute__((address_space(3))) const uint16_t lds_c16;
typedef uint32_t lds_v4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const lds_v4 lds_c4;
__device__ __forceinline__ uint16_t lds_u16(uint32_t addr) {
  return *(lds_c16 *)(size_t)addr;
}
__device__ __forceinline__ uint4 lds_u4(uint32_t addr) {
  const lds_v4 v = *(lds_c4 *)(size_t)addr;
  return make_uint4(v[0], v[1], v[2], v[3]);
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
// A slot's three arrays through one buffer resource: byte address =
// voff (per lane) + soff (wave-uniform, a scalar register).  Offsets stay
// 32-bit, and the per-lane part of a chunk's vector accesses is the same
// 16 * lane for every window.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9)
// CP: the cache policy bits of the access (0, or kStreamingPolicy for
// states that do not fit the caches: non-temporal, the lines are not
// expected to be reused before they leave).
constexpr int kStreamingPolicy = 2;  // nt
// sc1: coherent across the device's L2s (data another block reads in the
// same launch)
constexpr int kDevicePolicy = 16;
template <int CP = 0>
__device__ __forceinline__ void bload4(Rsrc r, uint32_t voff, uint32_t soff, uint32_t (&v)[4]) {
  const auto q = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, CP);
  v[0] = q[0]; v[1] = q[1]; v[2] = q[2]; v[3] = q[3];
}
template <int CP = 0>
__device__ __forceinline__ void bstore4(Rsrc r, uint32_t voff, uint32_t soff,
                                        const uint32_t (&v)[4]) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 q = {v[0], v[1], v[2], v[3]};
  __builtin_amdgcn_raw_buffer_store_b128(q, r, (int)voff, (int)soff, CP);
}
__device__ __forceinline__ uint32_t bload2(Rsrc r, uint32_t voff, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore2(Rsrc r, uint32_t voff, uint32_t soff, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Per-wave queue of draws the LDS image could not decide (or sites with
// N > n_max); drained by all lanes at once.
constexpr uint32_t kOverflow = kOverflowPerWave;

// Exact outcome for a queued site: global row, or the literal loop.  It is
// only reached from the drain, outside the unrolled per-site code, so the
// hot loop stays small enough for the instruction cache.
template <bool GAL>
__device__ __forceinline__ uint32_t resolve_queued(const uint4 e, const StepParams &p,
                                                const TableDev &tab, uint32_t t, uint32_t rid,
                                                uint32_t *err) {
  const uint32_t x = e.x, a = e.y & 0xffffu, b = e.y >> 16, c = e.z, r = e.w;
  const uint32_t N = a + b + c;
  if (N > 65535u) {  // a post-collision count might not fit: flagged, kept
    atomicOr(err, kErrOverflow);
    return b;
  }
  if (p.C == 0 || N < 2u) return b;  // no collision
  if (N <= p.n_max) {
    const uint32_t absJ = (uint32_t)abs((int32_t)c - (int32_t)a);
    const uint32_t par = (N - absJ) & 1u;
    return par + 2u * global_outcome(tab, N, absJ, b, par, r);
  }
  if (p.C < 0) {
    atomicOr(err, kErrEqRange);
    return b;
  }
  return collide_direct<GAL>(a, b, c, p, x, t, rid);
}

// Where a slot's three arrays are and how they are shifted at step t.
struct SlotView {
  uint32_t lo, hi;  // address of the slot's n_-1 array; n_0 and n_+1 follow
  uint32_t ab;      // bytes per array
  uint32_t L, tm, t, rid;
  // Site x of the view is site (x + xoff) mod lg of the lattice, which keys
  // its random numbers: xoff = 0 and lg = L for a slot itself, the region's
  // first site and the lattice's size for a block's copy of a region (a
  // multiple of 8 each, so that a lane's eight sites never wrap).
  uint32_t xoff, lg;
  template <bool TB>
  __device__ __forceinline__ uint32_t logical(uint32_t x) const {
    if constexpr (!TB) return x;
    const uint32_t y = x + xoff;
    return y >= lg ? y - lg : y;
  }
  // the buffer resource, rebuilt at each use from wave-uniform scalars
  __device__ __forceinline__ Rsrc rs() const {
    return __builtin_amdgcn_make_buffer_rsrc(
        reinterpret_cast<void *>(((uint64_t)hi << 32) | lo), 0, (int)(3u * ab), kRsrcWord3);
  }
};

// Decision of one site from the LDS image, in three phases so that the LDS
// reads of several sites are in flight together: (1) directory read, (2)
// record read, (3) decision.  There is no branch and no range test per site:
// the directory clamps min(a, c) to dim_a and max(a, c) to dim_c, whose row
// and column lead to never records, and b - b_lo (mod 2^16) is clamped to nb,
// every pair's never record.  A site outside the image (or of an absent
// pair, or with N > n_max) thus reads a never record, a site with N < 2 a
// record of move 0, and a site whose N does not fit 16 bits lies outside
// (the image holds N < 3072 only).  A record holds (b >> 1) - k_s, a lower
// bound L, inner values t2..t6 and an upper bound U (top 16 bits of seven
// consecutive thresholds of the site's fiber row, L rounded up); with the
// top half rh of the draw in [L, U) and equal to none of t2..t6 the drawn
// state index is k_s + #{t2..t6 < rh}, and the move of Eq. (collcons) is
// d = (b - b') / 2 = (b >> 1) - k_s - #{t2..t6 < rh}  (b' has b's parity).
struct SiteLook {
  uint4 q;
};

// Phase 1 of sites 2J and 2J + 1 with 16-bit packed arithmetic.
template <int J>
__device__ __forceinline__ void site_dir_pair(uint32_t &row0, uint32_t &row1, u16x2 &bis,
                                              const uint32_t (&va)[4],
                                              const uint32_t (&vb)[4], const uint32_t (&vc)[4],
                                              const LdsView &lv) {
  const u16x2 a = __builtin_bit_cast(u16x2, va[J]), b = __builtin_bit_cast(u16x2, vb[J]),
              c = __builtin_bit_cast(u16x2, vc[J]);
  const u16x2 lo = __builtin_elementwise_min(__builtin_elementwise_min(a, c),
                                             __builtin_bit_cast(u16x2, lv.da2));
  const u16x2 hi = __builtin_elementwise_min(__builtin_elementwise_max(a, c),
                                             __builtin_bit_cast(u16x2, lv.dc2));
  const uint32_t slot = __builtin_bit_cast(uint32_t, lo * __builtin_bit_cast(u16x2, lv.w2) + hi);
  const uint32_t bi = __builtin_bit_cast(
      uint32_t, __builtin_elementwise_min(b - __builtin_bit_cast(u16x2, lv.blo2),
                                          __builtin_bit_cast(u16x2, lv.nb2)));
  const uint32_t off = __builtin_bit_cast(uint32_t, slot + slot);  // byte offsets
  row0 = lds_u16(off & 0xffffu);
  row1 = lds_u16(off >> 16);
  bis = __builtin_bit_cast(u16x2, bi);
}

// Phase 2 of sites 2J and 2J + 1: record indices add in 16-bit lanes.
__device__ __forceinline__ void rec_pair(SiteLook &s0, SiteLook &s1, uint32_t row0, uint32_t row1,
                                         u16x2 bis) {
  const u16x2 rows = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(row1, row0, 0x05040100u));
  const uint32_t idx = __builtin_bit_cast(uint32_t, rows + bis);
  s0.q = lds_u4((idx & 0xffffu) << 4);
  s1.q = lds_u4((idx >> 16) << 4);
}

// Phase 3: whether the record decides the draw, and d in the low 16 bits
// (meaningless when it does not).
__device__ __forceinline__ uint32_t site_finish(const SiteLook &s, uint32_t r, bool &hit) {
  const uint4 q = s.q;
  const uint32_t rh = r >> 16;
  const uint32_t lb = q.x >> 16, t2 = q.y & 0xffffu, t3 = q.y >> 16, t4 = q.z & 0xffffu,
                 t5 = q.z >> 16, t6 = q.w & 0xffffu, ub = q.w >> 16;
  hit = (rh >= lb) & (rh < ub) & (rh != t2) & (rh != t3) & (rh != t4) & (rh != t5) & (rh != t6);
  return q.x - (uint32_t)(t2 < rh) - (uint32_t)(t3 < rh) - (uint32_t)(t4 < rh) -
         (uint32_t)(t5 < rh) - (uint32_t)(t6 < rh);
}

// The wave's queue of undecided draws: a virtual array of kQueue entries in
// LDS followed by kOverflow entries in global memory, filled to F
// (wave-uniform).  An entry is (x, a | b << 16, c, r) with the site's
// pre-collision counts; the chunk stores whatever its lane computed for such
// a site, and the drain overwrites it with the exact outcome.  When the
// chunk's draws are resolved before its store (kDrainPatch), the first word
// is instead the site's position in the chunk, 8 lane + K.
static_assert(kDrainAt + 512 <= kQueue + kOverflow, "a chunk's draws must fit the queue");

// Site K of every lane whose draw was not decided (and, in a chunk that
// passes the end of the lattice, that exists) goes to the queue, in lane
// order.  wa, wb, wc are the words holding the site's pre-collision counts;
// `slow` is wave-uniform.
template <int K, bool PATCH>
__device__ __forceinline__ void push_site(uint4 *queue, Rsrc over, uint32_t &F, bool hit,
                                          bool slow, uint32_t x8, uint32_t L, uint32_t wa,
                                          uint32_t wb, uint32_t wc, uint32_t r, uint32_t xs) {
  uint64_t mk = __ballot(!hit);
  if (mk == 0) return;
  if (slow) mk &= __builtin_amdgcn_uicmpl(x8 + K, L, 36);  // lanes with x8 + K < L
  const uint32_t n = (uint32_t)__popcll(mk);
  if (!hit && (!slow || x8 + K < L)) {
    const uint32_t pos = F + lanes_below(mk);
    const uint32_t ab = (K & 1) ? __builtin_amdgcn_perm(wb, wa, 0x07060302u)
                                : __builtin_amdgcn_perm(wb, wa, 0x05040100u);
    const uint32_t c = (K & 1) ? wc >> 16 : wc & 0xffffu;
    uint32_t w0 = x8 + K;
    if constexpr (PATCH) {
      // the position in the chunk (xs: its first site), computed here rather
      // than hoisted out of the chunk loop as a per-lane constant
      w0 -= xs;
      asm volatile("" : "+v"(w0));
    }
    if (pos < kQueue) {
      queue[pos] = make_uint4(w0, ab, c, r);
    } else {
      typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
      const u32x4 e = {w0, ab, c, r};
      __builtin_amdgcn_raw_buffer_store_b128(e, over, (int)(16u * (pos - kQueue)), 0, 0);
    }
  }
  F += n;
}

// Phase 3 of sites 2J and 2J + 1: d of both in one word (16-bit lanes) and
// whether each was decided.
__device__ __forceinline__ uint32_t finish_pair(const SiteLook &s0, const SiteLook &s1,
                                                uint32_t r0, uint32_t r1, bool &h0, bool &h1) {
  const uint32_t d0 = site_finish(s0, r0, h0), d1 = site_finish(s1, r1, h1);
  return __builtin_amdgcn_perm(d1, d0, 0x05040100u);
}
// Sites 2J and 2J + 1 move by d: n_-1 and n_+1 gain d, n_0 loses 2d.
__device__ __forceinline__ void apply_pair(uint32_t &a, uint32_t &b, uint32_t &c, uint32_t dp) {
  const u16x2 d = __builtin_bit_cast(u16x2, dp);
  a = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + d);
  c = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, c) + d);
  b = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, b) - (d + d));
}

// All eight sites of the lane: directory reads of all eight first, the
// Philox draws while they are in flight, then record reads and decisions;
// the undecided draws are queued with the pre-collision counts before the
// update.
template <bool PATCH>
__device__ __forceinline__ void decide_eight(uint4 &w0, uint4 &w1, uint2 key,
                                             uint32_t (&va)[4], uint32_t (&vb)[4],
                                             uint32_t (&vc)[4], const LdsView &lv, uint4 *queue,
                                             Rsrc over, uint32_t &F, bool slow, uint32_t x8,
                                             uint32_t L, uint32_t xs) {
  SiteLook s0, s1, s2, s3, s4, s5, s6, s7;
  uint32_t r0, r1, r2, r3, r4, r5, r6, r7;  // each site's first record
  u16x2 b01, b23, b45, b67;                  // clamped b - b_lo of each pair
  site_dir_pair<0>(r0, r1, b01, va, vb, vc, lv);
  site_dir_pair<1>(r2, r3, b23, va, vb, vc, lv);
  site_dir_pair<2>(r4, r5, b45, va, vb, vc, lv);
  site_dir_pair<3>(r6, r7, b67, va, vb, vc, lv);
  philox10_x2(w0, w1, key);
  rec_pair(s0, s1, r0, r1, b01);
  rec_pair(s2, s3, r2, r3, b23);
  rec_pair(s4, s5, r4, r5, b45);
  rec_pair(s6, s7, r6, r7, b67);
  bool h0, h1, h2, h3, h4, h5, h6, h7;
  const uint32_t d01 = finish_pair(s0, s1, w0.x, w0.y, h0, h1);
  const uint32_t d23 = finish_pair(s2, s3, w0.z, w0.w, h2, h3);
  const uint32_t d45 = finish_pair(s4, s5, w1.x, w1.y, h4, h5);
  const uint32_t d67 = finish_pair(s6, s7, w1.z, w1.w, h6, h7);
  uint32_t na[4] = {va[0], va[1], va[2], va[3]}, nb[4] = {vb[0], vb[1], vb[2], vb[3]},
           nc[4] = {vc[0], vc[1], vc[2], vc[3]};
  apply_pair(na[0], nb[0], nc[0], d01);
  apply_pair(na[1], nb[1], nc[1], d23);
  apply_pair(na[2], nb[2], nc[2], d45);
  apply_pair(na[3], nb[3], nc[3], d67);
#define MCLG_PUSH(K, H, R)                                                                \
  push_site<K, PATCH>(queue, over, F, H, slow, x8, L, va[K >> 1], vb[K >> 1], vc[K >> 1], R, \
                      xs)
  MCLG_PUSH(0, h0, w0.x); MCLG_PUSH(1, h1, w0.y); MCLG_PUSH(2, h2, w0.z); MCLG_PUSH(3, h3, w0.w);
  MCLG_PUSH(4, h4, w1.x); MCLG_PUSH(5, h5, w1.y); MCLG_PUSH(6, h6, w1.z); MCLG_PUSH(7, h7, w1.w);
#undef MCLG_PUSH
  for (int j = 0; j < 4; ++j) {
    va[j] = na[j];
    vb[j] = nb[j];
    vc[j] = nc[j];
  }
}

// Without collisions only a site whose N does not fit 16 bits is queued
// (the drain flags it and keeps its counts).
template <bool PATCH>
__device__ __forceinline__ void queue_saturated(const uint32_t (&va)[4], const uint32_t (&vb)[4],
                                                const uint32_t (&vc)[4], uint4 *queue,
                                                Rsrc over, uint32_t &F, bool slow,
                                                uint32_t x8, uint32_t L, uint32_t xs) {
#define MCLG_SAT(J)                                                                              \
  {                                                                                              \
    const uint32_t N2 = __builtin_bit_cast(                                                      \
        uint32_t, __builtin_elementwise_add_sat(                                                 \
                      __builtin_elementwise_add_sat(__builtin_bit_cast(u16x2, va[J]),            \
                                                    __builtin_bit_cast(u16x2, vb[J])),           \
                      __builtin_bit_cast(u16x2, vc[J])));                                        \
    push_site<2 * J, PATCH>(queue, over, F, (N2 & 0xffffu) != 0xffffu, slow, x8, L, va[J],      \
                            vb[J], vc[J], 0u, xs);                                               \
    push_site<2 * J + 1, PATCH>(queue, over, F, (N2 >> 16) != 0xffffu, slow, x8, L, va[J],      \
                                vb[J], vc[J], 0u, xs);                                           \
  }
  MCLG_SAT(0) MCLG_SAT(1) MCLG_SAT(2) MCLG_SAT(3)
#undef MCLG_SAT
}

// Resolve every queued draw of the wave (all lanes in parallel) and store
// the site's three final counts.  The wave first waits until all of its
// earlier memory operations have completed -- among them the stores that
// wrote the pre-collision counts of these sites -- so the final counts land
// after them.
template <bool GAL, bool TB = false>
__device__ __forceinline__ void drain_queue(const uint4 *queue, const uint4 *over, uint32_t F,
                                            uint32_t lane, const SlotView &v,
                                            const StepParams &p, const TableDev &tab,
                                            uint32_t *err) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0);  // vmcnt = expcnt = lgkmcnt = 0
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  for (uint32_t i = lane; i < F; i += 64u) {
    const uint4 e = i < kQueue ? queue[i] : over[i - kQueue];
    const uint32_t x = e.x, ea = e.y & 0xffffu, eb = e.y >> 16, ec = e.z;
    const uint32_t bn =
        resolve_queued<GAL>(make_uint4(v.logical<TB>(x), e.y, e.z, e.w), p, tab, v.t, v.rid, err);
    const int32_t N = (int32_t)(ea + eb + ec), J = (int32_t)ec - (int32_t)ea;
    uint32_t pm = x + v.tm;
    pm -= (pm >= v.L) ? v.L : 0u;
    const uint32_t pp = x >= v.tm ? x - v.tm : x + v.L - v.tm;
    bstore2(v.rs(), 2u * pm, 0u, (uint32_t)((N - (int32_t)bn - J) >> 1));
    bstore2(v.rs(), 2u * x, v.ab, bn);
    bstore2(v.rs(), 2u * pp, 2u * v.ab, (uint32_t)((N - (int32_t)bn + J) >> 1));
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// The move decide_eight applied to one undecided site (a, b, c; draw r):
// the same directory and record reads from the LDS image, one site in
// 32-bit arithmetic with the 16-bit wrap-around of the packed form.
__device__ __forceinline__ uint32_t image_move(uint32_t a, uint32_t b, uint32_t c, uint32_t r,
                                               const LdsView &lv) {
  const uint32_t lo = min(min(a, c), lv.da2 & 0xffffu), hi = min(max(a, c), lv.dc2 & 0xffffu);
  const uint32_t slot = (lo * (lv.w2 & 0xffffu) + hi) & 0xffffu;
  const uint32_t row = lds_u16((2u * slot) & 0xffffu);
  const uint32_t bi = min((b - (lv.blo2 & 0xffffu)) & 0xffffu, lv.nb2 & 0xffffu);
  SiteLook sl;
  sl.q = lds_u4(((row + bi) & 0xffffu) << 4);
  bool hit;
  return site_finish(sl, r, hit) & 0xffffu;
}

// Resolve the draws queued by the current chunk before its store
// (kDrainPatch): each lane takes one entry at a time, finds the exact outcome
// and writes the correction of the move the site's lane applied (found again
// from the image), as a 16-bit patch at the site's position; the LDS queue's
// 1 KB holds the chunk's 512 patches once its entries have been read.  Every
// lane then adds its eight patches to its counts (zero for decided sites), so
// the chunk's vector stores write the final counts.
template <bool GAL, bool TB = false>
__device__ __forceinline__ void patch_chunk(uint4 *queue, const uint4 *over, uint32_t F,
                                            uint32_t lane, uint32_t xs, const SlotView &v,
                                            const LdsView &lv, const StepParams &p,
                                            const TableDev &tab, uint32_t *err, uint32_t (&m)[4],
                                            uint32_t (&z)[4], uint32_t (&c)[4]) {
  if (F > kQueue) {
    // entries past the LDS queue were written to global memory by other
    // lanes: wait for those stores before reading them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  const uint4 e0 = lane < F ? queue[lane] : make_uint4(0u, 0u, 0u, 0u);
  // each lane clears its own 16 bytes (its eight sites' patches) after
  // reading the entry stored there
  queue[lane] = make_uint4(0u, 0u, 0u, 0u);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint16_t *const patch = reinterpret_cast<uint16_t *>(queue);
  for (uint32_t i = lane; i < F; i += 64u) {
    uint4 e = i < kQueue ? e0 : over[i - kQueue];
    const uint32_t pos = e.x, b = e.y >> 16;
    // C = 0 queues only overflowing sites and applies no move
    const uint32_t dw = p.C != 0 ? image_move(e.y & 0xffffu, b, e.z, e.w, lv) : 0u;
    e.x = v.logical<TB>(xs + pos);
    const uint32_t bn = resolve_queued<GAL>(e, p, tab, v.t, v.rid, err);
    const uint32_t d = (uint32_t)(((int32_t)b - (int32_t)bn) >> 1);
    patch[pos] = (uint16_t)(d - dw);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint4 pv = queue[lane];
  apply_pair(m[0], z[0], c[0], pv.x);
  apply_pair(m[1], z[1], c[1], pv.y);
  apply_pair(m[2], z[2], c[2], pv.z);
  apply_pair(m[3], z[3], c[3], pv.w);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Streaming over a wave's run of consecutive chunks
// ---------------------------------------------------------------------------
// Where chunk xs .. xs + 511 of a slot lies at step t: the three physical
// windows (n_-1 at (x + t) mod L, n_0 at x, n_+1 at (x - t) mod L) and
// whether none of them wraps around the end of the lattice (fast path).
struct Win {
  uint32_t xs, sm, sp;
  uint32_t fast;  // 0 or 1
};
__device__ __forceinline__ Win locate(uint32_t xs, const SlotView &v) {
  Win w;
  w.xs = xs;
  w.sm = xs + v.tm;
  w.sm -= (w.sm >= v.L) ? v.L : 0u;
  w.sp = xs >= v.tm ? xs - v.tm : xs + v.L - v.tm;
  w.fast = (uint32_t)((xs + 512u <= v.L) & (w.sm + 512u <= v.L) & (w.sp + 512u <= v.L));
  return w;
}
// A fast chunk's three windows, one 16-byte access per lane each: lane i
// owns elements s + 8 i .. s + 8 i + 7 of every window.  The n_+-1 windows
// start at any element (2-byte alignment); the hardware serves unaligned
// vector accesses, and neighbouring lanes, chunks and waves touch disjoint
// bytes, so each lane reads and writes exactly its own eight elements.
struct Raw {
  uint32_t m[4], z[4], p[4];
};
template <int CP>
__device__ __forceinline__ void issue_raw(const Win &w, const SlotView &v, uint32_t lane,
                                          Raw &r) {
  const uint32_t vo = 16u * lane;
  bload4<CP>(v.rs(), vo, 2u * w.sm, r.m);
  bload4<CP>(v.rs(), vo, v.ab + 2u * w.xs, r.z);
  bload4<CP>(v.rs(), vo, 2u * v.ab + 2u * w.sp, r.p);
}
// The chunk's three windows as eight consecutive sites per lane, in place in
// `r`: a fast chunk's vectors are there already; a chunk whose windows wrap
// around the end of the lattice (or pass it) is read element by element.
// Sites past the end read as empty (N = 0) and are never stored.
__device__ __forceinline__ void chunk_fill(const Win &w, Raw &r, const SlotView &v,
                                           uint32_t lane) {
  if (!w.fast) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t x = w.xs + 8u * lane + e;
      uint32_t ea = 0, eb = 0, ec = 0;
      if (x < v.L) {
        uint32_t pm = x + v.tm;
        pm -= (pm >= v.L) ? v.L : 0u;
        const uint32_t pp = x >= v.tm ? x - v.tm : x + v.L - v.tm;
        ea = bload2(v.rs(), 2u * pm, 0u);
        eb = bload2(v.rs(), 2u * x, v.ab);
        ec = bload2(v.rs(), 2u * pp, 2u * v.ab);
      }
      set16(r.m, e, ea); set16(r.z, e, eb); set16(r.p, e, ec);
    }
  }
  // complete here, so that no load of this chunk is still counted when the
  // next chunk's loads are issued
  for (int j = 0; j < 4; ++j) asm volatile("" : "+v"(r.m[j]), "+v"(r.z[j]), "+v"(r.p[j]));
}

// The block's next chunk index (an LDS counter), wave-uniform.
__device__ __forceinline__ uint32_t grab_chunk(uint32_t *ctr, uint32_t lane) {
  uint32_t v = 0;
  if (lane == 0) v = atomicAdd(ctr, 1u);
  return __builtin_amdgcn_readfirstlane(v);
}

// The chunks [k0, se) of one segment of a slot (chunk j at x0 + (j - i)
// 512, or with `rev`, for a segment that starts at i = 0, at x0 + (se - 1 -
// j) 512): the wave's first chunk k (its loads already issued into cr when
// fast), then chunks claimed one at a time from the block's counter.  One
// chunk: the next chunk's loads go out first (into the other register set;
// its bytes are disjoint from this chunk's), then this chunk is decided and
// stored, then the next chunk's vectors are taken.  The loop alternates the
// two register sets, so nothing is copied.
template <bool GAL, int MODE, bool TB = false, int CPO = -1>
__device__ __forceinline__ void run_segment(const StepParams &p, const TableDev &tab,
                                            uint32_t *err, const SlotView &sv,
                                            const LdsView &lv, uint2 key, uint4 *queue,
                                            uint4 *over, Rsrc ovr, uint32_t &F, uint32_t lane,
                                            uint32_t nwaves, bool youngest, bool second,
                                            uint32_t &next_chunk, uint32_t i, uint32_t se,
                                            uint32_t x0, uint32_t k, Win cw, Raw &cr,
                                            bool rev = false) {
  constexpr bool PATCH = MODE == kDrainPatch;
  // (CPO: the chunk accesses' cache policy when given, else streaming with
  // patched drains)
  constexpr int CP = CPO >= 0 ? CPO : PATCH ? kStreamingPolicy : 0;
  const uint32_t L = sv.L, tm = sv.tm, t = sv.t;  // of the segment's slot
  const Rsrc rs = sv.rs();
  const uint32_t ab = sv.ab;
  auto one = [&](Raw &cur, Raw &nxt) -> bool {
    // (young waves leave the segment's last chunks to the older ones)
    uint32_t nk = se;
    if (!(youngest || second) ||
        __builtin_amdgcn_readfirstlane(__atomic_load_n(&next_chunk, __ATOMIC_RELAXED)) +
                (youngest ? nwaves : nwaves / 2u) < se)
      nk = grab_chunk(&next_chunk, lane);
    nk = __builtin_amdgcn_readfirstlane(nk);  // wave-uniform after the join
    const bool has_next = nk < se;
    Win nw = cw;
    if (has_next) {
      nw = locate(x0 + (rev ? se - 1u - nk : nk - i) * 512u, sv);
      if (nw.fast) issue_raw<CP>(nw, sv, lane, nxt);
    }

    // ---- collide: LDS image first, the rest into the wave's queue ----
    {
      const uint32_t x8 = cw.xs + 8u * lane;
      const bool slow = __builtin_amdgcn_readfirstlane(cw.fast) == 0u;
      if (p.C != 0) {
        const uint32_t xl = sv.logical<TB>(x8);  // the lattice site keying the draws
        uint4 w0 = make_uint4(xl >> 2, t, sv.rid, 0u);
        uint4 w1 = make_uint4((xl >> 2) + 1u, t, sv.rid, 0u);
        decide_eight<PATCH>(w0, w1, key, cur.m, cur.z, cur.p, lv, queue, ovr, F, slow, x8, L,
                            cw.xs);
      } else {
        queue_saturated<PATCH>(cur.m, cur.z, cur.p, queue, ovr, F, slow, x8, L, cw.xs);
      }
      if constexpr (PATCH) {
        if (F) {
          patch_chunk<GAL, TB>(queue, over, F, lane, cw.xs, sv, lv, p, tab, err, cur.m,
                           cur.z, cur.p);
          F = 0;
        }
      }
    }

    // ---- store ----
    if (cw.fast) {
      const uint32_t vo = 16u * lane;
      bstore4<CP>(rs, vo, 2u * cw.sm, cur.m);
      bstore4<CP>(rs, vo, ab + 2u * cw.xs, cur.z);
      bstore4<CP>(rs, vo, 2u * ab + 2u * cw.sp, cur.p);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t x = cw.xs + 8u * lane + e;
        if (x < L) {
          uint32_t pm = x + tm;
          pm -= (pm >= L) ? L : 0u;
          const uint32_t pp = x >= tm ? x - tm : x + L - tm;
          bstore2(rs, 2u * pm, 0u, get16(cur.m, e));
          bstore2(rs, 2u * x, ab, get16(cur.z, e));
          bstore2(rs, 2u * pp, 2u * ab, get16(cur.p, e));
        }
      }
    }
    // ---- the next chunk's windows ----
    if (has_next) chunk_fill(nw, nxt, sv, lane);
    cw = nw;
    k = nk;
    // At most kDrainAt draws stay queued, so the next chunk's 64 x 8
    // always fit; kDrainChunk resolves every chunk's draws while its lines
    // are still in the L2 (kDrainPatch has none left here).
    if (!PATCH && has_next && F > (MODE == kDrainChunk ? 0u : kDrainAt)) {
      drain_queue<GAL, TB>(queue, over, F, lane, sv, p, tab, err);
      F = 0;
    }
    return has_next;
  };
  if (k < se) {
    Raw rb;
    chunk_fill(cw, cr, sv, lane);
    while (one(cr, rb) && one(rb, cr)) {
    }
  }
}

// Fused stream + collide.  Persistent blocks: block i takes a contiguous
// range of chunks; the slot's collision image is loaded into LDS for each
// run of one slot's chunks (a segment), whose chunks the block's waves then
// claim one at a time.  Each wave keeps one chunk of lookahead: the next
// chunk's vectors are requested before the current one is decided.  Each
// lane owns 8 consecutive sites of a chunk (two Philox calls).  Every
// physical element belongs to exactly one site per step, so the in-place
// update has no races.  Undecided draws wait in the wave's queue, which is
// drained between chunks once it nears capacity, and at the end of the
// slot's segment.
template <int MAXT, bool GAL, int MODE>
__global__ void __launch_bounds__(MAXT) k_step(StepLaunch a) {
  constexpr bool PATCH = MODE == kDrainPatch;
  // patched drains are the policy for states larger than the caches: their
  // chunk vectors are read and written as streaming (non-temporal) accesses
  constexpr int CP = PATCH ? kStreamingPolicy : 0;
  extern __shared__ uint4 lds[];
  const StepParams &p = a.p;
  const uint2 key = make_uint2((uint32_t)p.seed, (uint32_t)(p.seed >> 32));
  const uint32_t lane = threadIdx.x & 63u, nwaves = blockDim.x >> 6;
  // wave-uniform, which the compiler cannot infer from threadIdx.x
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint4 *const queue = lds + a.lds_bytes / 16u + wave * (kWaveLdsBytes / 16u);
  uint4 *const over = a.overflow + (size_t)(blockIdx.x * nwaves + wave) * kOverflow;
  const Rsrc ovr = __builtin_amdgcn_make_buffer_rsrc(over, 0, (int)(16u * kOverflow), kRsrcWord3);
  uint32_t F = 0;  // queue fill (wave-uniform), all draws of slot `cur`
  // Waves are spread over the four SIMDs in order, and the hardware issues
  // a SIMD's younger waves after its older ones, so a chunk held by a young
  // wave at the end of a segment finishes last: the youngest wave of each
  // SIMD stops claiming once at most nwaves chunks are left, the next
  // youngest once at most nwaves / 2 are.  The oldest wave of each SIMD
  // always claims, so every chunk is taken.
  const bool youngest = nwaves >= 8u && wave + 4u >= nwaves;
  const bool second = nwaves >= 12u && wave + 8u >= nwaves && !youngest;
  // after the image and the queues: the block's next unclaimed chunk of the
  // segment, and the last-block flag (so that the image starts at LDS 0)
  uint32_t *const ctl =
      reinterpret_cast<uint32_t *>(lds + a.lds_bytes / 16u + nwaves * (kWaveLdsBytes / 16u));
  uint32_t &next_chunk = ctl[0];
  const uint32_t per = (a.n_tiles + gridDim.x - 1) / gridDim.x;
  const uint32_t cb = blockIdx.x * per;
  const uint32_t ce = min(a.n_tiles, cb + per);
  uint32_t cur = 0xFFFFFFFFu;
  uint64_t img_off = ~0ull;  // pool offset of the image in LDS
  SlotView sv;
  sv.lo = sv.hi = 0;
  sv.ab = 0;
  sv.L = 1; sv.tm = sv.t = sv.rid = 0;
  sv.xoff = 0;
  sv.lg = 1;
  LdsView lv;
  lv.da2 = lv.dc2 = lv.w2 = lv.blo2 = lv.nb2 = 0;

  for (uint32_t i = cb;;) {
    TileDev t0;
    t0.slot = cur;
    if (i < ce) {
      if (a.single) {
        t0.slot = a.slot_first;
        t0.x0 = i * 512u;
        t0.next = a.n_tiles;
      } else {
        t0 = a.tiles[i];
      }
    }
    if (!PATCH && F && (i >= ce || t0.slot != cur)) {  // queued draws belong to slot `cur`
      drain_queue<GAL>(queue, over, F, lane, sv, p, a.tab, a.err);
      F = 0;
    }
    if (i >= ce) break;
    t0.x0 = __builtin_amdgcn_readfirstlane(t0.x0);
    const uint32_t se = __builtin_amdgcn_readfirstlane(min(ce, t0.next));
    // Each wave's first chunk of the segment is fixed, so that its loads are
    // in flight while the image is copied; the rest go to the block's waves
    // one at a time from a shared counter, so that waves issued less often
    // (the hardware favours older waves) take fewer chunks and all finish
    // together.
    const bool first = cur == 0xFFFFFFFFu;
    cur = t0.slot;
    const ImageDesc im = a.single ? a.im1 : a.images[cur];
    // replicas that share an image keep it in LDS from segment to segment
    const bool new_image = first || im.off != img_off;
    img_off = im.off;
    const SlotDev sl = a.single ? a.sl1 : a.slots[cur];
    const uint32_t tn = a.tslot[cur] + a.t_off;
    if (!first) __syncthreads();  // previous image and chunk counter no longer in use
    // (wave-uniform values kept in scalar registers)
    sv.t = __builtin_amdgcn_readfirstlane(tn);
    sv.L = __builtin_amdgcn_readfirstlane(sl.L);
    sv.tm = p.no_stream ? 0u : sv.t % sv.L;
    sv.rid = __builtin_amdgcn_readfirstlane(sl.rid);
    const uint64_t base = reinterpret_cast<uint64_t>(a.state + sl.off);
    sv.lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    sv.hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    sv.ab = __builtin_amdgcn_readfirstlane(2u * sl.stride);
    sv.lg = sv.L;
    uint32_t k = min(i + wave, se);
    if (threadIdx.x == 0) next_chunk = i + nwaves;
    Win cw = locate(t0.x0 + (k - i) * 512u, sv);
    Raw cr;
    if (k < se && cw.fast) issue_raw<CP>(cw, sv, lane, cr);
    if (new_image) {
      // ten independent 16-byte loads per thread per round (a 1024-thread
      // block moves 160 KiB in one round), then the stores (indices clamped
      // into the image; the stores past its end are skipped)
      const uint4 *src = reinterpret_cast<const uint4 *>(a.image_pool + im.off);
      const uint32_t n16 = im.bytes / 16u, bd = blockDim.x, last = n16 - 1u;
      for (uint32_t b0 = threadIdx.x; b0 < n16; b0 += 10u * bd) {
        uint4 v[10];
#pragma unroll
        for (uint32_t j = 0; j < 10; ++j) v[j] = src[min(b0 + j * bd, last)];
        // all ten loads are issued before the first store waits for its data
        // (otherwise the compiler moves each load into its store's branch)
#pragma unroll
        for (uint32_t j = 0; j < 10; ++j)
          asm volatile("" : "+v"(v[j].x), "+v"(v[j].y), "+v"(v[j].z), "+v"(v[j].w));
        lds[b0] = v[0];
#pragma unroll
        for (uint32_t j = 1; j < 10; ++j)
          if (b0 + j * bd < n16) lds[b0 + j * bd] = v[j];
      }
      lv.da2 = im.dim_a * 0x10001u;
      lv.dc2 = im.dim_c * 0x10001u;
      lv.w2 = (im.dim_c + 1u) * 0x10001u;
      lv.blo2 = im.b_lo * 0x10001u;
      lv.nb2 = im.nb * 0x10001u;
    }
    __syncthreads();  // the image and the counter are in place
    const uint32_t L = sv.L, tm = sv.tm, t = sv.t;  // of the segment's slot
    const Rsrc rs = sv.rs();
    const uint32_t ab = sv.ab;
    // One chunk: the next chunk's loads go out first (into the other
    // register set; its bytes are disjoint from this chunk's), then this
    // chunk is decided and stored, then the next chunk's vectors are taken.
    // The loop alternates the two register sets, so nothing is copied.
    auto one = [&](Raw &cur, Raw &nxt) -> bool {
      // (young waves leave the segment's last chunks to the older ones)
      uint32_t nk = se;
      if (!(youngest || second) ||
          __builtin_amdgcn_readfirstlane(__atomic_load_n(&next_chunk, __ATOMIC_RELAXED)) +
                  (youngest ? nwaves : nwaves / 2u) < se)
        nk = grab_chunk(&next_chunk, lane);
      nk = __builtin_amdgcn_readfirstlane(nk);  // wave-uniform after the join
      const bool has_next = nk < se;
      Win nw = cw;
      if (has_next) {
        nw = locate(t0.x0 + (nk - i) * 512u, sv);
        if (nw.fast) issue_raw<CP>(nw, sv, lane, nxt);
      }

      // ---- collide: LDS image first, the rest into the wave's queue ----
      {
        const uint32_t x8 = cw.xs + 8u * lane;
        const bool slow = __builtin_amdgcn_readfirstlane(cw.fast) == 0u;
        if (p.C != 0) {
          uint4 w0 = make_uint4(x8 >> 2, t, sv.rid, 0u);
          uint4 w1 = make_uint4((x8 >> 2) + 1u, t, sv.rid, 0u);
          decide_eight<PATCH>(w0, w1, key, cur.m, cur.z, cur.p, lv, queue, ovr, F, slow, x8, L,
                              cw.xs);
        } else {
          queue_saturated<PATCH>(cur.m, cur.z, cur.p, queue, ovr, F, slow, x8, L, cw.xs);
        }
        if constexpr (PATCH) {
          if (F) {
            patch_chunk<GAL>(queue, over, F, lane, cw.xs, sv, lv, p, a.tab, a.err, cur.m,
                             cur.z, cur.p);
            F = 0;
          }
        }
      }

      // ---- store ----
      if (cw.fast) {
        const uint32_t vo = 16u * lane;
        bstore4<CP>(rs, vo, 2u * cw.sm, cur.m);
        bstore4<CP>(rs, vo, ab + 2u * cw.xs, cur.z);
        bstore4<CP>(rs, vo, 2u * ab + 2u * cw.sp, cur.p);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t x = cw.xs + 8u * lane + e;
          if (x < L) {
            uint32_t pm = x + tm;
            pm -= (pm >= L) ? L : 0u;
            const uint32_t pp = x >= tm ? x - tm : x + L - tm;
            bstore2(rs, 2u * pm, 0u, get16(cur.m, e));
            bstore2(rs, 2u * x, ab, get16(cur.z, e));
            bstore2(rs, 2u * pp, 2u * ab, get16(cur.p, e));
          }
        }
      }
      // ---- the next chunk's windows ----
      if (has_next) chunk_fill(nw, nxt, sv, lane);
      cw = nw;
      k = nk;
      // At most kDrainAt draws stay queued, so the next chunk's 64 x 8
      // always fit; kDrainChunk resolves every chunk's draws while its lines
      // are still in the L2 (kDrainPatch has none left here).
      if (!PATCH && has_next && F > (MODE == kDrainChunk ? 0u : kDrainAt)) {
        drain_queue<GAL>(queue, over, F, lane, sv, p, a.tab, a.err);
        F = 0;
      }
      return has_next;
    };
    if (k < se) {
      Raw rb;
      chunk_fill(cw, cr, sv, lane);
      while (one(cr, rb) && one(rb, cr)) {
      }
    }
    i = se;
  }
  // With a ticket, the last block of the launch advances t of every slot in
  // the launch.  Every block has consumed its loads of t before it takes its
  // ticket (the values shaped its work), so nothing reads the new value
  // during this launch; the next launch sees it through the kernel boundary.
  if (!a.ticket) return;
  uint32_t &last = ctl[1];
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(a.ticket, 1u) == gridDim.x - 1u;
  __syncthreads();
  if (last) {
    for (uint32_t k = threadIdx.x; k < a.n_slots; k += blockDim.x) {
      const uint32_t s = a.slot_list ? a.slot_list[k] : a.slot_first + k;
      a.tslot[s] += 1u;
    }
    if (threadIdx.x == 0) atomicExch(a.ticket, 0u);
  }
}

// Eight consecutive elements pos .. pos + 7 (mod n) of the array at byte
// offset `arr` of r: one 16-byte access unless they wrap around n.
__device__ __forceinline__ void load8_wrap(Rsrc r, uint32_t arr, uint32_t pos, uint32_t n,
                                           uint32_t (&v)[4]) {
  if (pos + 8u <= n) {
    bload4(r, 2u * pos, arr, v);
    return;
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    uint32_t q = pos + (uint32_t)e;
    q -= q >= n ? n : 0u;
    set16(v, e, bload2(r, 2u * q, arr));
  }
}
__device__ __forceinline__ void store8_wrap(Rsrc r, uint32_t arr, uint32_t pos, uint32_t n,
                                            const uint32_t (&v)[4]) {
  if (pos + 8u <= n) {
    bstore4(r, 2u * pos, arr, v);
    return;
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    uint32_t q = pos + (uint32_t)e;
    q -= q >= n ? n : 0u;
    bstore2(r, 2u * q, arr, get16(v, e));
  }
}

// The grid-wide barrier of a blocked launch, without memory fences.  What it
// orders: every block's reads of the state (and of its step counter) before
// any block writes them.  A block's reads have returned once their values
// are stored into its copy, before it arrives; nothing else crosses blocks,
// and fences would write back and invalidate the L2s that hold the copies.
// `bar` counts arrivals across launches; this launch's blocks have all
// arrived when it reaches `target`.  Every block is resident (a cooperative
// launch), so the wait ends; one that has not ended after 2^24 polls flags an
// internal error and goes on, so that no launch can hang.
__device__ __forceinline__ void grid_barrier(uint32_t *bar, uint32_t target, uint32_t *err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(bar, 1u);
    for (uint32_t n = 0;
         (int32_t)(__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0;
         ++n) {
      if (n == (1u << 24)) {
        atomicOr(err, kErrInternal);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
}

// A pass of a blocked launch over the block's owned sites, eight per thread,
// read from its copy after `done` steps: WB writes them back into the state
// (the launch's last part, done = steps); LOG sums their moments (NM Fourier
// modes, the digest with DIG) in the lanes and writes the block's partial
// record of log `j` with device-coherent stores.  red: LDS of at least 8 KiB
// that no other part of the block uses meanwhile.
template <int NM, bool DIG, bool WB, bool LOG>
__device__ __forceinline__ void owned_pass(const TbLaunch &tb, Rsrc srs, Rsrc mrs, uint32_t sab,
                                           uint32_t mab, bool active, uint32_t L, uint32_t X0,
                                           uint32_t t0, uint32_t done, bool no_stream,
                                           uint32_t j, uint4 *red) {
  using namespace mom3;
  // Between steps (!WB) the Fourier sums take a second loop over the sites
  // (from the L2), so that the step loop's registers hold both.
  constexpr bool SPLIT = !WB && NM > 0;
  constexpr int NA = SPLIT ? 0 : NM;
  const uint32_t es = tb.es;
  Acc3<NA> A;
  i64 fs[2 * NM > 0 ? 2 * NM : 1] = {};
  if constexpr (LOG) acc_clear<NA>(A);
  if (active) {
    const uint32_t tms = no_stream ? 0u : done % es;
    const uint32_t tmk = no_stream ? 0u : (uint32_t)(((uint64_t)t0 + done) % L);
    const uint32_t x1 = min(L - X0, tb.R);
    for (uint32_t k = 8u * threadIdx.x; k < x1; k += 8u * blockDim.x) {
      const uint32_t i = tb.kh + k, x = X0 + k;
      uint32_t im_ = i + tms;
      im_ -= im_ >= es ? es : 0u;
      const uint32_t ip = i >= tms ? i - tms : i + es - tms;
      uint32_t m[4], z[4], q[4];
      load8_wrap(srs, 0u, im_, es, m);
      bload4(srs, 2u * i, sab, z);
      load8_wrap(srs, 2u * sab, ip, es, q);
      if constexpr (WB) {
        uint32_t pm = x + tmk;
        pm -= pm >= L ? L : 0u;
        const uint32_t pp = x >= tmk ? x - tmk : x + L - tmk;
        store8_wrap(mrs, 0u, pm, L, m);
        bstore4(mrs, 2u * x, mab, z);
        store8_wrap(mrs, 2u * mab, pp, L, q);
      }
      if constexpr (LOG) {
        // the eight sites x .. x + 7 (L and R are multiples of 8)
        Eight<NA> E;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          E.a[e] = m[e];
          E.b[e] = z[e];
          E.c[e] = q[e];
        }
        E.x = x;
        E.n = 8u;
#pragma unroll
        for (int r = 0; r < 2 * NA; ++r) {
          const uint4 *row = reinterpret_cast<const uint4 *>(tb.tw + (uint64_t)r * L + x);
          const uint4 w0 = row[0], w1 = row[1];
          E.w[r][0] = (int32_t)w0.x; E.w[r][1] = (int32_t)w0.y;
          E.w[r][2] = (int32_t)w0.z; E.w[r][3] = (int32_t)w0.w;
          E.w[r][4] = (int32_t)w1.x; E.w[r][5] = (int32_t)w1.y;
          E.w[r][6] = (int32_t)w1.z; E.w[r][7] = (int32_t)w1.w;
        }
        add_eight<NA, DIG>(A, E, tb.tw, L);
      }
    }
    if constexpr (LOG && SPLIT) {
      for (uint32_t k = 8u * threadIdx.x; k < x1; k += 8u * blockDim.x) {
        const uint32_t i = tb.kh + k, x = X0 + k;
        uint32_t im_ = i + tms;
        im_ -= im_ >= es ? es : 0u;
        const uint32_t ip = i >= tms ? i - tms : i + es - tms;
        uint32_t m[4], z[4], q[4];
        load8_wrap(srs, 0u, im_, es, m);
        bload4(srs, 2u * i, sab, z);
        load8_wrap(srs, 2u * sab, ip, es, q);
        int32_t N[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) N[e] = (int32_t)(get16(m, e) + get16(z, e) + get16(q, e));
#pragma unroll
        for (int r = 0; r < 2 * NM; ++r) {
          const uint4 *row = reinterpret_cast<const uint4 *>(tb.tw + (uint64_t)r * L + x);
          const uint4 w0 = row[0], w1 = row[1];
          fs[r] += (i64)N[0] * (int32_t)w0.x + (i64)N[1] * (int32_t)w0.y +
                   (i64)N[2] * (int32_t)w0.z + (i64)N[3] * (int32_t)w0.w +
                   (i64)N[4] * (int32_t)w1.x + (i64)N[5] * (int32_t)w1.y +
                   (i64)N[6] * (int32_t)w1.z + (i64)N[7] * (int32_t)w1.w;
        }
      }
    }
  }
  if constexpr (LOG) {
    constexpr int W = 12 + 2 * NM, V = 16;
    u64 v[V];
    const uint32_t mx = fold<NA, V>(A, v);
    if constexpr (SPLIT) {
#pragma unroll
      for (int r = 0; r < 2 * NM; ++r) v[12 + r] = (u64)fs[r];
    }
    u64 *const rd = reinterpret_cast<u64 *>(red);                     // 16 x V values
    uint32_t *const rmx = reinterpret_cast<uint32_t *>(rd + 16 * V);  // 16
    block_record<V, W, 11, true>(
        v, mx, tb.records + ((uint64_t)j * gridDim.x + blockIdx.x) * kMom3Rec, rd, rmx);
  }
}

// One launch's log j from the grid's partial records (read with
// device-coherent loads once every block has written them): the result row
// at tb.out + j kMom3Out, at step t.  red: LDS as for owned_pass.
__device__ __forceinline__ void log_final(const TbLaunch &tb, uint32_t j, uint32_t t, uint32_t L,
                                          uint4 *red) {
  using namespace mom3;
  const uint32_t n_modes = (tb.log - 1u) >> 1;
  const uint32_t npairs = 6u + n_modes;  // values 0 .. 11 + 2 n_modes
  u64 *const fin = reinterpret_cast<u64 *>(red);  // 16 waves x 32 values
  u64 *const T = fin + 16 * 32;                   // the grid's sums
  // thread (g, p) adds pair p (values 2p, 2p + 1) of records g, g + 64, ...
  const uint32_t p = threadIdx.x & 15u, g = threadIdx.x >> 4;
  const bool m0 = 2u * p == 11u, m1 = 2u * p + 1u == 11u;
  u64 a0 = 0, a1 = 0;
  if (p < npairs) {
    const u64 *const base = tb.records + (uint64_t)j * gridDim.x * kMom3Rec + 2u * p;
    for (uint32_t r = g; r < gridDim.x; r += 64u) {
      const u64 *const q = base + (uint64_t)r * kMom3Rec;
      const u64 v0 = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const u64 v1 = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      a0 = m0 ? max(a0, v0) : a0 + v0;
      a1 = m1 ? max(a1, v1) : a1 + v1;
    }
  }
  // the four groups of a wave, then the 16 waves
#pragma unroll
  for (int o = 16; o <= 32; o <<= 1) {
    const u64 b0 = shfl_xor_u64(a0, o), b1 = shfl_xor_u64(a1, o);
    a0 = m0 ? max(a0, b0) : a0 + b0;
    a1 = m1 ? max(a1, b1) : a1 + b1;
  }
  const uint32_t wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) < 16u) {
    fin[wave * 32u + 2u * p] = a0;
    fin[wave * 32u + 2u * p + 1u] = a1;
  }
  __syncthreads();
  if (threadIdx.x < kMom3Rec) {
    const uint32_t k = threadIdx.x;
    u64 s = 0;
    for (uint32_t w = 0; w < 16u; ++w) {
      const u64 y = fin[w * 32u + k];
      s = k == 11u ? max(s, y) : s + y;
    }
    T[k] = s;
  }
  __syncthreads();
  if (threadIdx.x < kMom3Out)
    tb.out[(uint64_t)j * kMom3Out + threadIdx.x] = (i64)result_field(threadIdx.x, T, t, L, n_modes);
  __syncthreads();  // (fin and T are reused by the next log)
}

// The log kinds of TbLaunch::log as instantiations of owned_pass.
template <bool WB, bool LOG>
__device__ __forceinline__ void owned_pass_kind(uint32_t kind, const TbLaunch &tb, Rsrc srs,
                                                Rsrc mrs, uint32_t sab, uint32_t mab, bool active,
                                                uint32_t L, uint32_t X0, uint32_t t0,
                                                uint32_t done, bool ns, uint32_t j, uint4 *red) {
  if constexpr (!LOG) {
    owned_pass<0, false, WB, false>(tb, srs, mrs, sab, mab, active, L, X0, t0, done, ns, j, red);
  } else {
    switch (kind) {
      case 1: owned_pass<0, false, WB, true>(tb, srs, mrs, sab, mab, active, L, X0, t0, done, ns, j, red); break;
      case 2: owned_pass<0, true, WB, true>(tb, srs, mrs, sab, mab, active, L, X0, t0, done, ns, j, red); break;
      case 3: owned_pass<1, false, WB, true>(tb, srs, mrs, sab, mab, active, L, X0, t0, done, ns, j, red); break;
      case 4: owned_pass<1, true, WB, true>(tb, srs, mrs, sab, mab, active, L, X0, t0, done, ns, j, red); break;
      default: owned_pass<2, false, WB, true>(tb, srs, mrs, sab, mab, active, L, X0, t0, done, ns, j, red); break;
    }
  }
}

// A log between two steps of a blocked launch: without the digest (whose
// mixing would make the step loop spill registers; the host ends a launch at
// each log with the digest instead).
__device__ __forceinline__ void log_between_steps(const TbLaunch &tb, Rsrc srs, Rsrc mrs,
                                                  uint32_t sab, uint32_t mab, bool active,
                                                  uint32_t L, uint32_t X0, uint32_t t0,
                                                  uint32_t done, bool ns, uint32_t j,
                                                  uint4 *red) {
  switch (tb.log) {
    case 1: owned_pass<0, false, false, true>(tb, srs, mrs, sab, mab, active, L, X0, t0, done, ns, j, red); break;
    case 3: owned_pass<1, false, false, true>(tb, srs, mrs, sab, mab, active, L, X0, t0, done, ns, j, red); break;
    default: owned_pass<2, false, false, true>(tb, srs, mrs, sab, mab, active, L, X0, t0, done, ns, j, red); break;
  }
}

// Several steps of one lattice per launch (see TbLaunch).  Deferred drains:
// the block's copy stays in the caches, and each step ends with the drain of
// every wave's queue and a block barrier, so step s + 1 reads what step s
// wrote.
template <int MAXT, bool GAL>
__global__ void __launch_bounds__(MAXT) k_step_tb(StepLaunch a, TbLaunch tb) {
  constexpr int MODE = kDrainDeferred;
  extern __shared__ uint4 lds[];
  const StepParams &p = a.p;
  const uint2 key = make_uint2((uint32_t)p.seed, (uint32_t)(p.seed >> 32));
  const uint32_t lane = threadIdx.x & 63u, nwaves = blockDim.x >> 6;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint4 *const queue = lds + a.lds_bytes / 16u + wave * (kWaveLdsBytes / 16u);
  uint4 *const over = a.overflow + (size_t)(blockIdx.x * nwaves + wave) * kOverflow;
  const Rsrc ovr = __builtin_amdgcn_make_buffer_rsrc(over, 0, (int)(16u * kOverflow), kRsrcWord3);
  uint32_t F = 0;
  const bool youngest = nwaves >= 8u && wave + 4u >= nwaves;
  const bool second = nwaves >= 12u && wave + 8u >= nwaves && !youngest;
  uint32_t *const ctl =
      reinterpret_cast<uint32_t *>(lds + a.lds_bytes / 16u + nwaves * (kWaveLdsBytes / 16u));
  uint32_t &next_chunk = ctl[0];

  // the lattice: one slot, its descriptors carried by value
  const SlotDev sl = a.sl1;
  const ImageDesc im = a.im1;
  const uint32_t L = sl.L;
  const uint32_t t0 = __builtin_amdgcn_readfirstlane(a.tslot[a.slot_first] + a.t_off);
  const uint32_t X0 = blockIdx.x * tb.R;  // first owned site
  const bool active = X0 < L;
  const uint32_t xoff = X0 >= tb.kh ? X0 - tb.kh : X0 + L - tb.kh;  // site of copy index 0
  uint16_t *const main_m = a.state + sl.off;
  uint16_t *const scr = tb.scratch + (uint64_t)blockIdx.x * tb.bstride;
  const uint32_t es = tb.es;

  // (1) the region and its extra sites at step t0, in logical order, eight
  // sites per thread (the region's first site, L and es are multiples of 8)
  const uint32_t mab = 2u * sl.stride, sab = 2u * tb.stride;
  const Rsrc mrs = __builtin_amdgcn_make_buffer_rsrc(main_m, 0, (int)(3u * mab), kRsrcWord3);
  const Rsrc srs = __builtin_amdgcn_make_buffer_rsrc(scr, 0, (int)(3u * sab), kRsrcWord3);
  if (active) {
    const uint32_t tm = p.no_stream ? 0u : t0 % L;
    for (uint32_t i = 8u * threadIdx.x; i < es; i += 8u * blockDim.x) {
      uint32_t x = xoff + i;
      x -= x >= L ? L : 0u;
      uint32_t pm = x + tm;
      pm -= pm >= L ? L : 0u;
      const uint32_t pp = x >= tm ? x - tm : x + L - tm;
      uint32_t m[4], z[4], q[4];
      load8_wrap(mrs, 0u, pm, L, m);
      load8_wrap(mrs, mab, x, L, z);
      load8_wrap(mrs, 2u * mab, pp, L, q);
      bstore4(srs, 2u * i, 0u, m);
      bstore4(srs, 2u * i, sab, z);
      bstore4(srs, 2u * i, 2u * sab, q);
    }
  }
  // the collision image, once for all steps
  LdsView lv;
  {
    const uint4 *src = reinterpret_cast<const uint4 *>(a.image_pool + im.off);
    const uint32_t n16 = im.bytes / 16u, bd = blockDim.x;
    for (uint32_t b0 = threadIdx.x; b0 < n16; b0 += bd) lds[b0] = src[b0];
    lv.da2 = im.dim_a * 0x10001u;
    lv.dc2 = im.dim_c * 0x10001u;
    lv.w2 = (im.dim_c + 1u) * 0x10001u;
    lv.blo2 = im.b_lo * 0x10001u;
    lv.nb2 = im.nb * 0x10001u;
  }
  // (2) every block has read the state (and its step counter) before any
  // writes it; the launch advances the counter itself
  grid_barrier(tb.bar, tb.bar_target, a.err);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.tslot[a.slot_first] += tb.steps;

  // (3) the steps on the block's copy: a periodic lattice of es sites
  SlotView sv;
  const uint64_t base = reinterpret_cast<uint64_t>(scr);
  sv.lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
  sv.hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
  sv.ab = 2u * tb.stride;
  sv.L = es;
  sv.rid = sl.rid;
  sv.xoff = xoff;
  sv.lg = L;
  const uint32_t nch = (es + 511u) / 512u;
  for (uint32_t s = 0; s < tb.steps; ++s) {
    sv.t = t0 + s;
    sv.tm = p.no_stream ? 0u : s % es;
    const uint32_t k = min(wave, nch);
    // odd steps take the chunks from the copy's end: a step starts on the
    // chunks the step before finished with, which the L2 still holds (the
    // order of a step's chunks does not change its results)
    const bool rev = (s & 1u) != 0u;
    if (threadIdx.x == 0) next_chunk = nwaves;
    const Win cw = locate((rev && k < nch ? nch - 1u - k : k) * 512u, sv);
    Raw cr;
    if (active && k < nch && cw.fast) issue_raw<0>(cw, sv, lane, cr);
    __syncthreads();  // the counter is reset
    if (active) {
      run_segment<GAL, MODE, true>(p, a.tab, a.err, sv, lv, key, queue, over, ovr, F, lane,
                                   nwaves, youngest, second, next_chunk, 0u, nch, 0u, k, cw, cr,
                                   rev);
      if (F) {
        drain_queue<GAL, true>(queue, over, F, lane, sv, p, a.tab, a.err);
        F = 0;
      }
    }
    __syncthreads();  // step s is written before step s + 1 reads it
    // a log after this step (the write-back sums the one after the last)
    const uint32_t done = s + 1u;
    if (!GAL && tb.n_logs && done < tb.steps && done >= tb.log_first &&
        (done - tb.log_first) % tb.log_every == 0u)
      log_between_steps(tb, srs, mrs, sab, mab, active, L, X0, t0, done, p.no_stream != 0,
                        (done - tb.log_first) / tb.log_every, lds + a.lds_bytes / 16u);
  }

  // (4) the owned sites back into the state at step t0 + steps, with the
  // moments of a log after the last step; the miss queues' LDS is free now
  uint4 *const red = lds + a.lds_bytes / 16u;
  const bool ns = p.no_stream != 0;
  const uint32_t last = tb.n_logs ? tb.log_first + (tb.n_logs - 1u) * tb.log_every : 0u;
  if (tb.n_logs && last == tb.steps)
    owned_pass_kind<true, true>(tb.log, tb, srs, mrs, sab, mab, active, L, X0, t0, tb.steps, ns,
                                tb.n_logs - 1u, red);
  else
    owned_pass_kind<true, false>(0u, tb, srs, mrs, sab, mab, active, L, X0, t0, tb.steps, ns, 0u,
                                 red);
  // (5) the logs: once every block's records are stored (a second barrier),
  // block b adds logs b, b + grid, ...
  if (tb.n_logs) {
    __builtin_amdgcn_s_waitcnt(0);
    grid_barrier(tb.bar, tb.bar_target + gridDim.x, a.err);
    for (uint32_t j = blockIdx.x; j < tb.n_logs; j += gridDim.x)
      log_final(tb, j, t0 + tb.log_first + j * tb.log_every, L, red);
  }
}

// Several steps per launch in tiles (TbLaunch::T > 0), for lattices whose
// blocks' whole copies would stream from memory at every step.  Block b owns
// the sites [X0, end) = [b R, min(L, b R + R)) and goes through them in
// tiles of T sites from left to right: tile [a, a + n) is copied with kh
// extra sites on each side into the copy area (es = n + 2 kh sites; all
// blocks' copies together stay in the caches while they are stepped),
// advanced `steps` steps as in k_step_tb, and written back at step
// t + steps before the next tile.  Every site a tile reads must be at step
// t, and a write-back overwrites step-t values kh sites to either side of
// the written ones (shifted layout), so the tile's first 2 kh sites come
// from the carry area the previous tile filled, the sites within kh of the
// region's ends from side areas where every block put its region's first
// and last kh sites before the grid-wide barrier (with device-coherent
// stores and loads: the barrier has no fence), and only the rest from the
// state; see the copy-in below.
// Per-block scratch (elements): the copy (3 x stride), two carry areas (3 x
// 2 kh each) and the two side areas (3 x kh each).
template <int MAXT, bool GAL>
__global__ void __launch_bounds__(MAXT) k_step_tt(StepLaunch a, TbLaunch tb) {
  constexpr int MODE = kDrainDeferred;
  extern __shared__ uint4 lds[];
  const StepParams &p = a.p;
  const uint2 key = make_uint2((uint32_t)p.seed, (uint32_t)(p.seed >> 32));
  const uint32_t lane = threadIdx.x & 63u, nwaves = blockDim.x >> 6;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint4 *const queue = lds + a.lds_bytes / 16u + wave * (kWaveLdsBytes / 16u);
  uint4 *const over = a.overflow + (size_t)(blockIdx.x * nwaves + wave) * kOverflow;
  const Rsrc ovr = __builtin_amdgcn_make_buffer_rsrc(over, 0, (int)(16u * kOverflow), kRsrcWord3);
  uint32_t F = 0;
  const bool youngest = nwaves >= 8u && wave + 4u >= nwaves;
  const bool second = nwaves >= 12u && wave + 8u >= nwaves && !youngest;
  uint32_t *const ctl =
      reinterpret_cast<uint32_t *>(lds + a.lds_bytes / 16u + nwaves * (kWaveLdsBytes / 16u));
  uint32_t &next_chunk = ctl[0];

  const SlotDev sl = a.sl1;
  const ImageDesc im = a.im1;
  const uint32_t L = sl.L, kh = tb.kh;
  const uint32_t t0 = __builtin_amdgcn_readfirstlane(a.tslot[a.slot_first] + a.t_off);
  const uint32_t nact = (L + tb.R - 1u) / tb.R;  // blocks that own sites
  const uint32_t X0 = blockIdx.x * tb.R;
  const bool active = blockIdx.x < nact;
  const uint32_t end = active ? min(L, X0 + tb.R) : X0;
  const uint32_t pb = blockIdx.x > 0u ? blockIdx.x - 1u : nact - 1u;  // neighbours' areas
  const uint32_t nb = blockIdx.x + 1u < nact ? blockIdx.x + 1u : 0u;
  uint16_t *const main_m = a.state + sl.off;
  const uint32_t mab = 2u * sl.stride, sab = 2u * tb.stride;
  const Rsrc mrs = __builtin_amdgcn_make_buffer_rsrc(main_m, 0, (int)(3u * mab), kRsrcWord3);
  uint16_t *const scr = tb.scratch + (uint64_t)blockIdx.x * tb.bstride;
  // the block's whole scratch (the copy and the small areas after it)
  const Rsrc srs = __builtin_amdgcn_make_buffer_rsrc(scr, 0, (int)(2u * tb.bstride), kRsrcWord3);
  // a block's small areas, as byte offsets from its scratch: carry c (2 kh
  // sites, array i at + 4 kh i), the region's first and last kh sites (array
  // i at + 2 kh i)
  const uint32_t kc = 12u * kh, ks = 6u * kh;  // bytes per carry, per side area
  auto carry_at = [&](uint32_t c) { return 3u * sab + c * kc; };
  const uint32_t first_at = 3u * sab + 2u * kc, last_at = first_at + ks;
  const Rsrc all = __builtin_amdgcn_make_buffer_rsrc(tb.scratch, 0, 0x7fffffff, kRsrcWord3);
  const uint64_t area_bytes = 2ull * tb.bstride;
  const uint32_t tm = p.no_stream ? 0u : t0 % L;

  // (1) the region's first and last kh sites at step t0 into the side areas
  if (active) {
    for (uint32_t i = 8u * threadIdx.x; i < 2u * kh; i += 8u * blockDim.x) {
      const bool last = i >= kh;
      const uint32_t o = last ? i - kh : i;
      uint32_t x = last ? end + L - kh + o : X0 + o;
      x -= x >= L ? L : 0u;
      x -= x >= L ? L : 0u;
      uint32_t pm = x + tm;
      pm -= pm >= L ? L : 0u;
      const uint32_t pp = x >= tm ? x - tm : x + L - tm;
      uint32_t m[4], z[4], q[4];
      load8_wrap(mrs, 0u, pm, L, m);
      load8_wrap(mrs, mab, x, L, z);
      load8_wrap(mrs, 2u * mab, pp, L, q);
      const uint32_t at = (last ? last_at : first_at) + 2u * o;
      bstore4<kDevicePolicy>(srs, at, 0u, m);
      bstore4<kDevicePolicy>(srs, at, 2u * kh, z);
      bstore4<kDevicePolicy>(srs, at, 4u * kh, q);
    }
  }
  // the side areas are complete before this block arrives at the barrier
  __builtin_amdgcn_s_waitcnt(0);
  LdsView lv;
  {
    const uint4 *src = reinterpret_cast<const uint4 *>(a.image_pool + im.off);
    const uint32_t n16 = im.bytes / 16u, bd = blockDim.x;
    for (uint32_t b0 = threadIdx.x; b0 < n16; b0 += bd) lds[b0] = src[b0];
    lv.da2 = im.dim_a * 0x10001u;
    lv.dc2 = im.dim_c * 0x10001u;
    lv.w2 = (im.dim_c + 1u) * 0x10001u;
    lv.blo2 = im.b_lo * 0x10001u;
    lv.nb2 = im.nb * 0x10001u;
  }
  // (2) every block's side areas are written and every block has read its
  // step counter before any block writes the state
  grid_barrier(tb.bar, tb.bar_target, a.err);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.tslot[a.slot_first] += tb.steps;
  if (!active) return;

  SlotView sv;
  const uint64_t base = reinterpret_cast<uint64_t>(scr);
  sv.lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
  sv.hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
  sv.ab = sab;
  sv.rid = sl.rid;
  sv.lg = L;
  const uint32_t pbo = (uint32_t)((uint64_t)pb * area_bytes), nbo = (uint32_t)((uint64_t)nb * area_bytes);
  uint32_t c = 0;
  for (uint32_t x0 = X0; x0 < end; x0 += tb.T, c ^= 1u) {
    const uint32_t n = min(tb.T, end - x0), es = n + 2u * kh;
    const uint32_t xoff = x0 >= kh ? x0 - kh : x0 + L - kh;  // site of copy index 0
    // (3) the tile and its extra sites at step t0, eight sites per thread.
    // A write-back at step t0 + steps moves the n_-1 of sites up to `steps`
    // to the right of the written ones and the n_+1 of sites up to `steps`
    // to their left (in-place shifted layout), so what earlier tiles, and
    // the neighbouring blocks, may have written over is taken from copies
    // made before: copy index i < 2 kh (sites within kh of the tile's
    // start) from the previous tile's carry, or for the first tile from the
    // side areas; sites within kh of the region's end from its side area;
    // sites past it from the next block's.  Copy indices [n, n + 2 kh) also
    // go into carry c for the next tile.
    for (uint32_t i = 8u * threadIdx.x; i < es; i += 8u * blockDim.x) {
      uint32_t m[4], z[4], q[4];
      const uint32_t y = x0 + i;  // the site plus kh, unwrapped
      uint32_t at = 0, ah = 0;    // an area: byte offset, bytes per array
      bool area = true, dev = false;
      if (x0 != X0 && i < 2u * kh) {
        at = carry_at(c ^ 1u) + 2u * i;
        ah = 4u * kh;
      } else if (x0 == X0 && i < kh) {
        dev = true;  // the previous block's last sites (another block's area)
        at = pbo + last_at + 2u * i;
        ah = 2u * kh;
      } else if (x0 == X0 && i < 2u * kh) {
        at = first_at + 2u * (i - kh);
        ah = 2u * kh;
      } else if (y - kh >= end) {
        dev = true;  // the next block's first sites
        at = nbo + first_at + 2u * (y - kh - end);
        ah = 2u * kh;
      } else if (y >= end) {
        at = last_at + 2u * (y - end);  // (y - kh) - (end - kh)
        ah = 2u * kh;
      } else {
        area = false;
      }
      if (!area) {
        uint32_t x = y - kh;
        x -= x >= L ? L : 0u;
        uint32_t pm = x + tm;
        pm -= pm >= L ? L : 0u;
        const uint32_t pp = x >= tm ? x - tm : x + L - tm;
        load8_wrap(mrs, 0u, pm, L, m);
        load8_wrap(mrs, mab, x, L, z);
        load8_wrap(mrs, 2u * mab, pp, L, q);
      } else if (dev) {
        bload4<kDevicePolicy>(all, at, 0u, m);
        bload4<kDevicePolicy>(all, at, ah, z);
        bload4<kDevicePolicy>(all, at, 2u * ah, q);
      } else {
        bload4(srs, at, 0u, m);
        bload4(srs, at, ah, z);
        bload4(srs, at, 2u * ah, q);
      }
      bstore4(srs, 2u * i, 0u, m);
      bstore4(srs, 2u * i, sab, z);
      bstore4(srs, 2u * i, 2u * sab, q);
      if (i >= n) {
        const uint32_t cat = carry_at(c) + 2u * (i - n);
        bstore4(srs, cat, 0u, m);
        bstore4(srs, cat, 4u * kh, z);
        bstore4(srs, cat, 8u * kh, q);
      }
    }
    __syncthreads();
    // (4) the steps on the tile's copy: a periodic lattice of es sites
    sv.L = es;
    sv.xoff = xoff;
    const uint32_t nch = (es + 511u) / 512u;
    for (uint32_t s = 0; s < tb.steps; ++s) {
      sv.t = t0 + s;
      sv.tm = p.no_stream ? 0u : s % es;
      const uint32_t k = min(wave, nch);
      const bool rev = (s & 1u) != 0u;  // alternating chunk order, as in k_step_tb
      if (threadIdx.x == 0) next_chunk = nwaves;
      const Win cw = locate((rev && k < nch ? nch - 1u - k : k) * 512u, sv);
      Raw cr;
      if (k < nch && cw.fast) issue_raw<0>(cw, sv, lane, cr);
      __syncthreads();  // the counter is reset
      run_segment<GAL, MODE, true>(p, a.tab, a.err, sv, lv, key, queue, over, ovr, F, lane,
                                   nwaves, youngest, second, next_chunk, 0u, nch, 0u, k, cw, cr,
                                   rev);
      if (F) {
        drain_queue<GAL, true>(queue, over, F, lane, sv, p, a.tab, a.err);
        F = 0;
      }
      __syncthreads();  // step s is written before step s + 1 reads it
    }
    // (5) the tile back into the state at step t0 + steps
    TbLaunch tt = tb;
    tt.R = n;
    tt.es = es;
    owned_pass<0, false, true, false>(tt, srs, mrs, sab, mab, true, L, x0, t0, tb.steps,
                                      p.no_stream != 0, 0u, nullptr);
    __syncthreads();  // the copy area is read before the next tile fills it
  }
}

// Several steps per launch for a context of several replicas (TbLaunch::reps):
// block b advances the replicas of its list one after the other, each as a
// whole.  A replica is copied at its step t into the block's copy area (a
// periodic lattice of L sites, so no extra sites: its own periodic boundary
// is the copy's), advanced `steps` steps there with its own collision image,
// and written back at step t + steps; then its step counter moves.  No data
// crosses blocks, so there is no grid-wide barrier.
template <int MAXT, bool GAL, int MODE>
__global__ void __launch_bounds__(MAXT) k_step_tr(StepLaunch a, TbLaunch tb) {
  extern __shared__ uint4 lds[];
  const StepParams &p = a.p;
  const uint2 key = make_uint2((uint32_t)p.seed, (uint32_t)(p.seed >> 32));
  const uint32_t lane = threadIdx.x & 63u, nwaves = blockDim.x >> 6;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint4 *const queue = lds + a.lds_bytes / 16u + wave * (kWaveLdsBytes / 16u);
  uint4 *const over = a.overflow + (size_t)(blockIdx.x * nwaves + wave) * kOverflow;
  const Rsrc ovr = __builtin_amdgcn_make_buffer_rsrc(over, 0, (int)(16u * kOverflow), kRsrcWord3);
  uint32_t F = 0;
  const bool youngest = nwaves >= 8u && wave + 4u >= nwaves;
  const bool second = nwaves >= 12u && wave + 8u >= nwaves && !youngest;
  uint32_t *const ctl =
      reinterpret_cast<uint32_t *>(lds + a.lds_bytes / 16u + nwaves * (kWaveLdsBytes / 16u));
  uint32_t &next_chunk = ctl[0];
  uint16_t *const scr = tb.scratch + (uint64_t)blockIdx.x * tb.bstride;
  const uint32_t sab = 2u * tb.stride;
  const Rsrc srs = __builtin_amdgcn_make_buffer_rsrc(scr, 0, (int)(3u * sab), kRsrcWord3);
  SlotView sv;
  const uint64_t base = reinterpret_cast<uint64_t>(scr);
  sv.lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
  sv.hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
  sv.ab = sab;
  sv.xoff = 0;
  LdsView lv;
  uint64_t loaded = ~0ull;  // pool offset of the image in LDS
  const uint32_t i0 = tb.item_first[blockIdx.x], i1 = tb.item_first[blockIdx.x + 1u];
  for (uint32_t it = i0; it < i1; ++it) {
    const uint32_t r = __builtin_amdgcn_readfirstlane(tb.items[it]);
    const SlotDev sl = a.slots[r];
    const ImageDesc im = a.images[r];
    const uint32_t L = sl.L;
    const uint32_t t0 = __builtin_amdgcn_readfirstlane(a.tslot[r] + a.t_off);
    const Rsrc mrs =
        __builtin_amdgcn_make_buffer_rsrc(a.state + sl.off, 0, (int)(6u * sl.stride), kRsrcWord3);
    const uint32_t mab = 2u * sl.stride;
    // the previous replica is written back (the copy area and the image are
    // free) and its counter read
    __syncthreads();
    if (im.off != loaded) {
      const uint4 *src = reinterpret_cast<const uint4 *>(a.image_pool + im.off);
      const uint32_t n16 = im.bytes / 16u;
      for (uint32_t b0 = threadIdx.x; b0 < n16; b0 += blockDim.x) lds[b0] = src[b0];
      lv.da2 = im.dim_a * 0x10001u;
      lv.dc2 = im.dim_c * 0x10001u;
      lv.w2 = (im.dim_c + 1u) * 0x10001u;
      lv.blo2 = im.b_lo * 0x10001u;
      lv.nb2 = im.nb * 0x10001u;
      loaded = im.off;
    }
    // (1) the replica at step t0 into the copy, in logical order; a group of
    // eight that passes L takes its sites one by one
    const uint32_t tm = p.no_stream ? 0u : t0 % L;
    for (uint32_t i = 8u * threadIdx.x; i < L; i += 8u * blockDim.x) {
      uint32_t pm = i + tm;
      pm -= pm >= L ? L : 0u;
      const uint32_t pp = i >= tm ? i - tm : i + L - tm;
      if (i + 8u <= L) {
        uint32_t m[4], z[4], q[4];
        load8_wrap(mrs, 0u, pm, L, m);
        load8_wrap(mrs, mab, i, L, z);
        load8_wrap(mrs, 2u * mab, pp, L, q);
        bstore4(srs, 2u * i, 0u, m);
        bstore4(srs, 2u * i, sab, z);
        bstore4(srs, 2u * i, 2u * sab, q);
      } else {
        for (uint32_t x = i; x < L; ++x) {
          uint32_t a1 = x + tm;
          a1 -= a1 >= L ? L : 0u;
          const uint32_t a3 = x >= tm ? x - tm : x + L - tm;
          bstore2(srs, 2u * x, 0u, bload2(mrs, 2u * a1, 0u));
          bstore2(srs, 2u * x, sab, bload2(mrs, 2u * x, mab));
          bstore2(srs, 2u * x, 2u * sab, bload2(mrs, 2u * a3, 2u * mab));
        }
      }
    }
    __syncthreads();
    // (2) the steps on the copy: the replica itself, shifted from step t0
    sv.L = L;
    sv.lg = L;
    sv.rid = sl.rid;
    const uint32_t nch = (L + 511u) / 512u;
    for (uint32_t s = 0; s < tb.steps; ++s) {
      sv.t = t0 + s;
      sv.tm = p.no_stream ? 0u : s % L;
      const uint32_t k = min(wave, nch);
      const bool rev = (s & 1u) != 0u;  // alternating chunk order, as in k_step_tb
      if (threadIdx.x == 0) next_chunk = nwaves;
      const Win cw = locate((rev && k < nch ? nch - 1u - k : k) * 512u, sv);
      Raw cr;
      if (k < nch && cw.fast) issue_raw<0>(cw, sv, lane, cr);
      __syncthreads();  // the counter is reset
      run_segment<GAL, MODE, true, 0>(p, a.tab, a.err, sv, lv, key, queue, over, ovr, F, lane,
                                   nwaves, youngest, second, next_chunk, 0u, nch, 0u, k, cw, cr,
                                   rev);
      if (F) {
        drain_queue<GAL, true>(queue, over, F, lane, sv, p, a.tab, a.err);
        F = 0;
      }
      __syncthreads();  // step s is written before step s + 1 reads it
    }
    // (3) the replica back at step t0 + steps (a group that passes L site by
    // site)
    const uint32_t tms = p.no_stream ? 0u : tb.steps % L;
    const uint32_t tmk = p.no_stream ? 0u : (uint32_t)(((uint64_t)t0 + tb.steps) % L);
    for (uint32_t i = 8u * threadIdx.x; i < L; i += 8u * blockDim.x) {
      if (i + 8u <= L) {
        uint32_t cm = i + tms;
        cm -= cm >= L ? L : 0u;
        const uint32_t cp = i >= tms ? i - tms : i + L - tms;
        uint32_t m[4], z[4], q[4];
        load8_wrap(srs, 0u, cm, L, m);
        load8_wrap(srs, sab, i, L, z);
        load8_wrap(srs, 2u * sab, cp, L, q);
        uint32_t pm = i + tmk;
        pm -= pm >= L ? L : 0u;
        const uint32_t pp = i >= tmk ? i - tmk : i + L - tmk;
        store8_wrap(mrs, 0u, pm, L, m);
        store8_wrap(mrs, mab, i, L, z);
        store8_wrap(mrs, 2u * mab, pp, L, q);
      } else {
        for (uint32_t x = i; x < L; ++x) {
          uint32_t c1 = x + tms;
          c1 -= c1 >= L ? L : 0u;
          const uint32_t c3 = x >= tms ? x - tms : x + L - tms;
          uint32_t a1 = x + tmk;
          a1 -= a1 >= L ? L : 0u;
          const uint32_t a3 = x >= tmk ? x - tmk : x + L - tmk;
          bstore2(mrs, 2u * a1, 0u, bload2(srs, 2u * c1, 0u));
          bstore2(mrs, 2u * x, mab, bload2(srs, 2u * x, sab));
          bstore2(mrs, 2u * a3, 2u * mab, bload2(srs, 2u * c3, 2u * sab));
        }
      }
    }
    if (threadIdx.x == 0) a.tslot[r] = t0 - a.t_off + tb.steps;
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

__global__ void k_add_t(uint32_t *tslot, uint32_t slot_first, uint32_t n, uint32_t add) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    tslot[slot_first + k] += add;
}
__global__ void k_set_t(uint32_t *tslot, const uint32_t *slot_list, uint32_t n, uint32_t value) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) tslot[slot_list[i]] = value;
}

// Occupation-number histograms.  Each block takes a contiguous run of tiles
// (tiles are ordered by slot), reads every velocity array in physical order
// (a marginal histogram does not depend on which site an element belongs
// to), bins in LDS, and adds each non-empty bin to the slot's global row with
// one 64-bit atomic whenever the run moves to another slot or ends.
__global__ void __launch_bounds__(256) k_histogram(
    const uint16_t *__restrict__ state, const SlotDev *__restrict__ slots,
    const TileDev *__restrict__ tiles, uint32_t n_tiles, uint32_t tile_sites, uint32_t n_bins,
    unsigned long long *__restrict__ hist) {
  extern __shared__ uint32_t bins[];  // [3][n_bins]
  const uint32_t per = (n_tiles + gridDim.x - 1u) / gridDim.x;
  const uint32_t t_begin = blockIdx.x * per, t_end = min(n_tiles, t_begin + per);
  if (t_begin >= t_end) return;
  const uint32_t nb3 = 3u * n_bins, top = n_bins - 1u;
  for (uint32_t j = threadIdx.x; j < nb3; j += blockDim.x) bins[j] = 0u;
  uint32_t cur = tiles[t_begin].slot;
  auto flush = [&](uint32_t slot) {
    __syncthreads();
    unsigned long long *row = hist + (uint64_t)slot * nb3;
    for (uint32_t j = threadIdx.x; j < nb3; j += blockDim.x) {
      const uint32_t v = bins[j];
      if (v) {
        atomicAdd(&row[j], (unsigned long long)v);
        bins[j] = 0u;
      }
    }
    __syncthreads();
  };
  __syncthreads();
  for (uint32_t t = t_begin; t < t_end; ++t) {
    const TileDev tile = tiles[t];
    if (tile.slot != cur) {
      flush(cur);
      cur = tile.slot;
    }
    const SlotDev sl = slots[tile.slot];
    const uint32_t end = min(sl.L, tile.x0 + tile_sites);
    for (uint32_t x = tile.x0 + threadIdx.x; x < end; x += blockDim.x) {
#pragma unroll
      for (uint32_t i = 0; i < 3u; ++i) {
        const uint32_t n = state[sl.off + (uint64_t)i * sl.stride + x];
        atomicAdd(&bins[i * n_bins + min(n, top)], 1u);
      }
    }
  }
  flush(cur);
}

}  // namespace

// Sets the dynamic LDS limit of the six instantiations for this block size
// and returns the smallest of their occupancies.
template <int MAXT, bool GAL, int MODE>
static hipError_t occupancy_one(uint32_t threads, uint32_t lds, int &blocks) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_step<MAXT, GAL, MODE>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e) return e;
  int b = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_step<MAXT, GAL, MODE>, (int)threads, lds);
  blocks = std::min(blocks, b);
  return e;
}
template <int MAXT, bool GAL>
static hipError_t occupancy_modes(uint32_t threads, uint32_t lds, int &blocks) {
  hipError_t e = occupancy_one<MAXT, GAL, kDrainDeferred>(threads, lds, blocks);
  if (!e) e = occupancy_one<MAXT, GAL, kDrainChunk>(threads, lds, blocks);
  if (!e) e = occupancy_one<MAXT, GAL, kDrainPatch>(threads, lds, blocks);
  return e;
}
template <int MAXT>
static hipError_t occupancy_of(uint32_t threads, uint32_t lds, int &blocks) {
  blocks = 1 << 30;
  hipError_t e = occupancy_modes<MAXT, false>(threads, lds, blocks);
  if (!e) e = occupancy_modes<MAXT, true>(threads, lds, blocks);
  return e;
}

uint32_t step_lds_bytes(const Schedule &sch, uint32_t image_bytes) {
  return (image_bytes + 15u) / 16u * 16u + (sch.threads / 64u) * kWaveLdsBytes + 16u;
}

// Blocks of up to 512 threads may use up to 256 VGPRs per lane.
hipError_t step_occupancy(const Schedule &sch, uint32_t lds_bytes, uint32_t n_cu,
                          uint32_t &max_blocks) {
  int b = 0;
  if (sch.groups != 1) return hipErrorInvalidValue;
  const uint32_t lds = step_lds_bytes(sch, lds_bytes);
  hipError_t e = sch.threads <= 512 ? occupancy_of<512>(sch.threads, lds, b)
                                    : occupancy_of<1024>(sch.threads, lds, b);
  if (e) return e;
  if (b < 1) return hipErrorInvalidConfiguration;
  max_blocks = (uint32_t)b * n_cu;
  return hipSuccess;
}

template <int MAXT, bool GAL>
static void launch_mode(dim3 grid, dim3 block, uint32_t lds, hipStream_t s, const StepLaunch &a) {
  switch (a.p.drain) {
    case kDrainChunk: k_step<MAXT, GAL, kDrainChunk><<<grid, block, lds, s>>>(a); break;
    case kDrainPatch: k_step<MAXT, GAL, kDrainPatch><<<grid, block, lds, s>>>(a); break;
    default: k_step<MAXT, GAL, kDrainDeferred><<<grid, block, lds, s>>>(a); break;
  }
}

template <typename K>
static hipError_t blocked_occupancy_one(K kernel, uint32_t lds, int &blocks) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e) return e;
  int b = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, 1024, lds);
  blocks = std::min(blocks, b);
  return e;
}

hipError_t step_blocked_occupancy(const Schedule &sch, uint32_t lds_bytes, uint32_t n_cu,
                                  uint32_t &max_blocks) {
  if (sch.groups != 1 || sch.threads != 1024) return hipErrorInvalidValue;
  const uint32_t lds = step_lds_bytes(sch, lds_bytes);
  int b = 1 << 30;
  hipError_t e = blocked_occupancy_one(k_step_tb<1024, false>, lds, b);
  if (!e) e = blocked_occupancy_one(k_step_tb<1024, true>, lds, b);
  if (!e) e = blocked_occupancy_one(k_step_tt<1024, false>, lds, b);
  if (!e) e = blocked_occupancy_one(k_step_tt<1024, true>, lds, b);
  if (!e) e = blocked_occupancy_one(k_step_tr<1024, false, kDrainDeferred>, lds, b);
  if (!e) e = blocked_occupancy_one(k_step_tr<1024, true, kDrainDeferred>, lds, b);
  if (!e) e = blocked_occupancy_one(k_step_tr<1024, false, kDrainPatch>, lds, b);
  if (!e) e = blocked_occupancy_one(k_step_tr<1024, true, kDrainPatch>, lds, b);
  if (e) return e;
  if (b < 1) return hipErrorInvalidConfiguration;
  max_blocks = (uint32_t)b * n_cu;
  return hipSuccess;
}

hipError_t launch_step_blocked(const Schedule &sch, hipStream_t s, const StepLaunch &a,
                               const TbLaunch &tb, uint32_t grid) {
  if (tb.reps) {
    if (sch.groups != 1 || sch.threads != 1024 || tb.steps == 0 || !tb.scratch ||
        tb.bstride < 3ull * tb.stride || 6ull * tb.stride >= (1ull << 31))
      return hipErrorInvalidValue;
  } else if (sch.groups != 1 || sch.threads != 1024 || !a.single || tb.steps == 0 ||
      tb.steps > tb.kh || tb.stride < tb.es || tb.bstride < 3ull * tb.stride ||
      tb.es != (tb.T ? tb.T : tb.R) + 2u * tb.kh)
    return hipErrorInvalidValue;
  // tiles: the copy area, two carries and two side areas per block, each
  // block's areas addressed with 32-bit byte offsets; no logs
  if (tb.T && (tb.bstride < 3ull * tb.stride + 18ull * tb.kh ||
               2ull * tb.bstride * grid >= (1ull << 31) || tb.n_logs))
    return hipErrorInvalidValue;
  if (!tb.bar) return hipErrorInvalidValue;
  if (tb.n_logs && (tb.log < 1u || tb.log > 5u || !tb.records || !tb.out || tb.log_first < 1u ||
                    tb.log_every < 1u || tb.log_first + (tb.n_logs - 1u) * tb.log_every > tb.steps ||
                    (tb.log >= 3u && !tb.tw)))
    return hipErrorInvalidValue;
  // logs before the last step: not with the digest or the Galilean acceptance
  if (tb.n_logs && tb.log_first < tb.steps && ((tb.log & 1u) == 0u || a.p.galilean))
    return hipErrorInvalidValue;
  const uint32_t lds = step_lds_bytes(sch, a.lds_bytes);
  StepLaunch av = a;
  TbLaunch tv = tb;
  void *args[] = {&av, &tv};
  const void *f = tb.T ? (a.p.galilean ? reinterpret_cast<const void *>(k_step_tt<1024, true>)
                                       : reinterpret_cast<const void *>(k_step_tt<1024, false>))
                       : (a.p.galilean ? reinterpret_cast<const void *>(k_step_tb<1024, true>)
                                       : reinterpret_cast<const void *>(k_step_tb<1024, false>));
  if (tb.reps) {
    // replicas: an ordinary launch (no grid-wide barrier)
    if (!tb.items || !tb.item_first || tb.n_logs) return hipErrorInvalidValue;
    // misses resolved per chunk (patched) or per step (deferred)
    const bool patch = a.p.drain == kDrainPatch;
    if (a.p.galilean) {
      if (patch) k_step_tr<1024, true, kDrainPatch><<<grid, 1024, lds, s>>>(a, tb);
      else k_step_tr<1024, true, kDrainDeferred><<<grid, 1024, lds, s>>>(a, tb);
    } else {
      if (patch) k_step_tr<1024, false, kDrainPatch><<<grid, 1024, lds, s>>>(a, tb);
      else k_step_tr<1024, false, kDrainDeferred><<<grid, 1024, lds, s>>>(a, tb);
    }
    return hipGetLastError();
  }
  return hipLaunchCooperativeKernel(f, dim3(grid), dim3(1024), args, lds, s);
}

hipError_t launch_step(const Schedule &sch, hipStream_t s, const StepLaunch &a) {
  if (a.n_tiles == 0) return hipSuccess;
  dim3 grid(std::max<uint32_t>(1, std::min(a.n_tiles, a.max_blocks))), block(sch.threads);
  const uint32_t lds = step_lds_bytes(sch, a.lds_bytes);
  if (sch.groups != 1) return hipErrorInvalidValue;
  if (a.p.drain > kDrainPatch) return hipErrorInvalidValue;
  const bool small = sch.threads <= 512;
  if (a.p.galilean) {
    if (small) launch_mode<512, true>(grid, block, lds, s, a);
    else launch_mode<1024, true>(grid, block, lds, s, a);
  } else {
    if (small) launch_mode<512, false>(grid, block, lds, s, a);
    else launch_mode<1024, false>(grid, block, lds, s, a);
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

hipError_t launch_histogram(hipStream_t s, const uint16_t *state, const SlotDev *slots,
                            const TileDev *tiles, uint32_t n_tiles, uint32_t tile_sites,
                            uint32_t n_bins, unsigned long long *hist) {
  if (n_tiles == 0) return hipSuccess;
  const uint32_t blocks = std::min<uint32_t>(n_tiles, 2048u);
  k_histogram<<<blocks, 256, 3u * n_bins * sizeof(uint32_t), s>>>(state, slots, tiles, n_tiles,
                                                                  tile_sites, n_bins, hist);
  return hipGetLastError();
}

hipError_t launch_add_t(hipStream_t s, uint32_t *tslot, uint32_t slot_first, uint32_t n,
                        uint32_t add) {
  if (n == 0 || add == 0) return hipSuccess;
  k_add_t<<<std::min<uint32_t>(64, (n + 255) / 256), 256, 0, s>>>(tslot, slot_first, n, add);
  return hipGetLastError();
}

hipError_t launch_set_t(hipStream_t s, uint32_t *tslot, const uint32_t *slot_list, uint32_t n,
                        uint32_t value) {
  if (n == 0) return hipSuccess;
  k_set_t<<<1, 256, 0, s>>>(tslot, slot_list, n, value);
  return hipGetLastError();
}

}  // namespace mclg
