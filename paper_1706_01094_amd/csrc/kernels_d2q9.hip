// HIP kernels of the D2Q9 path of the MCLG library (Sec. "A D2Q9
// implementation"): one thread per site runs the literal loop of C
// sub-collisions with the rule table in LDS, in place in the shifted 2D
// layout; Poisson start, counts start, exact moments and histograms.  The
// rules and the layout are stated in mclg.h.
#include "d2q9.h"
#include "device.h"
#include "rng.h"

#include <algorithm>

namespace mclg {
namespace {

// ---- D2Q9 --------------------------------------------------------------
// Step9::rules holds the rules in the form device_rules9 builds (d2q9.h):
// kRule9DevWords per ordered source pair.
__constant__ int32_t kV9x[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int32_t kV9y[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Physical element of velocity i of logical site s = y Lx + x at shift
// (tx, ty): ((x - vx tx) mod Lx, (y - vy ty) mod Ly), element y' Lx + x'.
// The row offsets y' Lx are (y Lx -/+ ty Lx) mod S, with y Lx = s - x.
struct Site9 {
  uint32_t e[9];
  __device__ Site9(uint32_t s, uint32_t x, uint32_t tx, uint32_t ty, uint32_t Lx, uint32_t S) {
    const uint32_t xs[3] = {x + tx >= Lx ? x + tx - Lx : x + tx, x, x >= tx ? x - tx : x + Lx - tx};
    const uint32_t yL = s - x, tyL = ty * Lx;
    const uint32_t rows[3] = {yL + tyL >= S ? yL + tyL - S : yL + tyL, yL,
                              yL >= tyL ? yL - tyL : yL + S - tyL};
#pragma unroll
    for (int i = 0; i < 9; ++i) e[i] = rows[kV9y[i] + 1] + xs[kV9x[i] + 1];
  }
};

// Packed pairs of 16-bit partial sums (element 0 = low half).
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// #{j < 8 : K_j <= r} for the partial sums K held as four 16-bit pairs and
// r < 65535: max(0, r + 1 - K_j) is at least 1 exactly when K_j <= r.  `one`
// holds 1 in both halves; passed in a register it keeps the saturated
// difference and the minimum as two packed instructions per pair.
__device__ __forceinline__ uint32_t count_partial_le(const u16x2 (&K)[4], uint32_t r, u16x2 one) {
  const u16x2 R = as_u16x2((r + 1u) * 0x10001u);
  u16x2 acc = __builtin_elementwise_min(__builtin_elementwise_sub_sat(R, K[0]), one);
#pragma unroll
  for (int m = 1; m < 4; ++m) acc += __builtin_elementwise_min(__builtin_elementwise_sub_sat(R, K[m]), one);
  return (uint32_t)acc.x + (uint32_t)acc.y;
}

// One step of every site of one tile: the literal loop of C sub-collisions
// (Eq. (select), Eq. (omega) with the D2Q9 rules), in place in the shifted
// layout.  Sites with N < 2 (or C = 0) are left untouched.  The loop keeps
// the partial sums K_j = n_0 + ... + n_j (j < 8) as packed 16-bit pairs: the
// velocity of particle r is #{j : K_j <= r}, and a collision adds one of the
// rule table's packed changes.
__global__ void __launch_bounds__(256) k_step9(Step9 a) {
  __shared__ __align__(16) uint4 rules[81 * kRule9DevWords / 4];
  const uint4 *src = reinterpret_cast<const uint4 *>(a.rules);
  for (uint32_t i = threadIdx.x; i < 81 * kRule9DevWords / 4; i += blockDim.x) rules[i] = src[i];
  __syncthreads();
  const Tile9 tile = a.tiles[blockIdx.x];
  const Rep9 rp = a.reps[tile.rep];
  const uint32_t s = tile.s0 + threadIdx.x;
  if (s >= rp.S) return;
  const uint32_t y = s / rp.Lx, x = s - y * rp.Lx;
  const uint32_t tx = a.no_stream ? 0u : (uint32_t)(a.t % rp.Lx);
  const uint32_t ty = a.no_stream ? 0u : (uint32_t)(a.t % rp.Ly);
  const Site9 ph(s, x, tx, ty, rp.Lx, rp.S);
  uint16_t *base = a.state + rp.off;
  uint32_t n[9], N = 0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    n[i] = base[(uint64_t)i * rp.stride + ph.e[i]];
    N += n[i];
  }
  if (N > 65535u) {
    atomicOr(a.err, kErrOverflow);
    return;
  }
  if (N < 2u || a.C <= 0) return;
  u16x2 K[4];
  {
    uint32_t k = 0, lo;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      k += n[2 * m];
      lo = k;
      k += n[2 * m + 1];
      K[m] = as_u16x2(lo | k << 16);
    }
  }
  // Sub-collision k reads Philox block (s, t, replica, 2 | k << 2): words 0,
  // 1, 2 draw the first particle, the second and the target; a rejected
  // draw continues on the blocks (s, t, replica, 2 | (C + j) << 2).
  const uint2 key = make_uint2((uint32_t)a.seed, (uint32_t)(a.seed >> 32));
  WordStream more;
  more.key = key;
  more.x = s; more.t = (uint32_t)a.t; more.rid = rp.rid;
  more.block = (uint32_t)a.C; more.used = 4;
  uint32_t one_ = 0x10001u, one32_ = 1u;
  // opaque constants: no compare-and-select rewrite of the minima below
  asm volatile("" : "+v"(one_), "+v"(one32_));
  const u16x2 one = as_u16x2(one_);
  for (int32_t sub = 0; sub < a.C; ++sub) {
    const uint4 w = philox10(make_uint4(s, (uint32_t)a.t, rp.rid, 2u | ((uint32_t)sub << 2)), key);
    uint32_t r1 = more.uniform_from(w.x, N);
    uint32_t r2 = more.uniform_from(w.y, N - 1);
    const uint32_t u = more.uniform_from(w.z, a.D);
    asm volatile("" : "+v"(r1), "+v"(r2));  // compared as 32-bit values
    r2 += (r2 >= r1);
    const uint32_t v1 = count_partial_le(K, r1, one), v2 = count_partial_le(K, r2, one);
    const uint32_t rec = (v1 * 9u + v2) * (kRule9DevWords / 4);
    const uint4 c = rules[rec];
    // q = #{cumulative weights <= u} (u + 1 <= D < 2^32)
    const uint32_t u1 = u + 1u, one32 = one32_;
    uint32_t q = __builtin_elementwise_min(__builtin_elementwise_sub_sat(u1, c.x), one32) +
                       __builtin_elementwise_min(__builtin_elementwise_sub_sat(u1, c.y), one32) +
                       __builtin_elementwise_min(__builtin_elementwise_sub_sat(u1, c.z), one32) +
                       __builtin_elementwise_min(__builtin_elementwise_sub_sat(u1, c.w), one32);
    asm volatile("" : "+v"(q));  // one shift for the record offset
    const uint4 d = rules[rec + 1u + q];
    K[0] += as_u16x2(d.x);
    K[1] += as_u16x2(d.y);
    K[2] += as_u16x2(d.z);
    K[3] += as_u16x2(d.w);
  }
  uint32_t prev = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const uint32_t k = as_u32(K[m]), lo = k & 0xFFFFu, hi = k >> 16;
    n[2 * m] = lo - prev;
    n[2 * m + 1] = hi - lo;
    prev = hi;
  }
  n[8] = N - prev;
#pragma unroll
  for (int i = 0; i < 9; ++i) base[(uint64_t)i * rp.stride + ph.e[i]] = (uint16_t)n[i];
}

// Poisson start: site s draws Philox blocks (s, j, replica, 1), j = 0, 1, 2;
// word w of block j serves velocity 4 j + w.  At t = 0 the layout is
// unshifted.
__global__ void __launch_bounds__(256) k_init9_poisson(
    uint16_t *__restrict__ state, const Rep9 *__restrict__ reps, const Tile9 *__restrict__ tiles,
    const PoisDesc *__restrict__ desc, const uint32_t *__restrict__ pool, uint64_t seed,
    uint32_t *err) {
  const Tile9 tile = tiles[blockIdx.x];
  const Rep9 rp = reps[tile.rep];
  const uint32_t s = tile.s0 + threadIdx.x;
  if (s >= rp.S) return;
  const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
#pragma unroll
  for (uint32_t j = 0; j < 3; ++j) {
    const uint4 w = philox10(make_uint4(s, j, rp.rid, 1u), key);
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t i = 4 * j + q;
      if (i >= 9) break;
      const PoisDesc d = desc[9u * tile.rep + i];
      const uint32_t n = d.k_first + count_le(pool + d.off, d.nthr, word_of(w, q));
      if (n > 65535u) atomicOr(err, kErrOverflow);
      state[rp.off + (uint64_t)i * rp.stride + s] = (uint16_t)n;
    }
  }
}

// Counts given in logical order ([9][Ly][Lx] per replica, replicas packed
// from dense[rep]); at t = 0 the layout is unshifted.
__global__ void __launch_bounds__(256) k_init9_counts(uint16_t *__restrict__ state,
                                                      const Rep9 *__restrict__ reps,
                                                      const Tile9 *__restrict__ tiles,
                                                      const uint64_t *__restrict__ dense,
                                                      const uint16_t *__restrict__ counts) {
  const Tile9 tile = tiles[blockIdx.x];
  const Rep9 rp = reps[tile.rep];
  const uint32_t s = tile.s0 + threadIdx.x;
  if (s >= rp.S) return;
  const uint16_t *src = counts + dense[tile.rep];
#pragma unroll
  for (uint32_t i = 0; i < 9; ++i)
    state[rp.off + (uint64_t)i * rp.stride + s] = src[(uint64_t)i * rp.S + s];
}

// Occupation-number histograms of D2Q9 replicas, as k_histogram: each block
// takes a run of tiles, bins the nine arrays of their sites in LDS and adds
// the non-empty bins to its replica's row whenever the run changes replica.
__global__ void __launch_bounds__(256) k_histogram9(const uint16_t *__restrict__ state,
                                                    const Rep9 *__restrict__ reps,
                                                    const Tile9 *__restrict__ tiles,
                                                    uint32_t n_tiles, uint32_t n_bins,
                                                    unsigned long long *__restrict__ hist) {
  extern __shared__ uint32_t bins[];  // [9][n_bins]
  const uint32_t per = (n_tiles + gridDim.x - 1u) / gridDim.x;
  const uint32_t t_begin = blockIdx.x * per, t_end = min(n_tiles, t_begin + per);
  if (t_begin >= t_end) return;
  const uint32_t nb9 = 9u * n_bins, top = n_bins - 1u;
  for (uint32_t j = threadIdx.x; j < nb9; j += blockDim.x) bins[j] = 0u;
  uint32_t cur = tiles[t_begin].rep;
  auto flush = [&](uint32_t rep) {
    __syncthreads();
    unsigned long long *row = hist + (uint64_t)rep * nb9;
    for (uint32_t j = threadIdx.x; j < nb9; j += blockDim.x) {
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
    const Tile9 tile = tiles[t];
    if (tile.rep != cur) {
      flush(cur);
      cur = tile.rep;
    }
    const Rep9 rp = reps[tile.rep];
    const uint32_t s = tile.s0 + threadIdx.x;
    if (s < rp.S) {
#pragma unroll
      for (uint32_t i = 0; i < 9u; ++i) {
        const uint32_t n = state[rp.off + (uint64_t)i * rp.stride + s];
        atomicAdd(&bins[i * n_bins + min(n, top)], 1u);
      }
    }
  }
  flush(cur);
}

}  // namespace

hipError_t launch_step9(hipStream_t s, const Step9 &a, uint32_t n_tiles) {
  if (n_tiles == 0) return hipSuccess;
  k_step9<<<n_tiles, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_init9_poisson(hipStream_t s, uint16_t *state, const Rep9 *reps,
                                const Tile9 *tiles, uint32_t n_tiles, const PoisDesc *desc,
                                const uint32_t *pool, uint64_t seed, uint32_t *err) {
  if (n_tiles == 0) return hipSuccess;
  k_init9_poisson<<<n_tiles, 256, 0, s>>>(state, reps, tiles, desc, pool, seed, err);
  return hipGetLastError();
}

hipError_t launch_init9_counts(hipStream_t s, uint16_t *state, const Rep9 *reps,
                               const Tile9 *tiles, uint32_t n_tiles, const uint64_t *dense,
                               const uint16_t *counts) {
  if (n_tiles == 0) return hipSuccess;
  k_init9_counts<<<n_tiles, 256, 0, s>>>(state, reps, tiles, dense, counts);
  return hipGetLastError();
}

hipError_t launch_histogram9(hipStream_t s, const uint16_t *state, const Rep9 *reps,
                             const Tile9 *tiles, uint32_t n_tiles, uint32_t n_bins,
                             unsigned long long *hist) {
  if (n_tiles == 0) return hipSuccess;
  const uint32_t blocks = std::min<uint32_t>(n_tiles, 2048u);
  k_histogram9<<<blocks, 256, 9u * n_bins * sizeof(uint32_t), s>>>(state, reps, tiles, n_tiles,
                                                                   n_bins, hist);
  return hipGetLastError();
}

}  // namespace mclg
