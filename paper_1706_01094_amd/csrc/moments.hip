// Exact moment sums of the MCLG state: the observables of the paper's
// statistics -- sums of n_i and n_i n_j for the Poisson and correlation
// checks (Eq. (poisson), Eq. (corr)), N and J for the conserved mass and
// momentum, Fourier projections of the density for the decaying density wave
// (Eq. (A)) and S(k) -- plus a digest of the whole state for comparing runs.
//
// One block per segment of a slot's sites accumulates in registers (each
// lane eight consecutive sites per pass, 16-byte loads from the shifted
// layout), reduces its sums once, and writes one partial record; a second
// kernel adds a replica's records.  No atomics, nothing to clear, and the
// result is independent of the split (integer sums modulo 2^64).
#include "moments.h"
#include "mom3_sum.h"
#include "rng.h"

#include <algorithm>
#include <mutex>

namespace mclg {
namespace {

using namespace mom3;
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format

__device__ __forceinline__ Rsrc make_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, kRsrcWord3);
}
__device__ __forceinline__ void load16(Rsrc r, uint32_t off, uint32_t (&v)[4]) {
  const auto q = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
  v[0] = q[0]; v[1] = q[1]; v[2] = q[2]; v[3] = q[3];
}
__device__ __forceinline__ uint32_t load2(Rsrc r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
}

// One segment's partial record from its block's lanes (block_record over
// this kernel's LDS).
template <int V, int W, int MS>
__device__ __forceinline__ void write_partial(u64 (&v)[V], uint32_t mx, u64 *rec) {
  __shared__ u64 red[16 * V];
  __shared__ uint32_t redmx[16];
  block_record<V, W, MS>(v, mx, rec, red, redmx);
}

// ---- D1Q3 ----------------------------------------------------------------
// The eight sites x .. x+7 of a lane in logical order: n_-1 from physical
// (x + tm) mod L, n_0 from x, n_+1 from (x - tm) mod L, two sites per 32-bit
// word; sites at or past L read as zero.  Returns how many of the eight exist.
__device__ __forceinline__ uint32_t load_eight(Rsrc rs, uint32_t ab, uint32_t L, uint32_t tm,
                                               uint32_t x, uint32_t (&va)[4], uint32_t (&vb)[4],
                                               uint32_t (&vc)[4]) {
  uint32_t pm = x + tm;
  pm -= (pm >= L) ? L : 0u;
  const uint32_t pp = x >= tm ? x - tm : x + L - tm;
  if (x + 8u <= L && pm + 8u <= L && pp + 8u <= L) {
    load16(rs, 2u * pm, va);
    load16(rs, ab + 2u * x, vb);
    load16(rs, 2u * ab + 2u * pp, vc);
    return 8u;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) va[j] = vb[j] = vc[j] = 0u;
#pragma unroll
  for (uint32_t e = 0; e < 8u; ++e) {
    const uint32_t xe = x + e;
    if (xe < L) {
      uint32_t m = xe + tm;
      m -= (m >= L) ? L : 0u;
      const uint32_t p = xe >= tm ? xe - tm : xe + L - tm;
      const uint32_t sh = 16u * (e & 1u);
      va[e >> 1] |= load2(rs, 2u * m) << sh;
      vb[e >> 1] |= load2(rs, ab + 2u * xe) << sh;
      vc[e >> 1] |= load2(rs, 2u * ab + 2u * p) << sh;
    }
  }
  return x < L ? min(8u, L - x) : 0u;
}

template <int NM>
__device__ __forceinline__ void load_window(Rsrc rs, uint32_t ab, uint32_t L, uint32_t tm,
                                            uint32_t x, const int32_t *tw, Eight<NM> &E) {
  E.x = x;
  E.n = load_eight(rs, ab, L, tm, x, E.a, E.b, E.c);
#pragma unroll
  for (int r = 0; r < Eight<NM>::PR; ++r) load_tw8(tw + (uint64_t)r * L + x, E.n, E.w[r]);
}

// Whether the eight sites x .. x + 7 are all in the lattice and none of
// their three shifted windows wraps around its end.
__device__ __forceinline__ bool window_fast(uint32_t L, uint32_t tm, uint32_t x) {
  uint32_t pm = x + tm;
  pm -= (pm >= L) ? L : 0u;
  const uint32_t pp = x >= tm ? x - tm : x + L - tm;
  return x + 8u <= L && pm + 8u <= L && pp + 8u <= L;
}

// The loads of a window without a branch, for the pipelined passes: a fast
// window loads its vectors; any other loads from in-bounds offset 0 and is
// cleared by clear_slow once its loads have arrived (its sites are summed
// afterwards on the element-wise path).
template <int NM>
__device__ __forceinline__ void issue_fast(Rsrc rs, uint32_t ab, uint32_t L, uint32_t tm,
                                           uint32_t x, Rsrc twr, Eight<NM> &E) {
  uint32_t pm = x + tm;
  pm -= (pm >= L) ? L : 0u;
  const uint32_t pp = x >= tm ? x - tm : x + L - tm;
  const bool f = x + 8u <= L && pm + 8u <= L && pp + 8u <= L;
  load16(rs, f ? 2u * pm : 0u, E.a);
  load16(rs, f ? ab + 2u * x : 0u, E.b);
  load16(rs, f ? 2u * ab + 2u * pp : 0u, E.c);
#pragma unroll
  for (int r = 0; r < Eight<NM>::PR; ++r) {
    const uint32_t o = 4u * ((uint32_t)r * L + (f ? x : 0u));
    uint32_t q[4];
    load16(twr, o, q);
#pragma unroll
    for (int e = 0; e < 4; ++e) E.w[r][e] = (int32_t)q[e];
    load16(twr, o + 16u, q);
#pragma unroll
    for (int e = 0; e < 4; ++e) E.w[r][4 + e] = (int32_t)q[e];
  }
  E.x = x;
  E.n = f ? 8u : 0u;
}
template <int NM>
__device__ __forceinline__ void clear_slow(Eight<NM> &E) {
  const bool f = E.n != 0u;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    E.a[j] = f ? E.a[j] : 0u;
    E.b[j] = f ? E.b[j] : 0u;
    E.c[j] = f ? E.c[j] : 0u;
  }
}

template <int NM, bool DIG>
__global__ void __launch_bounds__(256) k_mom3(const uint16_t *__restrict__ state,
                                              const SlotDev *__restrict__ slots,
                                              const uint32_t *__restrict__ tslot,
                                              const MomSeg *__restrict__ segs, uint32_t no_stream,
                                              const int32_t *__restrict__ twiddle,
                                              u64 *__restrict__ partial) {
  const MomSeg sg = segs[blockIdx.x];
  const SlotDev sl = slots[sg.slot];
  const uint32_t L = sl.L;
  const uint32_t tm = no_stream ? 0u : tslot[sg.slot] % L;
  const Rsrc rs = make_rsrc(state + sl.off, 6u * sl.stride);
  const uint32_t ab = 2u * sl.stride;
  const int32_t *tw = NM > 0 ? twiddle + 2ull * NM * sl.dense : nullptr;
  Acc3<NM> A;
  acc_clear<NM>(A);
  const uint32_t step = 8u * blockDim.x;
  const uint32_t xb = sg.x0 + 8u * threadIdx.x;
  // Full passes (every lane's eight sites inside the segment) go in batches
  // of U passes, software-pipelined over two register sets: a batch's loads
  // are issued before the previous batch is summed.  Every batch issues the
  // same loads whatever its windows, so each wait covers exactly the batch
  // being summed.  Segments hold a multiple of 2 U passes except a run's
  // last; what the batches leave is summed on the element-wise path.
  constexpr int U = NM == 0 && !DIG ? 4 : NM == 1 && !DIG ? 2 : 1;
  // (more than two modes, or twiddle rows too long for 32-bit byte offsets:
  // one pass at a time, unpipelined)
  const bool pipelined = NM == 0 || (NM <= 2 && 8ull * NM * L < (1ull << 31));
  const uint32_t nb2 = pipelined ? ((sg.x1 - sg.x0) / step / U) & ~1u : 0u;  // batches, even
  if (nb2) {
    // the slot's twiddle rows through a buffer resource (at most 2 modes x 2
    // rows of L int32, below 2^31 bytes when pipelined)
    const Rsrc twr = make_rsrc(NM > 0 ? tw : nullptr, NM > 0 ? 8u * NM * L : 0u);
    Eight<NM> E0[U], E1[U];
    // (the scheduling barrier keeps the sums of the previous batch from
    // being hoisted above these loads, which would wait for that batch first)
    auto issue = [&](Eight<NM>(&E)[U], uint32_t b) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u) issue_fast<NM>(rs, ab, L, tm, xb + (b * U + u) * step, twr, E[u]);
      __builtin_amdgcn_sched_barrier(0);
    };
    auto sum = [&](Eight<NM>(&E)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        clear_slow<NM>(E[u]);
        add_eight<NM, DIG>(A, E[u], tw, L);
      }
    };
    // (after the last pair the loop loads batch nb2 - 1 once more, from
    // the L2, and does not sum it: no iteration ends differently)
    issue(E0, 0);
    for (uint32_t b = 0; b < nb2; b += 2) {
      issue(E1, b + 1);
      sum(E0);
      issue(E0, min(b + 2, nb2 - 1));
      sum(E1);
    }
    // the windows of those passes that wrap (at most three per lattice)
    for (uint32_t q = 0; q < nb2 * U; ++q) {
      const uint32_t x = xb + q * step;
      if (!window_fast(L, tm, x)) {
        Eight<NM> E;
        load_window<NM>(rs, ab, L, tm, x, tw, E);
        add_eight<NM, DIG>(A, E, tw, L);
      }
    }
  }
  for (uint32_t x = xb + nb2 * U * step; x < sg.x1; x += step) {
    Eight<NM> E;
    load_window<NM>(rs, ab, L, tm, x, tw, E);
    add_eight<NM, DIG>(A, E, tw, L);
  }
  // record slots: the 11 sums, the maximum, then the Fourier sums
  constexpr int W = 12 + 2 * NM;
  constexpr int V = W <= 16 ? 16 : 32;
  u64 v[V];
  const uint32_t mx = fold<NM, V>(A, v);
  write_partial<V, W, 11>(v, mx, partial + (uint64_t)blockIdx.x * kMom3Rec);
}

// Sums of the partial records [s0, s1) of one run in the final pass (one
// block per run): the block's threads form G = blockDim / (REC / 2) groups
// of REC / 2; thread p of group g loads values 2p and 2p + 1 of records
// s0 + g, s0 + g + G, ... with 16-byte loads, eight in flight (pairs at or
// past npairs are not read), and the groups are added in LDS.  Value MS is
// a maximum, the others are sums modulo 2^64.  tot[k] holds value k after.
template <int REC, int MS>
__device__ __forceinline__ void sum_run(const u64 *__restrict__ partial, uint32_t s0,
                                        uint32_t s1, uint32_t npairs, u64 *tot) {
  constexpr uint32_t P = REC / 2;
  __shared__ u64 red[2][1024];
  const uint32_t G = blockDim.x / P;
  const uint32_t p = threadIdx.x % P, g = threadIdx.x / P;
  const bool m0 = 2u * p == (uint32_t)MS, m1 = 2u * p + 1u == (uint32_t)MS;
  u64 a0 = 0, a1 = 0;
  auto add = [&](uint4 q) {
    const u64 v0 = ((u64)q.y << 32) | q.x, v1 = ((u64)q.w << 32) | q.z;
    a0 = m0 ? max(a0, v0) : a0 + v0;
    a1 = m1 ? max(a1, v1) : a1 + v1;
  };
  if (p < npairs) {
    const uint4 *base = reinterpret_cast<const uint4 *>(partial) + p;
    uint32_t r = s0 + g;
    for (; r + 7u * G < s1; r += 8u * G) {
      uint4 q[8];
#pragma unroll
      for (uint32_t i = 0; i < 8u; ++i) q[i] = base[(uint64_t)(r + i * G) * P];
#pragma unroll
      for (uint32_t i = 0; i < 8u; ++i) add(q[i]);
    }
    for (; r < s1; r += G) add(base[(uint64_t)r * P]);
  }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  __syncthreads();
  if (threadIdx.x < 2u * P) {
    const uint32_t k = threadIdx.x, h = k & 1u, q = k >> 1;
    u64 t = 0;
    for (uint32_t gg = 0; gg < G; ++gg) {
      const u64 v = red[h][gg * P + q];
      t = k == (uint32_t)MS ? max(t, v) : t + v;
    }
    tot[k] = t;
  }
  __syncthreads();
}

// Final pass, one block per run j: the replica's result in the field order
// of mclg_moments_t (result_field), t from the device step counter.
__global__ void __launch_bounds__(1024) k_mom3_final(const u64 *__restrict__ partial,
                                                     const uint32_t *__restrict__ run_seg,
                                                     const uint32_t *__restrict__ run_slot,
                                                     const SlotDev *__restrict__ slots,
                                                     const uint32_t *__restrict__ tslot,
                                                     uint32_t n_modes, i64 *__restrict__ out) {
  __shared__ u64 T[kMom3Rec];
  const uint32_t j = blockIdx.x, slot = run_slot[j];
  sum_run<kMom3Rec, 11>(partial, run_seg[j], run_seg[j + 1], 6u + n_modes, T);
  const uint32_t k = threadIdx.x;
  if (k >= kMom3Out) return;
  out[(uint64_t)j * kMom3Out + k] =
      (i64)result_field(k, T, k == 0u ? tslot[slot] : 0u, k == 1u ? slots[slot].L : 0u, n_modes);
}

// ---- D2Q9 ----------------------------------------------------------------
__constant__ int32_t kVx9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int32_t kVy9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// One block per segment of a replica's sites s = y Lx + x; each lane takes
// eight consecutive sites of a row per pass.  Logical n_i(x, y, t) sits at
// physical ((x - vx t) mod Lx, (y - vy t) mod Ly), so eight sites of a row
// are eight consecutive elements of each array unless a shifted window wraps
// around Lx: one 16-byte load per velocity (nine per pass), else element by
// element.  Windows whose counts are all below 256 add the 9 sums and 45
// products n_i n_j with packed dot products into 32-bit sums (each adds at
// most 8 x 255^2 per window; a lane sums at most 2^23 / 2048 windows of a
// segment); other windows add each site's exact products to 64-bit sums in
// LDS.
__device__ __forceinline__ void load_row9(Rsrc rs, uint32_t stride, uint32_t Lx, uint32_t Ly,
                                          uint32_t tx, uint32_t ty, uint32_t x, uint32_t y,
                                          uint32_t (&w)[9][4]) {
  const uint32_t xc[3] = {x + tx >= Lx ? x + tx - Lx : x + tx, x, x >= tx ? x - tx : x + Lx - tx};
  const uint32_t yr[3] = {(y + ty >= Ly ? y + ty - Ly : y + ty) * Lx, y * Lx,
                          (y >= ty ? y - ty : y + Ly - ty) * Lx};
#pragma unroll
  for (int i = 0; i < 9; ++i)
    load16(rs, 2u * ((uint32_t)i * stride + yr[kVy9[i] + 1] + xc[kVx9[i] + 1]), w[i]);
}

__global__ void __launch_bounds__(256) k_mom9(const uint16_t *__restrict__ state,
                                              const Rep9 *__restrict__ reps, uint64_t t,
                                              uint32_t no_stream,
                                              const MomSeg *__restrict__ segs,
                                              u64 *__restrict__ partial) {
  __shared__ u64 big[45];
  __shared__ u64 red64[4][64];
  __shared__ uint32_t redmx[4];
  for (uint32_t k = threadIdx.x; k < 45u; k += blockDim.x) big[k] = 0;
  __syncthreads();
  const MomSeg sg = segs[blockIdx.x];
  const Rep9 rp = reps[sg.slot];
  const uint32_t Lx = rp.Lx, Ly = rp.Ly;
  const uint32_t tx = no_stream ? 0u : (uint32_t)(t % Lx);
  const uint32_t ty = no_stream ? 0u : (uint32_t)(t % Ly);
  const Rsrc rs = make_rsrc(state + rp.off, 18u * rp.stride);
  const uint32_t stride = rp.stride;
  uint32_t acc[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) acc[k] = 0;
  uint32_t mx = 0, mxp = 0;
  const uint32_t step = 8u * blockDim.x;
  for (uint32_t s = sg.x0 + 8u * threadIdx.x; s < sg.x1; s += step) {
    const uint32_t y = s / Lx, x = s - y * Lx;
    uint32_t w[9][4];
    const uint32_t xm = x + tx >= Lx ? x + tx - Lx : x + tx, xp = x >= tx ? x - tx : x + Lx - tx;
    const bool fast = s + 8u <= sg.x1 && x + 8u <= Lx && xm + 8u <= Lx && xp + 8u <= Lx;
    if (fast) {
      load_row9(rs, stride, Lx, Ly, tx, ty, x, y, w);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) w[i][j] = 0;
      uint32_t xe = x, ye = y;
#pragma unroll
      for (uint32_t e = 0; e < 8u; ++e) {
        if (s + e < sg.x1) {
          const uint32_t xc[3] = {xe + tx >= Lx ? xe + tx - Lx : xe + tx, xe,
                                  xe >= tx ? xe - tx : xe + Lx - tx};
          const uint32_t yr[3] = {(ye + ty >= Ly ? ye + ty - Ly : ye + ty) * Lx, ye * Lx,
                                  (ye >= ty ? ye - ty : ye + Ly - ty) * Lx};
#pragma unroll
          for (int i = 0; i < 9; ++i)
            w[i][e >> 1] |= load2(rs, 2u * ((uint32_t)i * stride + yr[kVy9[i] + 1] +
                                            xc[kVx9[i] + 1])) << (16u * (e & 1u));
        }
        if (++xe == Lx) { xe = 0; ++ye; }
      }
    }
    uint32_t any = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) any |= w[i][0] | w[i][1] | w[i][2] | w[i][3];
    if ((any & 0xff00ff00u) == 0u) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        u16x2 n2 = {0, 0};
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          acc[i] = dot2(w[i][j], 0x00010001u, acc[i]);
          n2 += __builtin_bit_cast(u16x2, w[i][j]);
        }
        int k = 9;
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
          for (int l = i; l < 9; ++l) { acc[k] = dot2(w[i][j], w[l][j], acc[k]); ++k; }
        mxp = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, mxp), n2));
      }
    } else {
#pragma unroll
      for (uint32_t e = 0; e < 8u; ++e) {
        uint32_t n[9], N = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          n[i] = (w[i][e >> 1] >> (16u * (e & 1u))) & 0xffffu;
          N += n[i];
          acc[i] += n[i];
        }
        mx = max(mx, N);
        int k = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
          for (int l = i; l < 9; ++l) {
            if (n[i] && n[l]) atomicAdd(&big[k], (u64)n[i] * n[l]);
            ++k;
          }
      }
    }
  }
  mx = max(mx, max(mxp & 0xffffu, mxp >> 16));
  // first level of the reduce-scatter in 32-bit inputs (lanes with bit 5
  // set keep values 32..63), then 64-bit sums
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  u64 v[32];
  {
    const bool up = (lane & 32u) != 0;
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      const uint32_t send = up ? acc[j] : acc[j + 32];
      const uint32_t keep = up ? acc[j + 32] : acc[j];
      v[j] = (u64)keep + (uint32_t)__shfl_xor(send, 32);
    }
  }
  int wd = 32, m = 16;
#pragma unroll
  for (int lvl = 0; lvl < 5; ++lvl) {
    const bool up = (lane & (uint32_t)m) != 0;
    const int h = wd >> 1;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j < h) {
        const u64 send = up ? v[j] : v[j + h];
        const u64 keep = up ? v[j + h] : v[j];
        v[j] = keep + shfl_xor_u64(send, m);
      }
    }
    wd = h;
    m >>= 1;
  }
  // lane l now holds the wave's total of value l
  mx = wave_max(mx);
  red64[wave][lane] = v[0];
  if (lane == 0) redmx[wave] = mx;
  __syncthreads();
  const uint32_t nw = blockDim.x >> 6;
  u64 *rec = partial + (uint64_t)blockIdx.x * kMom9Rec;
  for (uint32_t k = threadIdx.x; k < kMom9Used; k += blockDim.x) {
    u64 o = 0;
    if (k == kMom9Max) {
      uint32_t mm = 0;
      for (uint32_t q = 0; q < nw; ++q) mm = max(mm, redmx[q]);
      o = mm;
    } else if (k < 54u) {
      for (uint32_t q = 0; q < nw; ++q) o += red64[q][k];
      if (k >= 9u) o += big[k - 9u];
    }
    rec[k] = o;
  }
}

// Final pass, one block per run j: the replica's result in the field order
// of mclg_moments9_t: t, sites, sum n_i, sum n_i n_j (i <= j), sum N, sum
// Jx, sum Jy (from the per-velocity sums), max N.
__global__ void __launch_bounds__(1024) k_mom9_final(const u64 *__restrict__ partial,
                                                     const uint32_t *__restrict__ run_seg,
                                                     const uint32_t *__restrict__ run_slot,
                                                     const Rep9 *__restrict__ reps, uint64_t t,
                                                     i64 *__restrict__ out) {
  __shared__ u64 T[kMom9Rec];
  const uint32_t j = blockIdx.x, slot = run_slot[j];
  sum_run<kMom9Rec, kMom9Max>(partial, run_seg[j], run_seg[j + 1], kMom9Used / 2u, T);
  const uint32_t k = threadIdx.x;
  if (k >= kMom9Out) return;
  u64 v = 0;
  if (k == 0u) {
    v = t;
  } else if (k == 1u) {
    v = reps[slot].S;
  } else if (k < 56u) {
    v = T[k - 2u];
  } else if (k == 59u) {
    v = T[kMom9Max];
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i)
      v += (u64)(k == 56u ? 1 : k == 57u ? kVx9[i] : kVy9[i]) * T[i];
  }
  out[(uint64_t)j * kMom9Out + k] = (i64)v;
}

// Threads per block of the final pass: 1024 when runs have many records
// (about 512 segments for one lattice), else 256.
uint32_t final_threads(const MomArgs &a) {
  return a.n_segs >= 64u * a.n_runs ? 1024u : 256u;
}

template <int NM>
hipError_t launch3(hipStream_t s, const MomArgs &a) {
  if (a.digest)
    k_mom3<NM, true><<<a.n_segs, 256, 0, s>>>(a.state, a.slots, a.tslot, a.segs, a.no_stream,
                                              a.twiddle, a.partial);
  else
    k_mom3<NM, false><<<a.n_segs, 256, 0, s>>>(a.state, a.slots, a.tslot, a.segs, a.no_stream,
                                               a.twiddle, a.partial);
  return hipGetLastError();
}

}  // namespace

// Partial records of mclg_moments_noalloc: a fixed array in device memory
// (one per GPU, alive until the process ends), so that the call needs no
// workspace.  Host code must not pass this name to a kernel -- on the host it
// is only a stand-in for the symbol; moments_scratch() returns the device
// address.
static __device__ __align__(256) unsigned long long scratch[kMomScratchBytes / 8];

hipError_t moments_scratch(unsigned long long **ptr) {
  // device addresses of `scratch`, looked up once per device
  static std::mutex mu;
  static unsigned long long *addr[kMomScratchDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e) return e;
  if (dev < 0 || dev >= (int)kMomScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e) return e;
    addr[dev] = static_cast<unsigned long long *>(p);
  }
  *ptr = addr[dev];
  return hipSuccess;
}

MomPlan plan_moments(const uint32_t *slots, const uint64_t *sites, uint32_t n) {
  MomPlan p;
  uint64_t total = 0;
  for (uint32_t j = 0; j < n; ++j) total += sites[j];
  uint64_t seg = (total + kMomMaxSegsBase - 1) / kMomMaxSegsBase;
  seg = std::min<uint64_t>(kMomMaxSegSites, std::max<uint64_t>(16384, (seg + 16383) / 16384 * 16384));
  p.run_seg.push_back(0);
  for (uint32_t j = 0; j < n; ++j) {
    for (uint64_t x0 = 0; x0 < sites[j]; x0 += seg) {
      MomSeg m;
      m.slot = slots[j];
      m.run = j;
      m.x0 = (uint32_t)x0;
      m.x1 = (uint32_t)std::min<uint64_t>(sites[j], x0 + seg);
      p.segs.push_back(m);
    }
    if (sites[j] == 0) {  // an empty run still gets its (zero) record
      MomSeg m;
      m.slot = slots[j];
      m.run = j;
      p.segs.push_back(m);
    }
    p.run_seg.push_back((uint32_t)p.segs.size());
    p.run_slot.push_back(slots[j]);
  }
  return p;
}

hipError_t launch_moments3(hipStream_t s, const MomArgs &a) {
  if (a.n_runs == 0) return hipSuccess;
  if (a.n_modes > 8 || (a.n_modes && !a.twiddle)) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  switch (a.n_modes) {
    case 0: e = launch3<0>(s, a); break;
    case 1: e = launch3<1>(s, a); break;
    case 2: e = launch3<2>(s, a); break;
    case 3: e = launch3<3>(s, a); break;
    case 4: e = launch3<4>(s, a); break;
    case 5: e = launch3<5>(s, a); break;
    case 6: e = launch3<6>(s, a); break;
    case 7: e = launch3<7>(s, a); break;
    default: e = launch3<8>(s, a); break;
  }
  if (e) return e;
  k_mom3_final<<<a.n_runs, final_threads(a), 0, s>>>(a.partial, a.run_seg, a.run_slot, a.slots,
                                                     a.tslot, a.n_modes, a.out);
  return hipGetLastError();
}

hipError_t launch_moments9(hipStream_t s, const MomArgs &a) {
  if (a.n_runs == 0) return hipSuccess;
  k_mom9<<<a.n_segs, 256, 0, s>>>(a.state, a.reps, a.t9, a.no_stream, a.segs, a.partial);
  hipError_t e = hipGetLastError();
  if (e) return e;
  k_mom9_final<<<a.n_runs, final_threads(a), 0, s>>>(a.partial, a.run_seg, a.run_slot, a.reps,
                                                     a.t9, a.out);
  return hipGetLastError();
}

}  // namespace mclg
