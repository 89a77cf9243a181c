// Sums of the D1Q3 moments (mclg_moments_t) over a lane's sites and a
// block's lanes: the exact integer sums behind the paper's statistics (means
// and variances of n_i for Eq. (poisson), the correlator of Eq. (corr), N and
// J, Fourier projections of the density for Eq. (A) and S(k)) and the state
// digest.  Shared by the moment kernels and by the blocked step kernel, which
// sums the sites it writes back on a logging launch.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "moments.h"
#include "rng.h"

namespace mclg {
namespace mom3 {

typedef unsigned long long u64;
typedef long long i64;
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// MurmurHash3's 32-bit finaliser (Appleby): a bijective mix of 32 bits.
__device__ __forceinline__ uint32_t fmix32(uint32_t k) {
  k ^= k >> 16;
  k *= 0x85ebca6bu;
  k ^= k >> 13;
  k *= 0xc2b2ae35u;
  k ^= k >> 16;
  return k;
}

// Reduce-scatter of V (a power of two up to 64) 64-bit sums over the 64
// lanes of a wave: each level exchanges half of the values with the lane
// whose id differs in one bit and adds, so V - 1 exchanges move what V x 6
// would in a plain butterfly.  Afterwards lane l holds the wave's total of
// value l >> (6 - log2 V).
template <int V>
__device__ __forceinline__ u64 wave_sum_scatter(u64 (&v)[V], uint32_t lane) {
  int w = V, m = 32;
#pragma unroll
  for (int lvl = 0; (1 << lvl) < V; ++lvl) {
    const bool up = (lane & (uint32_t)m) != 0;
    const int h = w >> 1;
#pragma unroll
    for (int j = 0; j < V / 2; ++j) {
      if (j < h) {
        const u64 send = up ? v[j] : v[j + h];
        const u64 keep = up ? v[j + h] : v[j];
        v[j] = keep + shfl_xor_u64(send, m);
      }
    }
    w = h;
    m >>= 1;
  }
  u64 s = v[0];
#pragma unroll
  for (; m >= 1; m >>= 1) s += shfl_xor_u64(s, m);
  return s;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, (uint32_t)__shfl_xor(v, m));
  return v;
}

// Block-wide combination of the lanes' sums and maxima into one partial
// record: sums of values 0 .. V-1 in record slots 0 .. W-1 except MS, the
// maximum in slot MS (value MS is zero).  red and redmx: LDS of 16 x V and 16
// values (one row per wave, at most 16 waves).  COHERENT: the record is
// written with device-coherent stores (past the L2 of the block's XCD), for
// a reader in the same launch.
template <int V, int W, int MS, bool COHERENT = false>
__device__ __forceinline__ void block_record(u64 (&v)[V], uint32_t mx, u64 *rec, u64 *red,
                                             uint32_t *redmx) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  constexpr int sh = V >= 64 ? 0 : V >= 32 ? 1 : V >= 16 ? 2 : V >= 8 ? 3 : V >= 4 ? 4 : 5;
  const u64 s = wave_sum_scatter<V>(v, lane);
  mx = wave_max(mx);
  if ((lane & ((1u << sh) - 1u)) == 0u) red[wave * V + (lane >> sh)] = s;
  if (lane == 0) redmx[wave] = mx;
  __syncthreads();
  const uint32_t nw = blockDim.x >> 6;
  for (uint32_t k = threadIdx.x; k < (uint32_t)W; k += blockDim.x) {
    u64 out = 0;
    if (k == (uint32_t)MS) {
      uint32_t m = 0;
      for (uint32_t w = 0; w < nw; ++w) m = max(m, redmx[w]);
      out = m;
    } else {
      for (uint32_t w = 0; w < nw; ++w) out += red[w * V + k];
    }
    if constexpr (COHERENT)
      __hip_atomic_store(rec + k, out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      rec[k] = out;
  }
}

// Accumulators of one lane (record slots 0 .. 10 + 2 NM, max N apart).
// Windows whose counts are all below 256 add their sums and products with
// packed dot products into 32-bit sums (f, in the order of record slots
// 0..8): each adds at most 8 x 255^2 per window, so f stays below 2^32 as
// long as a lane adds at most 4096 windows before fold() (the moment kernels:
// segments of at most 2^23 sites, 2048 per pass of 256 lanes; the blocked
// step kernel: at most 2^21 sites per block, 8192 per pass of 1024 lanes).
// Other windows add exact 64-bit sums.
template <int NM>
struct Acc3 {
  u64 s[11 + 2 * NM];
  uint32_t f[9];
  uint32_t mx;
  uint32_t mxp;  // packed 16-bit maxima of N of the packed windows
};

__device__ __forceinline__ uint32_t dot2(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b), c,
                                false);
}

// Eight sites of a lane as loaded: counts two to a word, and for up to two
// modes the twiddle values of the eight sites (more modes load theirs when
// they are summed, so that few registers are live).
template <int NM>
struct Eight {
  static constexpr int PR = NM <= 2 ? 2 * NM : 0;
  uint32_t a[4], b[4], c[4];
  int32_t w[PR > 0 ? PR : 1][8];
  uint32_t x, n;
};

// The eight twiddle values of row `row` at sites x .. x + n - 1 (zero past).
__device__ __forceinline__ void load_tw8(const int32_t *row, uint32_t n, int32_t (&w)[8]) {
  if (n == 8u) {
    __builtin_memcpy(&w[0], row, 16);
    __builtin_memcpy(&w[4], row + 4, 16);
  } else {
#pragma unroll
    for (uint32_t e = 0; e < 8u; ++e) w[e] = e < n ? row[e] : 0;
  }
}

template <int NM>
__device__ __forceinline__ void acc_clear(Acc3<NM> &A) {
#pragma unroll
  for (int k = 0; k < 11 + 2 * NM; ++k) A.s[k] = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) A.f[k] = 0;
  A.mx = 0;
  A.mxp = 0;
}

template <int NM, bool DIG>
__device__ __forceinline__ void add_eight(Acc3<NM> &A, const Eight<NM> &E, const int32_t *tw,
                                          uint32_t L) {
  const uint32_t(&va)[4] = E.a;
  const uint32_t(&vb)[4] = E.b;
  const uint32_t(&vc)[4] = E.c;
  const uint32_t x = E.x, nvalid = E.n;
  uint32_t Ns[8];
  uint32_t any = 0, odd = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) any |= va[j] | vb[j] | vc[j];
  if ((any & 0xff00ff00u) == 0u) {
    // every count below 256: packed products, packed N (below 768)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      A.f[0] = dot2(va[j], 0x00010001u, A.f[0]);
      A.f[1] = dot2(vb[j], 0x00010001u, A.f[1]);
      A.f[2] = dot2(vc[j], 0x00010001u, A.f[2]);
      A.f[3] = dot2(va[j], va[j], A.f[3]);
      A.f[4] = dot2(vb[j], vb[j], A.f[4]);
      A.f[5] = dot2(vc[j], vc[j], A.f[5]);
      A.f[6] = dot2(va[j], vb[j], A.f[6]);
      A.f[7] = dot2(vb[j], vc[j], A.f[7]);
      A.f[8] = dot2(va[j], vc[j], A.f[8]);
      const u16x2 n2 = __builtin_bit_cast(u16x2, va[j]) + __builtin_bit_cast(u16x2, vb[j]) +
                       __builtin_bit_cast(u16x2, vc[j]);
      A.mxp = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, A.mxp), n2));
      const uint32_t nw = __builtin_bit_cast(uint32_t, n2);
      Ns[2 * j] = nw & 0xffffu;
      Ns[2 * j + 1] = nw >> 16;
      odd += __popc(vb[j] & 0x00010001u);
    }
  } else {
    uint32_t sa = 0, sb = 0, sc = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t a0 = va[j] & 0xffffu, a1 = va[j] >> 16;
      const uint32_t b0 = vb[j] & 0xffffu, b1 = vb[j] >> 16;
      const uint32_t c0 = vc[j] & 0xffffu, c1 = vc[j] >> 16;
      sa += a0 + a1;
      sb += b0 + b1;
      sc += c0 + c1;
      A.s[3] += (u64)a0 * a0 + (u64)a1 * a1;
      A.s[4] += (u64)b0 * b0 + (u64)b1 * b1;
      A.s[5] += (u64)c0 * c0 + (u64)c1 * c1;
      A.s[6] += (u64)a0 * b0 + (u64)a1 * b1;
      A.s[7] += (u64)b0 * c0 + (u64)b1 * c1;
      A.s[8] += (u64)a0 * c0 + (u64)a1 * c1;
      odd += __popc(vb[j] & 0x00010001u);
      Ns[2 * j] = a0 + b0 + c0;
      Ns[2 * j + 1] = a1 + b1 + c1;
      A.mx = max(A.mx, max(Ns[2 * j], Ns[2 * j + 1]));
    }
    A.s[0] += sa;
    A.s[1] += sb;
    A.s[2] += sc;
  }
  A.s[9] += odd;
  if constexpr (DIG) {
    // digest: sum over existing sites and velocities of
    // fmix32(fmix32(4 x + i + 1) ^ n_i(x)), i = 0, 1, 2 for v = -1, 0, +1
    u64 d = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t k0 = 4u * (x + 2u * j) + 1u, k1 = k0 + 4u;
      if (2u * j < nvalid)
        d += (u64)fmix32(fmix32(k0) ^ (va[j] & 0xffffu)) + fmix32(fmix32(k0 + 1u) ^ (vb[j] & 0xffffu)) +
             fmix32(fmix32(k0 + 2u) ^ (vc[j] & 0xffffu));
      if (2u * j + 1u < nvalid)
        d += (u64)fmix32(fmix32(k1) ^ (va[j] >> 16)) + fmix32(fmix32(k1 + 1u) ^ (vb[j] >> 16)) +
             fmix32(fmix32(k1 + 2u) ^ (vc[j] >> 16));
    }
    A.s[10] += d;
  }
  if constexpr (NM > 0) {
    // twiddle rows of the slot: row r at tw + r L (4-byte aligned); beyond
    // two modes, one mode (two rows) at a time, so that at most 16 of their
    // values are live
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      int32_t w[2][8];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if constexpr (Eight<NM>::PR > 0) {
#pragma unroll
          for (int e = 0; e < 8; ++e) w[h][e] = E.w[Eight<NM>::PR > 0 ? 2 * m + h : 0][e];
        } else {
          load_tw8(tw + (uint64_t)(2 * m + h) * L + x, nvalid, w[h]);
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        i64 f = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) f += (i64)(int32_t)Ns[e] * (i64)w[h][e];
        A.s[11 + 2 * m + h] += (u64)f;
      }
      if constexpr (Eight<NM>::PR == 0) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// The lane's sums in record order (the 11 sums, zero in the maximum's slot
// 11, then the Fourier sums) and its maximum N, with the packed sums folded in.
template <int NM, int V>
__device__ __forceinline__ uint32_t fold(Acc3<NM> &A, u64 (&v)[V]) {
  constexpr int W = 12 + 2 * NM;
  static_assert(W <= V, "record values");
#pragma unroll
  for (int k = 0; k < 9; ++k) A.s[k] += A.f[k];
#pragma unroll
  for (int k = 0; k < V; ++k)
    v[k] = k < 11 ? A.s[k < 11 ? k : 0] : (k >= 12 && k < W) ? A.s[(k >= 12 && k < W) ? k - 1 : 0] : 0ull;
  return max(A.mx, max(A.mxp & 0xffffu, A.mxp >> 16));
}

// Field k (< kMom3Out) of a replica's mclg_moments_t from the sums T of its
// records: t (the device step counter), sites, sum n_i, sum n_i^2, sum n_i
// n_j, sum N = the three sums, sum J = sum n_+1 - sum n_-1, sum N^2 = sum
// n_i^2 + 2 sum n_i n_j, sites with odd n_0, max N, the Fourier sums of the
// n_modes modes (zero beyond), the digest.
__device__ __forceinline__ u64 result_field(uint32_t k, const u64 *T, uint32_t t, uint32_t L,
                                            uint32_t n_modes) {
  if (k == 0u) return t;
  if (k == 1u) return L;
  if (k <= 10u) return T[k - 2u];
  if (k == 11u) return T[0] + T[1] + T[2];
  if (k == 12u) return T[2] - T[0];
  if (k == 13u) return T[3] + T[4] + T[5] + 2ull * (T[6] + T[7] + T[8]);
  if (k == 14u) return T[9];
  if (k == 15u) return T[11];
  if (k < 32u) return k - 16u < 2u * n_modes ? T[k - 4u] : 0ull;
  return T[10];
}

}  // namespace mom3
}  // namespace mclg
