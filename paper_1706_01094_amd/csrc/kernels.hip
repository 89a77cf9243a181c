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
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
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
__device__ __noinline__ uint32_t collide_direct(uint32_t a, uint32_t b, uint32_t c,
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

// One site: returns the post-collision (a, b, c) in place.
__device__ __forceinline__ void collide(uint32_t &a, uint32_t &b, uint32_t &c, uint32_t r,
                                        const StepParams &p, const TableDev &tab, uint32_t x,
                                        uint32_t t, uint32_t rid, uint32_t *err) {
  const uint32_t N = a + b + c;
  if (N > 65535u) { atomicOr(err, kErrOverflow); return; }
  if (N < 2u || p.C == 0) return;
  const int32_t J = (int32_t)c - (int32_t)a;
  const uint32_t absJ = (uint32_t)(J < 0 ? -J : J);
  uint32_t bn;
  if (N <= p.n_max) {
    // fiber states ascend in n0 = par + 2k
    const uint32_t par = (N - absJ) & 1u;
    const uint32_t base = tab.rowbase[(N * (N + 1u) >> 1) + absJ];
    const uint2 d = tab.rowdesc[base + ((b - par) >> 1)];
    const uint32_t idx = count_le(tab.thr + d.x, (d.y >> 16) - 1u, r);
    bn = par + 2u * ((d.y & 0xffffu) + idx);
  } else if (p.C < 0) {
    atomicOr(err, kErrEqRange);
    return;
  } else {
    bn = collide_direct(a, b, c, p, x, t, rid);
  }
  a = (uint32_t)(((int32_t)N - (int32_t)bn - J) >> 1);
  c = (uint32_t)(((int32_t)N - (int32_t)bn + J) >> 1);
  b = bn;
}

// Fused stream + collide over one tile of tile_sites sites per block.
// G groups of four consecutive sites per thread; one Philox call per group.
template <int G>
__global__ void __launch_bounds__(1024) k_step(
    uint16_t *__restrict__ state, const SlotDev *__restrict__ slots, uint32_t *tslot,
    const TileDev *__restrict__ tiles, const uint32_t *__restrict__ slot_list,
    uint32_t slot_first, uint32_t n_slots, uint32_t *ticket, uint32_t *err, TableDev tab,
    StepParams p) {
  const TileDev tile = tiles[blockIdx.x];
  const SlotDev sl = slots[tile.slot];
  const uint32_t t = tslot[tile.slot];
  const uint32_t L = sl.L;
  const uint32_t tm = p.no_stream ? 0u : t % L;
  uint16_t *const nm = state + sl.off;
  uint16_t *const n0 = nm + sl.stride;
  uint16_t *const np = n0 + sl.stride;
  const uint2 key = make_uint2((uint32_t)p.seed, (uint32_t)(p.seed >> 32));
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const uint32_t xg = tile.x0 + (g * blockDim.x + threadIdx.x) * 4u;
    if (xg >= L) continue;
    const uint4 w = philox10(make_uint4(xg >> 2, t, sl.rid, 0u), key);
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      const uint32_t x = xg + k;
      if (x >= L) break;
      uint32_t pm = x + tm;
      pm -= (pm >= L) ? L : 0u;
      const uint32_t pp = x >= tm ? x - tm : x + L - tm;
      uint32_t a = nm[pm], b = n0[x], c = np[pp];
      collide(a, b, c, word_of(w, k), p, tab, x, t, sl.rid, err);
      nm[pm] = (uint16_t)a;
      n0[x] = (uint16_t)b;
      np[pp] = (uint16_t)c;
    }
  }
  // The last block of the launch advances t of every slot in the launch.
  // Every block has read t before it takes its ticket, so nothing reads the
  // new value during this launch.
  __shared__ uint32_t last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(ticket, 1u) == gridDim.x - 1u;
  }
  __syncthreads();
  if (last) {
    __threadfence();
    for (uint32_t i = threadIdx.x; i < n_slots; i += blockDim.x) {
      const uint32_t s = slot_list ? slot_list[i] : slot_first + i;
      tslot[s] += 1u;
    }
    if (threadIdx.x == 0) atomicExch(ticket, 0u);
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

hipError_t launch_step(const Schedule &sch, hipStream_t s, uint16_t *state, const SlotDev *slots,
                       uint32_t *tslot, const TileDev *tiles, uint32_t n_tiles,
                       const uint32_t *slot_list, uint32_t slot_first, uint32_t n_slots,
                       uint32_t *ticket, uint32_t *err, TableDev tab, StepParams p) {
  if (n_tiles == 0) return hipSuccess;
  dim3 grid(n_tiles), block(sch.threads);
  switch (sch.groups) {
    case 1: k_step<1><<<grid, block, 0, s>>>(state, slots, tslot, tiles, slot_list, slot_first, n_slots, ticket, err, tab, p); break;
    case 2: k_step<2><<<grid, block, 0, s>>>(state, slots, tslot, tiles, slot_list, slot_first, n_slots, ticket, err, tab, p); break;
    case 4: k_step<4><<<grid, block, 0, s>>>(state, slots, tslot, tiles, slot_list, slot_first, n_slots, ticket, err, tab, p); break;
    case 8: k_step<8><<<grid, block, 0, s>>>(state, slots, tslot, tiles, slot_list, slot_first, n_slots, ticket, err, tab, p); break;
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
