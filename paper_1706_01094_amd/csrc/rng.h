// Device helpers shared by the HIP kernels of the MCLG library: error flags,
// Philox4x32-10 (Salmon et al., SC'11), random-word streams with Lemire's
// exact bounded integers, small search and shuffle helpers.
#pragma once
#include "device.h"

namespace mclg {
namespace {

constexpr uint32_t kErrOverflow = 1u;   // a site with N > 65535
constexpr uint32_t kErrEqRange = 2u;    // C = infinity and N > n_max
constexpr uint32_t kErrInternal = 4u;   // a blocked launch's grid barrier timed out

// a ^ b ^ k in one instruction (v_bitop3_b32 with the XOR3 truth table)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
  return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds, multipliers 0xD2511F53,
// 0xCD9E8D57, Weyl increments 0x9E3779B9, 0xBB67AE85.
__device__ __forceinline__ uint4 philox10(uint4 c, uint2 k) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    if (i) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
      // recomputed at every use (scalar adds) rather than held in registers
      asm volatile("" : "+s"(k.x), "+s"(k.y));
    }
    // one 32x32 -> 64-bit multiply per product (v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k.x), (uint32_t)p1,
                   xor3((uint32_t)(p0 >> 32), c.w, k.y), (uint32_t)p0);
  }
  return c;
}
// Two Philox4x32-10 calls with the same key, interleaved round by round
// (one key schedule, two independent multiply chains).
__device__ __forceinline__ void philox10_x2(uint4 &c0, uint4 &c1, uint2 k) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    if (i) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
      asm volatile("" : "+s"(k.x), "+s"(k.y));
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0.x, q0 = (uint64_t)0xD2511F53u * c1.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c0.z, q1 = (uint64_t)0xCD9E8D57u * c1.z;
    c0 = make_uint4(xor3((uint32_t)(p1 >> 32), c0.y, k.x), (uint32_t)p1,
                    xor3((uint32_t)(p0 >> 32), c0.w, k.y), (uint32_t)p0);
    c1 = make_uint4(xor3((uint32_t)(q1 >> 32), c1.y, k.x), (uint32_t)q1,
                    xor3((uint32_t)(q0 >> 32), c1.w, k.y), (uint32_t)q0);
  }
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
  // the same with its first word given; rejections continue on this stream
  __device__ uint32_t uniform_from(uint32_t first, uint32_t s) {
    uint64_t m = (uint64_t)first * s;
    if ((uint32_t)m < s) {
      const uint32_t floor_ = (0u - s) % s;
      while ((uint32_t)m < floor_) m = (uint64_t)next() * s;
    }
    return (uint32_t)(m >> 32);
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

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)v, m);
  const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m);
  return ((unsigned long long)hi << 32) | lo;
}

}  // namespace
}  // namespace mclg
