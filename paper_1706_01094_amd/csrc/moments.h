// Exact moment sums of the MCLG state (D1Q3 and D2Q9): per-segment partial
// sums written by one kernel, combined per replica by a second one.  Every
// sum is an integer sum modulo 2^64, so the result does not depend on how
// the sites are split.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "device.h"

namespace mclg {

// Sites [x0, x1) of slot `slot` (D2Q9: sites s = y Lx + x of replica `slot`),
// part of run `run`.
struct MomSeg {
  uint32_t slot = 0, x0 = 0, x1 = 0, run = 0;
};

// The moment kernels' work for a list of slots: the segments of slot
// list[j] are segs[run_seg[j] .. run_seg[j + 1]).
struct MomPlan {
  std::vector<MomSeg> segs;
  std::vector<uint32_t> run_seg;   // runs + 1
  std::vector<uint32_t> run_slot;  // runs
};

// Segments of 16384 to 2^23 sites (a multiple of 16384: eight passes of a
// 256-thread block over eight sites per lane) and about 512 of them
// in all (two blocks per compute unit, one wave of blocks), so that at most
// 512 + n + total / 2^23 segments are made for n slots of `total` sites
// (2^23 bounds the 32-bit packed sums).
constexpr uint32_t kMomMaxSegsBase = 512;
constexpr uint64_t kMomMaxSegSites = 1ull << 23;
MomPlan plan_moments(const uint32_t *slots, const uint64_t *sites, uint32_t n);
inline uint64_t max_mom_segs(uint32_t n, uint64_t total_sites) {
  return kMomMaxSegsBase + n + total_sites / kMomMaxSegSites;
}

// Partial record of one D1Q3 segment: kMom3Rec uint64, of which the first
// 12 + 2 n_modes are written.  Slots 0-2 sum n_i, 3-5 sum n_i^2, 6-8 sum
// n_-1 n_0, n_0 n_+1, n_-1 n_+1, 9 sites with odd n_0, 10 the state digest,
// 11 max N, 12 + 2m and 13 + 2m the Fourier sums of mode m.
constexpr uint32_t kMom3Rec = 32;
// One replica's result in the field order of mclg_moments_t (33 int64).
constexpr uint32_t kMom3Out = 33;
// Partial record of one D2Q9 segment (kMom9Rec uint64, the first kMom9Used
// written): slots 0-8 sum n_i, 9-53 sum n_i n_j (i <= j, row-major), 54
// max N, 55 zero.
constexpr uint32_t kMom9Rec = 64;
constexpr uint32_t kMom9Used = 56;
constexpr uint32_t kMom9Max = 54;
// One replica's result in the field order of mclg_moments9_t (60 int64).
constexpr uint32_t kMom9Out = 60;

// Where the kernels of one moments call read and write.
struct MomArgs {
  const uint16_t *state = nullptr;
  const SlotDev *slots = nullptr;    // D1Q3
  const Rep9 *reps = nullptr;        // D2Q9
  const uint32_t *tslot = nullptr;   // D1Q3: per-slot step counters
  uint64_t t9 = 0;                   // D2Q9: steps taken
  uint32_t no_stream = 0;
  const MomSeg *segs = nullptr;
  uint32_t n_segs = 0;
  const uint32_t *run_seg = nullptr, *run_slot = nullptr;
  uint32_t n_runs = 0;
  const int32_t *twiddle = nullptr;  // D1Q3: [2 n_modes][L] per slot from its dense offset
  uint32_t n_modes = 0;
  uint32_t digest = 0;               // D1Q3: also sum the state digest
  unsigned long long *partial = nullptr;  // n_segs records
  long long *out = nullptr;                // run j's result at out[j * kMom*Out]
};

// Static partial-record area of the allocation-free moments call: 8 MiB per
// GPU (32768 D1Q3 records), for devices 0 .. kMomScratchDevices - 1.
constexpr uint64_t kMomScratchBytes = 8ull << 20;
constexpr uint32_t kMomScratchDevices = 64;
// Device address of the current device's area (looked up once per device;
// call it with the device current).
hipError_t moments_scratch(unsigned long long **ptr);

hipError_t launch_moments3(hipStream_t s, const MomArgs &a);
hipError_t launch_moments9(hipStream_t s, const MomArgs &a);

}  // namespace mclg
