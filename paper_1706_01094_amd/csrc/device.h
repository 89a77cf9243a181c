// Device-side data structures and launchers of the MCLG library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mclg {

// One simulated lattice ("slot").  Its state is three uint16 arrays of
// `stride` elements starting at element `off` of the state buffer:
// n_-1, n_0, n_+1.  In-place shifted layout: logical n_+1(x, t) is stored at
// physical (x - t) mod L, n_-1(x, t) at (x + t) mod L, n_0(x) at x, so that
// streaming costs nothing and every element is read and written by exactly
// one site per step.  With MCLG_FLAG_NO_STREAM the layout is unshifted.
struct SlotDev {
  uint64_t off;      // element offset of the n_-1 array in the state buffer
  uint64_t dense;    // packed site offset (init counts, twiddles)
  uint32_t L;        // sites
  uint32_t stride;   // elements per array (L rounded up to 128)
  uint32_t rid;      // RNG replica identity
  uint32_t pad;
};

// A chunk of 512 sites of one slot (the last chunk of a slot may be short).
struct TileDev {
  uint32_t slot;     // slot index
  uint32_t x0;       // first site (multiple of 512)
  uint32_t next;     // index of the first chunk after this slot's run of chunks
  uint32_t pad;
};

// Queued draws a wave may keep between chunks (the LDS queue and 32 more).
constexpr uint32_t kDrainAt = 64 + 32;

struct StepParams {
  uint64_t seed;
  int32_t C;
  uint32_t lam_p, lam_q;
  uint32_t n_max;
  uint32_t no_stream;
  uint32_t tile_sites;
  uint32_t galilean;  // per-site lambda (see collide_direct)
  // kDrainAt: a wave keeps up to kDrainAt queued draws between chunks; 0:
  // it resolves them after every chunk (set by drain_threshold)
  uint32_t drain_at = kDrainAt;
};

// Queued draws are resolved later with 2-byte writes into the lines the
// chunk stored.  While a launch's state fits the 256 MB Infinity Cache those
// lines are still cached and the writes are cheap, so draws are kept until
// more than kDrainAt are queued.  A larger state has left the caches by then,
// and partial-line writes into it are slow, so every chunk's draws are
// resolved right after its store.
constexpr uint64_t kCachedStateBytes = 256ull << 20;
inline uint32_t drain_threshold(uint64_t launch_state_bytes) {
  return launch_state_bytes > kCachedStateBytes ? 0u : kDrainAt;
}

// Stride (uint32) of the fixed-stride copy of the collision rows: a header
// k_first | q << 16 and up to 19 thresholds.
constexpr uint32_t kFixedStride = 20;

struct TableDev {
  const uint32_t *rowbase;
  const uint2 *rowdesc;
  const uint32_t *thr;
  const uint4 *fixed;  // rows at a fixed stride of kFixedStride uint32, or null
};

// Exact per-slot sums, all modulo 2^64.
struct MomDev {
  unsigned long long v[32];
  // 0..2 sum n, 3..5 sum n^2, 6..8 sum nn, 9 sum N, 10 sum J, 11 sum N^2,
  // 12 n0 odd, 13 max N, 14..29 fourier (m, cos/sin)
};

// Where a slot's LDS image lives in the image pool (see LdsImage).
struct ImageDesc {
  uint64_t off;        // byte offset in the image pool (16-byte aligned)
  uint32_t bytes;      // every slot has one (at least the two special slots)
  uint32_t dir_bytes;
  uint32_t dim_a, dim_c, b_lo, nb;
};

struct PoisDesc {
  uint32_t off;      // offset in the threshold pool
  uint32_t k_first;
  uint32_t nthr;     // q - 1
  uint32_t pad;
};

// Launch configuration of the fused stream+collide kernel.
struct Schedule {
  uint32_t groups = 1;       // chunks of 8 sites per lane (must be 1)
  uint32_t threads = 1024;   // threads per block
  uint32_t lds_budget = 160 * 1024;  // bytes of collision image per block (at most)
  uint32_t tile_sites() const { return 512; }  // one chunk: 64 lanes x 8 sites
};

struct StepLaunch {
  uint16_t *state;
  const SlotDev *slots;
  uint32_t *tslot;
  const TileDev *tiles;
  uint32_t n_tiles;
  const uint32_t *slot_list;  // slots advanced by this launch, or null for a range
  uint32_t slot_first, n_slots;
  // With `ticket` set, the launch's last block advances tslot of the launch's
  // slots by one; without it the slots' step is tslot + t_off and tslot is
  // advanced later (launch_add_t), which saves the end-of-launch ticket.
  uint32_t *ticket, *err;
  uint32_t t_off;
  // A launch over one slot's tiles (0 .. n_tiles - 1 from x = 0) carries the
  // slot's descriptors itself, so that its blocks start without dependent
  // loads: single = 1, slot slot_first, image im1, slot sl1.
  uint32_t single;
  ImageDesc im1;
  SlotDev sl1;
  TableDev tab;
  StepParams p;
  const ImageDesc *images;    // per slot
  const uint8_t *image_pool;
  uint4 *overflow;            // kOverflowPerWave entries per resident wave
  uint32_t lds_bytes;         // LDS per block for the image (largest image, 16-byte multiple);
                              // the per-wave miss queues follow it
  uint32_t max_blocks;        // persistent grid size
};

hipError_t launch_step(const Schedule &sch, hipStream_t s, const StepLaunch &a);

// Largest lattice (sites per replica or job): the step kernel addresses a
// slot's three arrays (6 bytes per site, 256-byte padded) with 32-bit byte
// offsets.
constexpr uint64_t kMaxSites = 1ull << 29;
constexpr uint32_t kQueue = 64;  // LDS queue entries (16 bytes) per wave
static_assert(kDrainAt == kQueue + 32, "drain threshold follows the LDS queue");
// per-wave LDS after the image: the queue of undecided draws
constexpr uint32_t kWaveLdsBytes = kQueue * 16;
// Entries of the global overflow area per wave (the queue continues there
// when its LDS part is full: up to 32 entries beyond it plus one chunk's
// 512 sites), and the number of waves the overflow region is sized for (all
// waves that can be resident on a 256-CU device).
constexpr uint32_t kOverflowPerWave = 576;
constexpr uint32_t kOverflowWaves = 256 * 32;
constexpr uint64_t kOverflowBytes = (uint64_t)kOverflowPerWave * kOverflowWaves * 16;

// Persistent grid size: resident blocks per CU for this LDS footprint x CUs.
hipError_t step_occupancy(const Schedule &sch, uint32_t lds_bytes, uint32_t n_cu,
                          uint32_t &max_blocks);
// Dynamic LDS of one block: image (rounded to 16 bytes) + miss queues.
uint32_t step_lds_bytes(const Schedule &sch, uint32_t image_bytes);

hipError_t launch_init_poisson(hipStream_t s, uint16_t *state, const SlotDev *slots,
                               const uint32_t *tslot, const TileDev *tiles, uint32_t n_tiles,
                               uint32_t tile_sites, const PoisDesc *desc, const uint32_t *pool,
                               uint64_t seed, uint32_t *err);

hipError_t launch_init_counts(hipStream_t s, uint16_t *state, const SlotDev *slots,
                              const TileDev *tiles, uint32_t n_tiles, uint32_t tile_sites,
                              const uint16_t *counts);

hipError_t launch_zero(hipStream_t s, unsigned long long *p, uint64_t n);

hipError_t launch_moments(hipStream_t s, const uint16_t *state, const SlotDev *slots,
                          const uint32_t *tslot, const TileDev *tiles, uint32_t n_tiles,
                          uint32_t tile_sites, uint32_t no_stream, const int32_t *twiddle,
                          uint32_t n_modes, MomDev *out);

// hist[(slot * 3 + i) * n_bins + min(n_i, n_bins - 1)] += 1 over every site
hipError_t launch_histogram(hipStream_t s, const uint16_t *state, const SlotDev *slots,
                            const TileDev *tiles, uint32_t n_tiles, uint32_t tile_sites,
                            uint32_t n_bins, unsigned long long *hist);

// tslot[slot_first + i] += add for i < n
hipError_t launch_add_t(hipStream_t s, uint32_t *tslot, uint32_t slot_first, uint32_t n,
                        uint32_t add);
hipError_t launch_set_t(hipStream_t s, uint32_t *tslot, const uint32_t *slot_list, uint32_t n,
                        uint32_t value);

// ---- D2Q9 --------------------------------------------------------------
// One replica: nine uint16 arrays of `stride` elements from `off`; logical
// n_i(x, y, t) lives at physical ((x - vx t) mod Lx, (y - vy t) mod Ly),
// element y Lx + x, so streaming is free as for D1Q3.
struct Rep9 {
  uint64_t off;
  uint32_t Lx, Ly, S, stride;
  uint32_t rid, pad;
};
struct Tile9 {
  uint32_t rep, s0;  // replica, first site (multiple of 256)
};
// Collision rules, per ordered source pair (v1, v2), kRule9Words uint32:
// words 0-3 the cumulative integer weights of the (up to four) targets, D
// where there is none; words 4-8 the change of the nine counts for target
// q = #{cumulative weights <= u} (word 4 + q; q = number of targets means no
// change), 3 bits per velocity i at bit 3i holding 2 + the change; 9-11 pad.
constexpr uint32_t kRule9Words = 12;
constexpr uint32_t kMom9Vals = 9 + 45 + 4;  // sum n_i, sum n_i n_j (i <= j), N, Jx, Jy, max N
struct Step9 {
  uint16_t *state;
  const Rep9 *reps;
  const Tile9 *tiles;
  const uint32_t *rules;
  uint32_t *err;
  uint64_t seed;
  uint64_t t;          // steps taken (the RNG counter uses its low 32 bits)
  uint32_t D, no_stream;
  int32_t C;
};
hipError_t launch_step9(hipStream_t s, const Step9 &a, uint32_t n_tiles);
hipError_t launch_init9_poisson(hipStream_t s, uint16_t *state, const Rep9 *reps,
                                const Tile9 *tiles, uint32_t n_tiles, const PoisDesc *desc,
                                const uint32_t *pool, uint64_t seed, uint32_t *err);
hipError_t launch_init9_counts(hipStream_t s, uint16_t *state, const Rep9 *reps,
                               const Tile9 *tiles, uint32_t n_tiles, const uint64_t *dense,
                               const uint16_t *counts);
hipError_t launch_histogram9(hipStream_t s, const uint16_t *state, const Rep9 *reps,
                             const Tile9 *tiles, uint32_t n_tiles, uint32_t n_bins,
                             unsigned long long *hist);
hipError_t launch_moments9(hipStream_t s, const uint16_t *state, const Rep9 *reps,
                           const Tile9 *tiles, uint32_t n_tiles, uint64_t t, uint32_t no_stream,
                           unsigned long long *out);

}  // namespace mclg
