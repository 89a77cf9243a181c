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
  uint64_t off = 0;      // element offset of the n_-1 array in the state buffer
  uint64_t dense = 0;    // packed site offset (init counts, twiddles)
  uint32_t L = 0;        // sites
  uint32_t stride = 0;   // elements per array (L rounded up to 128)
  uint32_t rid = 0;      // RNG replica identity
  uint32_t pad = 0;
};

// A chunk of 512 sites of one slot (the last chunk of a slot may be short).
struct TileDev {
  uint32_t slot = 0;     // slot index
  uint32_t x0 = 0;       // first site (multiple of 512)
  uint32_t next = 0;     // index of the first chunk after this slot's run of chunks
  uint32_t pad = 0;
};

// Queued draws a wave may keep between chunks (the LDS queue and 32 more).
constexpr uint32_t kDrainAt = 64 + 32;

// When the draws the LDS image cannot decide are resolved (from the exact
// global rows), per wave:
//   kDrainDeferred: queued until more than kDrainAt wait, then resolved after
//     the chunk's store and written with 2-byte stores into the lines the
//     chunks stored before;
//   kDrainChunk: the same after every chunk's store;
//   kDrainPatch: before the chunk's store -- the exact outcomes go into the
//     chunk's registers, so the chunk's 16-byte stores write final values and
//     nothing is written twice.
enum : uint32_t { kDrainDeferred = 0, kDrainChunk = 1, kDrainPatch = 2 };

struct StepParams {
  uint64_t seed = 0;
  int32_t C = 0;
  uint32_t lam_p = 1, lam_q = 1;
  uint32_t n_max = 0;
  uint32_t no_stream = 0;
  uint32_t tile_sites = 512;
  uint32_t galilean = 0;  // per-site lambda (see collide_direct)
  uint32_t drain = kDrainDeferred;
};

// Deferred 2-byte writes land in lines the chunks stored long before.  While
// a launch's state fits the 256 MB Infinity Cache those lines are still
// cached and the writes are cheap; a larger state has left the caches by
// then, and partial-line writes into it are slow, so each chunk's draws are
// resolved before its store.
constexpr uint64_t kCachedStateBytes = 256ull << 20;
inline uint32_t auto_drain(uint64_t launch_state_bytes) {
  return launch_state_bytes > kCachedStateBytes ? kDrainPatch : kDrainDeferred;
}

// Stride (uint32) of the fixed-stride copy of the collision rows: a header
// k_first | q << 16 and up to 19 thresholds.
constexpr uint32_t kFixedStride = 20;

// uint16 values per row of the 64-byte copy of the collision rows: k_first,
// q and the top 16 bits of up to 30 thresholds (0xFFFF beyond q - 1).
constexpr uint32_t kRow16 = 32;

struct TableDev {
  const uint32_t *rowbase = nullptr;
  const uint2 *rowdesc = nullptr;
  const uint32_t *thr = nullptr;
  const uint4 *fixed = nullptr;  // rows at a fixed stride of kFixedStride uint32, or null
  const uint4 *row16 = nullptr;  // rows of kRow16 uint16 (64 bytes), or null
};

// The 64-byte rows cost a missed draw fewer memory bytes than the 80-byte
// ones but about 60 more VALU instructions.  They pay when the missed rows
// come from memory rather than the L2: when the draws of many densities miss
// (a batch of replicas with their own images), or when one density misses
// very often.  Measured on MI355X at L = 2^27 (us per step, 80-byte / 64-byte
// rows): rho = 50, 0.5 % misses 346 / 356; rho = 80, 1.6 % misses 364 / 379;
// rho = 100, u = 0.2, 10 % misses 447 / 420; the 1024-replica batch (2 %
// misses over 1024 images) 495 / 465.
inline bool use_compact_rows(double miss_fraction, uint32_t n_images) {
  return miss_fraction > 0.06 || (n_images >= 16 && miss_fraction > 0.01);
}

// Where a slot's LDS image lives in the image pool (see LdsImage).
struct ImageDesc {
  uint64_t off = 0;        // byte offset in the image pool (16-byte aligned)
  uint32_t bytes = 0;      // every slot has one (at least the two special slots)
  uint32_t dir_bytes = 0;
  uint32_t dim_a = 0, dim_c = 0, b_lo = 0, nb = 0;
};

struct PoisDesc {
  uint32_t off = 0;      // offset in the threshold pool
  uint32_t k_first = 0;
  uint32_t nthr = 0;     // q - 1
  uint32_t pad = 0;
};

// Launch configuration of the fused stream+collide kernel.
struct Schedule {
  uint32_t groups = 1;       // chunks of 8 sites per lane (must be 1)
  uint32_t threads = 1024;   // threads per block
  uint32_t lds_budget = 160 * 1024;  // bytes of collision image per block (at most)
  uint32_t tile_sites() const { return 512; }  // one chunk: 64 lanes x 8 sites
};

// Every field has an initialiser, so that a launch record built field by
// field never carries an indeterminate value.
struct StepLaunch {
  uint16_t *state = nullptr;
  const SlotDev *slots = nullptr;
  uint32_t *tslot = nullptr;
  const TileDev *tiles = nullptr;
  uint32_t n_tiles = 0;
  const uint32_t *slot_list = nullptr;  // slots advanced by this launch, or null for a range
  uint32_t slot_first = 0, n_slots = 0;
  // With `ticket` set, the launch's last block advances tslot of the launch's
  // slots by one; without it the slots' step is tslot + t_off and tslot is
  // advanced later (launch_add_t), which saves the end-of-launch ticket.
  uint32_t *ticket = nullptr, *err = nullptr;
  uint32_t t_off = 0;
  // A launch over one slot's tiles (0 .. n_tiles - 1 from x = 0) carries the
  // slot's descriptors itself, so that its blocks start without dependent
  // loads: single = 1, slot slot_first, image im1, slot sl1.
  uint32_t single = 0;
  ImageDesc im1;
  SlotDev sl1;
  TableDev tab;
  StepParams p;
  const ImageDesc *images = nullptr;  // per slot
  const uint8_t *image_pool = nullptr;
  uint4 *overflow = nullptr;          // kOverflowPerWave entries per resident wave
  uint32_t lds_bytes = 0;             // LDS per block for the image (largest image, 16-byte
                                      // multiple); the per-wave miss queues follow it
  uint32_t max_blocks = 1;            // persistent grid size
};

hipError_t launch_step(const Schedule &sch, hipStream_t s, const StepLaunch &a);

// Several steps of one lattice per launch (temporal blocking).  Block b owns
// the sites [b R, b R + R) and keeps a copy of them and of kh more sites on
// each side (es = R + 2 kh sites) in its own part of `scratch`, a periodic
// lattice of es sites in the shifted layout.  It copies the region in at
// step t, and after a grid-wide barrier (every block has read the state)
// advances its copy `steps` steps (steps <= kh): the sites within j of the
// copy's ends are wrong after j steps, the owned sites stay exact, and the
// random numbers are keyed by each site's place in the lattice.  It then
// writes its owned sites back at step t + steps.  Block 0 advances the
// slot's step counter by `steps` once every block has read it.  The barrier
// counts arrivals in `bar` across launches (never reset): this launch's
// blocks have all arrived when it reaches bar_target.
constexpr uint32_t kTbMaxSteps = 256;
struct TbLaunch {
  uint16_t *scratch = nullptr;  // grid x bstride elements
  uint32_t stride = 0;          // elements per array of a block's copy (>= es)
  uint32_t R = 0;               // owned sites per block (a multiple of 8)
  uint32_t kh = 0;              // extra sites on each side (a multiple of 8)
  uint32_t es = 0;              // R + 2 kh
  uint32_t steps = 0;           // steps of the launch
  // Tiles (T > 0, for lattices whose blocks' copies would not stay in the
  // caches): block b goes through its region in tiles of T sites, each copied
  // with kh extra sites on each side (es = T + 2 kh) into the copy area,
  // advanced `steps` steps and written back before the next; see k_step_tt.
  uint32_t T = 0;
  uint64_t bstride = 0;         // elements of scratch per block
  // Replicas (reps != 0, a context of several lattices; see k_step_tr): block
  // b advances whole replicas, items[item_first[b] .. item_first[b + 1]),
  // each copied whole (stride >= the largest L), with no grid barrier.
  uint32_t reps = 0;
  const uint32_t *items = nullptr, *item_first = nullptr;
  uint32_t *bar = nullptr;      // arrivals of every blocked launch of the context
  uint32_t bar_target = 0;      // arrivals before this launch + its grid
  // Logs (n_logs > 0): the moments (mclg_moments_t) of the state after steps
  // log_first, log_first + log_every, ... (the last at most `steps`) of the
  // launch; log = 1 + 2 n_modes + digest, at most 5 (two modes without the
  // digest).  Logs before the last step: only without the digest and the
  // Galilean acceptance.  Block b writes its partial record of log j (kMom3Rec values) at
  // records + (j grid + b) kMom3Rec with device-coherent stores; after a
  // second barrier (bar_target + grid) block b adds the records of logs b,
  // b + grid, ... into out + j kMom3Out.  tw: the lattice's [2 n_modes][L]
  // twiddles.
  uint32_t log = 0, n_logs = 0, log_first = 0, log_every = 0;
  const int32_t *tw = nullptr;
  unsigned long long *records = nullptr;
  long long *out = nullptr;
};
hipError_t launch_step_blocked(const Schedule &sch, hipStream_t s, const StepLaunch &a,
                               const TbLaunch &tb, uint32_t grid);
// Blocks of the blocked kernel that fit the device at once (the grid it
// needs: every block must be resident for the barrier).
hipError_t step_blocked_occupancy(const Schedule &sch, uint32_t lds_bytes, uint32_t n_cu,
                                  uint32_t &max_blocks);

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
}  // namespace mclg
