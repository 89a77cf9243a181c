/*
 * mclg.h -- C ABI of the MI355X Monte Carlo Lattice Gas library (libmclg.so).
 *
 * The method is the integer lattice gas of Blommel & Wagner, "Integer Lattice
 * Gas with Monte Carlo collision operator recovers the entropic lattice
 * Boltzmann method with Poisson distributed fluctuations" (arXiv:1706.01094):
 * integer occupation numbers n_i(x,t) on a periodic D1Q3 lattice (velocities
 * -1, 0, +1, Eq. (D1Q3vel)) evolve by n_i(x+v_i, t+1) = n_i(x,t) + Xi_i
 * (Sec. "The Monte Carlo Lattice Gas algorithm"), where Xi is the result of C
 * random binary sub-collisions per site (Eq. (select), Eq. (omega)) with the
 * D1Q3 transition probabilities of Sec. "A D1Q3 implementation".  Mass N and
 * momentum J are conserved exactly at every site.
 *
 * Stated rules (the paper leaves them open; results are bit-exact functions
 * of them):
 *   - a sub-collision picks an ordered pair of distinct particles uniformly;
 *   - n(x,t) is the pre-collision state; one step collides every site, then
 *     streams; step t draws its random numbers with counter t;
 *   - the C sub-collisions of a site are sampled in one draw from their exact
 *     joint law (integer matrix power on the site's (N, |J|) fiber), quantised
 *     to uint32 thresholds floor(2^32 * cumulative probability); the outcome
 *     is the number of thresholds <= r for one Philox4x32-10 word r;
 *   - sites with N > n_max use the literal sub-collision loop instead;
 *   - Philox4x32-10 key = (seed low, seed high); counter =
 *     (site word, t, replica id, purpose | block << 2); collisions use word
 *     x & 3 of counter (x >> 2, t, replica, 0); Poisson initial counts use
 *     words 0, 1, 2 of counter (x, 0, replica, 1); the literal loop consumes
 *     blocks j = 0, 1, ... of counter (x, t, replica, 2 | j << 2) in order.
 *
 * Conventions for every entry point:
 *   - every call returns an int: MCLG_OK (0) or a negative MCLG_E_* code; no
 *     exception crosses the ABI;
 *   - device memory is owned by the caller (e.g. torch tensors) and must stay
 *     alive until mclg_destroy; the library never allocates device memory;
 *   - host arrays passed in are copied before the call returns;
 *   - device work is enqueued on the caller's stream in stream order; calls
 *     that return host data synchronise that stream;
 *   - a context is not thread-safe; distinct contexts are independent.
 */
#ifndef MCLG_H
#define MCLG_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCLG_ABI_VERSION 1u

enum {
  MCLG_OK = 0,
  MCLG_E_INVAL = -1,       /* bad argument, size, or buffer too small */
  MCLG_E_RANGE = -2,       /* a site exceeded N = 65535 (or n_max with C = inf) */
  MCLG_E_HIP = -3,         /* HIP runtime error; see mclg_last_hip_error */
  MCLG_E_NOMEM = -4,       /* host allocation failed */
  MCLG_E_UNSUPPORTED = -5, /* entry point not available for the context's lattice */
  MCLG_E_FULL = -6,        /* server: no slot or arena space for the job */
  MCLG_E_INTERNAL = -7,    /* a device-side consistency check failed (a library bug) */
  MCLG_E_TOO_LARGE = -8    /* more work than the static scratch area of
                              mclg_moments_noalloc holds */
};

enum { MCLG_D1Q3 = 1, MCLG_D2Q9 = 2 };
#define MCLG_C_EQUILIBRIUM (-1) /* C -> infinity: redraw from the fiber equilibrium */

enum {
  MCLG_FLAG_NO_STREAM = 1u, /* collisions only, no streaming (Fig. 5 variant, shear-wave init) */
  /* Galilean-invariant acceptance, the remedy the paper proposes after
   * Eq. (D1Q3relax) for the velocity dependence of the relaxation time:
   * lambda = lambda~ / sqrt(1 + 3 U^2), lambda~ = lambda_num / lambda_den,
   * with each site's own U = J / N.  The value is irrational, so every fiber
   * (N, |J|) uses it rounded down to 32 fractional bits, exactly:
   *   g = floor(2^32 N / sqrt(N^2 + 3 J^2)),  lambda = floor(g num / den) / 2^32
   * (mclg_galilean_lambda).  The tables are exact for that lambda; sites
   * above n_max draw their acceptances as 32-bit words compared with the
   * numerator: a {-1,+1} pair is accepted when w < p, a {0,0} pair (total
   * probability lambda / 8) when w1 * 8 + (w2 >> 29) < p. */
  MCLG_FLAG_GALILEAN = 2u
};

enum { MCLG_INIT_COUNTS = 1, MCLG_INIT_POISSON = 2 };

#define MCLG_MAX_MODES 8
#define MCLG_MAX_HIST_BINS 4096

typedef struct mclg_ctx mclg_ctx;

/* Simulation of n_replicas independent periodic lattices.  Replica r has
 * L[r] sites and RNG identity replica_id[r] (default r). */
typedef struct {
  uint32_t abi_version;        /* MCLG_ABI_VERSION */
  uint32_t lattice;            /* MCLG_D1Q3 or MCLG_D2Q9 */
  uint32_t n_replicas;         /* >= 1 */
  uint32_t flags;              /* MCLG_FLAG_* */
  const uint64_t *L;           /* host [n_replicas]; 1 <= L <= 2^29 */
  const uint64_t *replica_id;  /* host [n_replicas], each < 2^32, or NULL */
  uint64_t seed;               /* Philox key */
  int32_t C;                   /* sub-collisions per step, >= 0, or MCLG_C_EQUILIBRIUM */
  uint32_t lambda_num;         /* acceptance lambda = num / den in (0, 1] */
  uint32_t lambda_den;
  uint32_t n_max;              /* tables cover N <= n_max (<= 1023); default 255 */
  void *stream;                /* hipStream_t; NULL = null stream */
  void *state;                 /* device, caller-owned, >= state_bytes of mclg_sizes */
  uint64_t state_bytes;
  void *workspace;             /* device, caller-owned, >= workspace_bytes of mclg_sizes */
  uint64_t workspace_bytes;
  /* MCLG_D2Q9 only (NULL for D1Q3, where lambda_num/den and n_max apply): */
  const uint64_t *Ly;          /* host [n_replicas]; L[r] is then Lx; Lx Ly <= 2^28 */
  const uint32_t *lambda9;     /* host [18]: lambda_c = lambda9[2c-2] / lambda9[2c-1] in
                                  [0, 1], c = 1..9 (the D2Q9 classes below) */
} mclg_config;

typedef struct {
  uint32_t kind;               /* MCLG_INIT_COUNTS or MCLG_INIT_POISSON */
  const uint16_t *counts;      /* COUNTS: device [sum_r 3 L[r]] uint16, replica r's
                                  block is [3][L[r]] (n_-1, n_0, n_+1 rows) in
                                  logical site order; replicas packed densely */
  const double *rho;           /* POISSON: host [n_replicas], mean density >= 0 */
  const double *u0;            /* POISSON: host [n_replicas], velocity in [-1, 1]
                                  (D2Q9: its x component) */
  const double *u0y;           /* D2Q9 POISSON: host [n_replicas], y velocity, or NULL
                                  for 0.  D2Q9 COUNTS: replica r's block is
                                  [9][Ly][Lx] in logical order */
} mclg_init_spec;

/* Exact integer sums over the sites of one replica (modulo 2^64). */
typedef struct {
  int64_t t;           /* steps taken */
  int64_t sites;       /* L */
  int64_t sum_n[3];    /* sum_x n_i(x), i = -1, 0, +1 */
  int64_t sum_n2[3];   /* sum_x n_i(x)^2 */
  int64_t sum_nn[3];   /* sum n_-1 n_0, sum n_0 n_+1, sum n_-1 n_+1 */
  int64_t sum_N;       /* sum N(x) */
  int64_t sum_J;       /* sum J(x) = n_+1 - n_-1 */
  int64_t sum_N2;      /* sum N(x)^2 */
  int64_t n0_odd;      /* sites with odd n_0 (conserved per site) */
  int64_t max_N;       /* max_x N(x) */
  int64_t fourier[MCLG_MAX_MODES][2]; /* sum N(x) tw[2m][x], sum N(x) tw[2m+1][x] */
  /* With MCLG_MOMENTS_DIGEST (else 0): a checksum of the whole logical state,
   *   sum over x < L and i = 0, 1, 2 (v = -1, 0, +1) of
   *   fmix32(fmix32(4 x + i + 1) ^ n_i(x))   (mod 2^64),
   * fmix32 the 32-bit finaliser of MurmurHash3 (k ^= k >> 16; k *= 0x85ebca6b;
   * k ^= k >> 13; k *= 0xc2b2ae35; k ^= k >> 16).  Two states with equal
   * digests are equal unless a 2^-32-probability coincidence occurs; used to
   * compare runs without copying the state. */
  int64_t digest;
} mclg_moments_t;

#define MCLG_MOMENTS_DIGEST 1u  /* mclg_moments flag: also compute the state digest */

/* ---- D2Q9 (Sec. "A D2Q9 implementation") ----
 * Velocities numbered as the columns of the moment matrix Eq. (MomD2Q9):
 * 0 (0,0), 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1), 5 (1,1), 6 (-1,1), 7 (-1,-1),
 * 8 (1,-1); weights 4/9, 1/9, 1/36.  The paper leaves the binary collision
 * rules to a missing figure; the library (and its tests) take every swap of
 * an unordered velocity pair A = {i, j} for another pair B = {k, l} of the
 * same total momentum, with
 *   P(A -> B) = lambda_c min(1, m_B w_k w_l / (m_A w_i w_j)),
 * m = 2 for two different velocities and 1 for two equal ones (detailed
 * balance with respect to the product weights; the D1Q3 table is the same
 * rule), and number the classes c as the lambda_c of the linearised collision
 * term Eq. (D2Q9MOmega), whose coefficients this rule reproduces:
 *   1 {0,5}<->{1,2},  2 rest <-> axis pair,  3 rest <-> diagonal pair,
 *   4 axis <-> diagonal pair,  5 axis <-> axis pair,  6 diagonal <-> diagonal,
 *   7 {0,1}<->{2,8}, {0,1}<->{4,5},  8 {2,8}<->{4,5},  9 {1,1}<->{5,8},
 * and rotations by 90 degrees.  A sub-collision draws the ordered pair of
 * distinct particles as in D1Q3, then one uniform integer u in [0, D), D =
 * 128 lcm(lambda denominators) < 2^32: the targets of A in ascending
 * (min(k,l), max(k,l)) take consecutive ranges of D P(A -> B) values of u.
 * Sub-collision k of site s at step t reads Philox block (s, t, replica,
 * 2 | k << 2): Lemire draws of the first particle (word 0, of N), the second
 * (word 1, of N - 1) and u (word 2), the last one always; a rejected draw
 * continues on the words of blocks (s, t, replica, 2 | (C + j) << 2), j = 0,
 * 1, ... .  Every site runs this literal loop (the (N, Jx, Jy) fibers are too
 * many to tabulate).  Streaming: n_i(x + vx, y + vy, t + 1) <- n_i(x, y, t),
 * periodic; site s = y Lx + x keys the RNG as x does in D1Q3, and the Poisson
 * start of site s uses Philox blocks (s, j, replica, 1), j = 0..2, word w of
 * block j for velocity 4j + w, at f^eq of Eq. (D2Q9eqdist) evaluated as
 * (rho Fx[vx]) Fy[vy] with F the unit-density D1Q3 equilibrium.
 * D2Q9 contexts support mclg_sizes, mclg_init, mclg_step, mclg_get_counts
 * (host_out [9][Ly][Lx]), mclg_moments9, mclg_histogram, mclg_check and
 * mclg_destroy; the other entry points return MCLG_E_UNSUPPORTED. */
typedef struct {
  int64_t t, sites;
  int64_t sum_n[9];
  int64_t sum_nn[45];  /* sum n_i n_j for i <= j, row-major upper triangle */
  int64_t sum_N, sum_Jx, sum_Jy, max_N;
} mclg_moments9_t;

/* Exact moments of every replica of a D2Q9 context; synchronises. */
int mclg_moments9(mclg_ctx *ctx, mclg_moments9_t *host_out);

/* Host-only inspection of the D2Q9 rule table for lambda9 (18 values): per
 * ordered source pair (v1, v2), 12 uint32 at host_out[(v1 * 9 + v2) * 12]:
 * the cumulative integer weights of its (up to four) targets in order, D for
 * absent ones; then for q = 0..4 the change of the nine counts when the
 * target draw u in [0, D) has q cumulative weights <= u (q = number of
 * targets: no change), 3 bits per velocity i at bit 3i holding 2 + change;
 * and the denominator D. */
int mclg_d2q9_rules(const uint32_t *lambda9, uint32_t *host_out, uint32_t *D);

/* Bytes of device state and workspace needed by a configuration (state,
 * workspace and stream fields are ignored).  The state holds, per replica,
 * three uint16 arrays padded to 128 elements, in an internal in-place
 * shifted layout (use mclg_get_counts for logical order). */
int mclg_sizes(const mclg_config *cfg, uint64_t *state_bytes, uint64_t *workspace_bytes);

/* Validate cfg, build (or reuse) the exact collision tables on the host,
 * upload them into the workspace, write the initial state (t = 0) and
 * synchronise the stream.  On success *out owns a host context. */
int mclg_init(const mclg_config *cfg, const mclg_init_spec *init, mclg_ctx **out);

/* Enqueue n_steps steps of every replica (one batched launch per step). */
int mclg_step(mclg_ctx *ctx, uint64_t n_steps);

/* Enqueue n_steps steps of one replica only (one launch per step): the plain
 * per-lattice schedule.  Replicas may then differ in t. */
int mclg_step_replica(mclg_ctx *ctx, uint32_t replica, uint64_t n_steps);

/* Capture n_steps batched steps in a HIP graph (once per distinct n_steps)
 * and launch it; same results as mclg_step. */
int mclg_step_graph(mclg_ctx *ctx, uint64_t n_steps);

/* Exact moments of every replica into host_out[n_replicas]: the integer
 * sums behind the paper's statistics -- means and variances of n_i
 * (Eq. (poisson)), the correlator of Eq. (corr), the conserved N and J, and
 * Fourier projections of the density (Eq. (A), S(k)).  Synchronises.
 * twiddle: device int32, NULL when n_modes = 0; replica r's block is
 * [2 n_modes][L[r]], blocks packed densely in replica order.  flags: 0 or
 * MCLG_MOMENTS_DIGEST.  Uses the workspace; MCLG_E_INVAL for n_modes > 8,
 * a missing twiddle or unknown flags. */
int mclg_moments(mclg_ctx *ctx, const int32_t *twiddle, uint32_t n_modes, uint32_t flags,
                 mclg_moments_t *host_out);

/* For callers that cannot allocate memory or synchronise -- code under HIP
 * graph capture, tight serving or logging loops, harnesses that forbid
 * hipMalloc: mclg_moments with the same arguments and results, but written
 * to device memory and without any allocation (no hipMalloc, hipFree or
 * host allocation) or synchronisation.
 *   dev_out: device, caller-owned, n_replicas mclg_moments_t in replica
 *     order, written in stream order on the context's stream (read it after
 *     synchronising with that stream); t is the device's step counter (the
 *     steps taken modulo 2^32).
 *   Partial sums live in a static 8 MiB area of device memory, one per GPU,
 *     allocated with the library's code and kept until the process ends; a
 *     call needs 256 bytes per segment of the context's sites (at most
 *     512 + n_replicas + sites / 2^23 segments): MCLG_E_TOO_LARGE when that
 *     exceeds 8 MiB, i.e. for more than about 32000 replicas.
 *   Every call on a GPU uses that GPU's one area and overwrites what it
 *     reads, so nothing needs clearing between calls, but calls that overlap
 *     on one GPU (other streams, other threads) race: serialise them.
 * D2Q9 contexts: MCLG_E_UNSUPPORTED. */
int mclg_moments_noalloc(mclg_ctx *ctx, const int32_t *twiddle, uint32_t n_modes,
                         uint32_t flags, mclg_moments_t *dev_out);

/* The logging loop of a run that records its observables: n_logs times,
 * enqueue `every` steps (as mclg_step) and then the moments of the state
 * they reach (as mclg_moments: same arguments, same values) into dev_out,
 * in stream order on the context's stream, without synchronising.
 *   dev_out: device, caller-owned, n_logs x n_replicas mclg_moments_t (log j
 *     of replica r at j n_replicas + r); t is the device's step counter (the
 *     steps taken modulo 2^32).
 *   With several steps per launch on whole ranges (mclg_set_blocked for
 *     one lattice, not in tiles), at most two modes and not two modes with
 *     MCLG_MOMENTS_DIGEST, the run goes in launches of that many steps (the
 *     last one shorter) and each launch sums the logs that fall in it from
 *     the blocks' copies, the last one as it writes the sites back: the
 *     state is not read again, and one launch covers several logs when
 *     `every` is below its steps.  With the digest or MCLG_FLAG_GALILEAN a
 *     launch ends at each log.  Otherwise the moment kernels run after each
 *     interval's steps.  Either way the partial sums live in the blocked
 *     scratch or the workspace, so calls on one context are stream-ordered
 *     and need no clearing.
 * MCLG_E_INVAL for every = 0, every x n_logs >= 2^62 and as mclg_moments;
 * D2Q9 contexts: MCLG_E_UNSUPPORTED. */
int mclg_step_log(mclg_ctx *ctx, uint64_t every, uint64_t n_logs, const int32_t *twiddle,
                  uint32_t n_modes, uint32_t flags, mclg_moments_t *dev_out);

/* Logical counts of one replica into host_out[3][L]; synchronises. */
int mclg_get_counts(mclg_ctx *ctx, uint32_t replica, uint16_t *host_out);

/* Occupation-number histograms, the distributions P(n_i) compared with the
 * Poisson law of Eq. (poisson) (Fig. of the Poisson section for D2Q9) and,
 * in the rest-parity sector, with Fig. 1 of the D1Q3 section.  Adds, for
 * every replica r, velocity i (D1Q3: 0, 1, 2 for v = -1, 0, +1; D2Q9: the
 * nine velocities, V = 9) and site x, one to
 *   dev_hist[(r * V + i) * n_bins + min(n_i(x), n_bins - 1)],   V = 3 or 9,
 * so the last bin counts every n_i >= n_bins - 1.  dev_hist is device memory
 * of n_replicas * V * n_bins uint64 owned by the caller, who clears it; calls
 * accumulate, so repeated calls sum histograms over time.  Asynchronous on the
 * context's stream (read dev_hist after synchronising with it).  n_bins in
 * 1..MCLG_MAX_HIST_BINS (D2Q9: 1..1024), else MCLG_E_INVAL; overflow of a
 * site is reported by mclg_check, not here. */
int mclg_histogram(mclg_ctx *ctx, uint32_t n_bins, uint64_t *dev_hist);

/* Sticky error state of the device (MCLG_E_RANGE if any site overflowed);
 * synchronises. */
int mclg_check(mclg_ctx *ctx);

/* Select the launch schedule: chunks of eight sites per lane per tile (must
 * be 1), threads per block (64..1024, multiple of 64) and the
 * bytes of LDS each block devotes to its replica's collision image (0..163840,
 * capped by what the device's LDS leaves beside the per-wave queues;
 * the image caches the most visited table rows, misses read the exact rows in
 * global memory).  Any choice gives identical bits; synchronises the stream. */
int mclg_set_schedule(mclg_ctx *ctx, uint32_t groups_per_thread, uint32_t threads_per_block,
                      uint32_t lds_budget_bytes);

/* Upper bound on the persistent grid of the step kernel (0 = as many blocks
 * as fit on the device, the default).  A smaller grid gives each wave longer
 * runs of chunks (and leaves CUs to other work); any value gives identical
 * bits.  Drops captured graphs; synchronises the stream. */
int mclg_set_grid_limit(mclg_ctx *ctx, uint32_t max_blocks);

/* When the step kernel resolves the draws its LDS image cannot decide (from
 * the exact tables in the workspace): every policy gives identical bits.
 *   MCLG_DRAIN_AUTO (default): DEFERRED when a launch's state fits the 256 MB
 *     Infinity Cache, else PATCH;
 *   MCLG_DRAIN_DEFERRED: a wave queues up to 96 draws across chunks and
 *     writes their outcomes afterwards (2-byte stores into stored lines);
 *   MCLG_DRAIN_CHUNK: the same after every chunk;
 *   MCLG_DRAIN_PATCH: each chunk's draws are resolved before the chunk's
 *     stores, so every count is written once.
 * Drops captured graphs; synchronises the stream; MCLG_E_INVAL for an
 * unknown policy. */
enum { MCLG_DRAIN_AUTO = 0, MCLG_DRAIN_DEFERRED = 1, MCLG_DRAIN_CHUNK = 2, MCLG_DRAIN_PATCH = 3 };
int mclg_set_drain(mclg_ctx *ctx, uint32_t policy);

/* Several steps per launch (temporal blocking) for a context of lattices
 * (Sec. "The D1Q3 model": the update of a site at t + 1 reads only its
 * neighbours at t, so a block that holds its sites and `steps` more on each
 * side can advance them `steps` steps alone).  mclg_step then launches
 * whole groups of `steps` steps, each group as one launch: every block
 * copies its range of the state and the extra sites into its part of
 * `scratch`, waits for all blocks (a grid-wide barrier), advances its copy,
 * and writes its own sites back; the rest of a mclg_step call takes single
 * steps.  The bits are the same as with one step per launch.
 *   tile: 1 = each block copies its whole range (about L / 256 sites); >= 2
 *     = each block goes through its range in tiles, copies of `tile` sites
 *     (a multiple of 8, more than 2 x steps rounded up to 8, at most 2^20)
 *     whose own tile - 2 x (steps rounded up to 8) sites it writes back
 *     before the next tile, so that the copies stay in the caches when the
 *     ranges would not; 0 = whole ranges while all blocks' copies fit
 *     128 MiB, else tiles of 65536 sites.
 *   Several replicas: each block advances whole replicas (the host deals
 *     them out, longest first), each copied whole with its own image, so
 *     every replica length works; tile must be 0 or 1, and the scratch
 *     holds one copy of the largest replica per block.  mclg_set_blocked
 *     then uploads the blocks' replica lists and synchronises the stream.
 *   mclg_blocked_bytes: the scratch bytes `steps` steps per launch need (the
 *     blocks' copies, and room for the partial sums of mclg_step_log).
 *   mclg_set_blocked: steps in [2, 256] with scratch (device, caller-owned,
 *     at least mclg_blocked_bytes, kept until blocking is switched off or the
 *     context destroyed); steps <= 1 switches it off (scratch unused).
 * MCLG_E_UNSUPPORTED for D2Q9, a schedule other than 1024 threads, and for
 * one lattice L not a multiple of 8 or too short for the extra sites of 256
 * or so blocks; MCLG_E_INVAL for steps > 256, a bad `tile` or too small a
 * scratch.  mclg_set_schedule switches blocking off.
 * Graph launches (mclg_step_graph) take one step per launch. */
int mclg_blocked_bytes(mclg_ctx *ctx, uint32_t steps, uint32_t tile, uint64_t *scratch_bytes);
int mclg_set_blocked(mclg_ctx *ctx, uint32_t steps, uint32_t tile, void *scratch,
                     uint64_t scratch_bytes);

/* Expected fraction of site updates whose draw is decided from LDS (from the
 * product-Poisson law the images were built for) and the LDS bytes per block. */
int mclg_lds_coverage(const mclg_ctx *ctx, double *expected_fraction, uint32_t *lds_bytes);

int mclg_destroy(mclg_ctx *ctx);
const char *mclg_strerror(int code);
int mclg_last_hip_error(const mclg_ctx *ctx);

/* ---- Host-only inspection (no GPU needed) ---- */

/* Quantised row of the collision law: for the fiber (N, absJ) and incoming
 * rest count n0, writes the full-fiber thresholds (m - 1 values as uint64,
 * value 2^32 meaning "never") to thr, m = (N - absJ)/2 + 1 to *m_out.
 * flags: 0 or MCLG_FLAG_GALILEAN. */
int mclg_table_row(int32_t C, uint32_t lambda_num, uint32_t lambda_den, uint32_t flags,
                   uint32_t N, uint32_t absJ, uint32_t n0, uint64_t *thr, uint32_t cap,
                   uint32_t *m_out);

/* Numerator over 2^32 of the Galilean-invariant acceptance of fiber
 * (N, absJ) (MCLG_FLAG_GALILEAN) for lambda~ = num / den. */
int mclg_galilean_lambda(uint32_t num, uint32_t den, uint32_t N, uint32_t absJ,
                         uint64_t *lambda_q);

/* Poisson(mu) thresholds of the initial-state rule: outcomes k_lo..k_lo+cnt-1,
 * cnt - 1 thresholds (uint64) to thr. */
int mclg_poisson_thresholds(double mu, uint32_t *k_lo, uint32_t *cnt, uint64_t *thr,
                            uint32_t cap);

/* ---- Serving: continuous batching of simulation jobs ---- */

typedef struct mclg_server mclg_server;

typedef struct {
  uint32_t abi_version;
  uint32_t max_slots;          /* concurrent jobs */
  uint64_t seed;
  int32_t C;
  uint32_t lambda_num, lambda_den, n_max;
  void *stream;
  void *arena;                 /* device, caller-owned: job states */
  uint64_t arena_bytes;        /* admission budget */
  void *workspace;             /* device, caller-owned, >= mclg_server_sizes */
  uint64_t workspace_bytes;
} mclg_server_config;

typedef struct {
  uint64_t job_id;             /* RNG replica identity (< 2^32) and handle */
  uint64_t L;                  /* sites, 1 <= L <= 2^29 */
  uint64_t steps;              /* steps to run */
  double rho, u0;              /* Poisson initial state */
} mclg_job;

typedef struct {
  uint64_t job_id;
  mclg_moments_t moments;      /* final exact moments (t = steps) */
} mclg_job_result;

int mclg_server_sizes(const mclg_server_config *cfg, uint64_t *workspace_bytes);
int mclg_server_create(const mclg_server_config *cfg, mclg_server **out);
/* Queue a job (host only).  MCLG_E_INVAL if it can never fit the arena. */
int mclg_server_submit(mclg_server *srv, const mclg_job *job);
/* Admit queued jobs while slots and arena space allow (first-fit, FIFO
 * order), then enqueue k batched steps of every resident job; jobs that
 * reach their step count are retired (moments computed, space freed). */
int mclg_server_tick(mclg_server *srv, uint32_t k);
/* Copy up to cap finished results to out; *n_out = number copied. */
int mclg_server_poll(mclg_server *srv, mclg_job_result *out, uint32_t cap, uint32_t *n_out);
/* Jobs queued, resident, and arena bytes in use. */
int mclg_server_stats(const mclg_server *srv, uint64_t *queued, uint64_t *resident,
                      uint64_t *arena_used);
int mclg_server_destroy(mclg_server *srv);

#ifdef __cplusplus
}
#endif
#endif
