/*
 * mclg_oracle.h -- reference (oracle) implementation of the Monte Carlo
 * Lattice Gas (MCLG) on a periodic D1Q3 lattice.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded CPU
 * implementation written to be checked by eye against the paper
 * (Blommel & Wagner, "Integer Lattice Gas with Monte Carlo collision operator
 * recovers the entropic lattice Boltzmann method with Poisson distributed
 * fluctuations", arXiv:1706.01094).  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code with
 * the HIP library: its own Philox, its own big-integer table builder, its own
 * Poisson threshold builder, its own stream/collide and moment sums.
 *
 * Every function that produces a number from the method cites the passage of
 * the paper it follows; where the paper is silent the stated build rule is
 * named instead (the same rules the HIP library implements independently).
 */
#ifndef MCLG_ORACLE_H
#define MCLG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MCO_OK = 0, MCO_E_INVAL = -1, MCO_E_RANGE = -2, MCO_E_NOMEM = -3 };
enum {
  MCO_FLAG_NO_STREAM = 1u, /* collisions only, no streaming */
  MCO_FLAG_GALILEAN = 2u   /* lambda = lambda~ / sqrt(1 + 3 (J/N)^2) per site (R7) */
};
#define MCO_C_EQUILIBRIUM (-1)      /* C -> infinity: redraw from fiber equilibrium */
#define MCO_MAX_MODES 8

typedef struct mco_sim mco_sim;

/* Exact integer moments of one replica (all sums over sites x). */
typedef struct {
  int64_t t;          /* steps taken by this replica */
  int64_t sites;      /* L */
  int64_t sum_n[3];   /* sum n_i, i = -1, 0, +1 */
  int64_t sum_n2[3];  /* sum n_i^2 */
  int64_t sum_nn[3];  /* sum n_-1 n_0, sum n_0 n_+1, sum n_-1 n_+1 */
  int64_t sum_N;      /* sum N(x) */
  int64_t sum_J;      /* sum J(x) = n_+1 - n_-1 */
  int64_t sum_N2;     /* sum N(x)^2 */
  int64_t n0_odd;     /* number of sites with odd n_0 */
  int64_t max_N;      /* max over x of N(x) */
  int64_t fourier[MCO_MAX_MODES][2]; /* sum N(x) cos_m(x), sum N(x) sin_m(x) */
} mco_moments_t;

/* Simulation of n_rep independent periodic D1Q3 lattices. */
int mco_create(uint32_t n_rep, const uint64_t *L, const uint64_t *replica_id,
               uint64_t seed, int32_t C, uint32_t lam_p, uint32_t lam_q,
               uint32_t n_max, uint32_t flags, mco_sim **out);
void mco_destroy(mco_sim *s);
/* counts: [3][L] logical order (n_-1 row, n_0 row, n_+1 row). Sets t = 0. */
int mco_init_counts(mco_sim *s, uint32_t rep, const uint16_t *counts);
/* n_i(x) ~ Poisson(f_i^eq(rho, u0)) drawn with the stated threshold rule. */
int mco_init_poisson(mco_sim *s, uint32_t rep, double rho, double u0);
/* Advance one replica by n steps (collide at every site, then stream). */
int mco_step_replica(mco_sim *s, uint32_t rep, uint64_t n);
/* Advance every replica by n steps. */
int mco_step(mco_sim *s, uint64_t n);
int mco_get_counts(const mco_sim *s, uint32_t rep, uint16_t *out);
int64_t mco_get_t(const mco_sim *s, uint32_t rep);
/* Treat replica rep as the window [xoff, xoff + L) of a larger lattice for the
 * RNG (site index x + xoff) and set its step counter to t.  The window's own
 * periodic wrap is wrong near its ends; callers keep a halo of t sites. */
int mco_set_site_offset(mco_sim *s, uint32_t rep, uint64_t xoff, int64_t t);
/* twiddle: [2*n_modes][L] int32 rows (cos_1, sin_1, cos_2, sin_2, ...) or NULL */
int mco_moments(const mco_sim *s, uint32_t rep, const int32_t *twiddle,
                uint32_t n_modes, mco_moments_t *out);

/* ---- pieces exported for the pin tests ---- */
void mco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Exact quantised row of the C-step collision kernel on fiber (N, |J|) from
 * incoming rest count n0.  thr receives m-1 thresholds (uint64, may equal
 * 2^32) where m = (N-|J|)/2 + 1; outcome k is n0' = ((N-|J|) mod 2) + 2k. */
int mco_row_thresholds(int32_t C, uint32_t lam_p, uint32_t lam_q, uint32_t flags,
                       uint32_t N, uint32_t absJ, uint32_t n0, uint64_t *thr,
                       uint32_t *m_out);
/* R7: numerator over 2^32 of the Galilean-invariant lambda of fiber (N, |J|). */
uint64_t mco_galilean_lambda(uint32_t num, uint32_t den, uint64_t N, uint64_t absJ);
/* Poisson(mu) thresholds under the stated IEEE rule: outcomes k_lo..k_lo+cnt-1,
 * thr receives cnt-1 values. Returns MCO_E_INVAL if cap too small. */
int mco_poisson_thresholds(double mu, uint32_t *k_lo, uint32_t *cnt,
                           uint64_t *thr, uint32_t cap);
void mco_feq(double rho, double u, double out[3]);
/* One collision of a site (a, b, c) -> (a', b', c') using the table sampler
 * (N <= n_max) or the direct sampler (N > n_max), with the RNG coordinates
 * (seed, replica, t, x).  Used by the statistical tests. */
int mco_collide_site(int32_t C, uint32_t lam_p, uint32_t lam_q, uint32_t flags,
                     uint32_t n_max, uint64_t seed, uint64_t replica, uint64_t t,
                     uint64_t x, uint32_t abc[3]);
/* Always the direct (literal sub-collision) sampler. */
int mco_collide_site_direct(int32_t C, uint32_t lam_p, uint32_t lam_q, uint32_t flags,
                            uint64_t seed, uint64_t replica, uint64_t t,
                            uint64_t x, uint32_t abc[3]);
/* Many draws for chi-squared tests: histogram of n0' over n_draws sites
 * x = 0..n_draws-1 at step t, all starting from (a,b,c). hist has N+1 bins. */
int mco_histogram(int32_t C, uint32_t lam_p, uint32_t lam_q, uint32_t flags, int direct,
                  uint64_t seed, uint64_t t, uint64_t n_draws,
                  const uint32_t abc[3], uint64_t *hist);

/* ---- D2Q9 (velocities numbered as the columns of Eq. (MomD2Q9)) ---- */
typedef struct mco_sim9 mco_sim9;
typedef struct {
  int64_t t, sites;
  int64_t sum_n[9];
  int64_t sum_nn[45]; /* sum n_i n_j, i <= j, row-major upper triangle */
  int64_t sum_N, sum_Jx, sum_Jy, max_N;
} mco_moments9_t;
/* lam[2c-2] / lam[2c-1] = lambda_c, c = 1..9 (classes of Eq. (D2Q9MOmega)) */
int mco9_create(uint32_t n_rep, const uint64_t *Lx, const uint64_t *Ly,
                const uint64_t *replica_id, uint64_t seed, int32_t C,
                const uint32_t lam[18], uint32_t flags, mco_sim9 **out);
void mco9_destroy(mco_sim9 *s);
/* counts: [9][Ly][Lx] */
int mco9_init_counts(mco_sim9 *s, uint32_t rep, const uint16_t *counts);
int mco9_init_poisson(mco_sim9 *s, uint32_t rep, double rho, double ux, double uy);
int mco9_step(mco_sim9 *s, uint64_t n);
int mco9_get_counts(const mco_sim9 *s, uint32_t rep, uint16_t *out);
int64_t mco9_get_t(const mco_sim9 *s, uint32_t rep);
int mco9_moments(const mco_sim9 *s, uint32_t rep, mco_moments9_t *out);
void mco9_feq(double rho, double ux, double uy, double out[9]);
/* targets of the ordered source pair (i, j): n, pairs (k <= l), classes and
 * integer weights over D */
int mco9_targets(const uint32_t lam[18], uint32_t i, uint32_t j, uint32_t *n, uint32_t k[8],
                 uint32_t l[8], uint32_t cls[8], uint64_t wgt[8], uint64_t *D);
int mco9_collide_site(int32_t C, const uint32_t lam[18], uint64_t seed, uint64_t replica,
                      uint64_t t, uint64_t s, uint32_t n9[9]);

#ifdef __cplusplus
}
#endif
#endif
