// Host-side exact tables of the MCLG library.
//
// Collision tables: for every fiber (N, |J|) with N <= n_max and every
// incoming rest count n0, the law of n0' after C sub-collisions (or the
// fiber equilibrium for C = infinity), quantised to uint32 thresholds.
// Poisson tables: the initial-state thresholds.  See mclg.h for the rules.
#pragma once
#include <cstdint>
#include <memory>
#include <vector>

namespace mclg {

// Device image of the collision tables (copied verbatim to the workspace).
//   rowbase[N (N + 1) / 2 + |J|] = index of the fiber's first row
//   rowdesc[rowbase + (n0 - par) / 2] = {thr offset, k_first | q << 16},
//     par = (N - |J|) mod 2 (fiber states ascend in n0 = par + 2k)
//   thr[offset .. offset + q - 2] ascending uint32 thresholds
// Sampling: n0' = ((N - |J|) & 1) + 2 (k_first + #{i : thr[offset + i] <= r}).
struct CollisionTables {
  int32_t C = 0;
  uint32_t lam_p = 1, lam_q = 1, n_max = 0;
  std::vector<uint32_t> rowbase;
  std::vector<uint32_t> rowdesc;  // pairs (offset, k_first | q << 16)
  std::vector<uint32_t> thr;
  uint32_t max_q = 0;             // largest number of outcomes in a row
};

// Build (or fetch from the process cache) the tables for (C, lambda, n_max).
// Returns nullptr for invalid parameters.
std::shared_ptr<const CollisionTables> collision_tables(int32_t C, uint32_t lam_p,
                                                        uint32_t lam_q, uint32_t n_max);

// Full-fiber thresholds (uint64, 2^32 = "never") of one row, for inspection.
bool collision_row_full(int32_t C, uint32_t lam_p, uint32_t lam_q, uint32_t N, uint32_t absJ,
                        uint32_t n0, std::vector<uint64_t> &thr);

bool params_ok(int32_t C, uint32_t lam_p, uint32_t lam_q, uint32_t n_max);

// Equilibrium means of Eq. (D1Q3equil) with the stated IEEE evaluation order.
void feq(double rho, double u, double out[3]);

// Poisson(mu) thresholds of the initial-state rule (full list, uint64).
bool poisson_full(double mu, uint32_t &k_lo, std::vector<uint64_t> &thr);

// Compacted form used on the device: n = k_first + #{thr[i] <= r}.
struct CompactLaw {
  uint32_t k_first = 0;
  std::vector<uint32_t> thr;  // q - 1 values, all < 2^32
};
CompactLaw compact(uint32_t k_lo, const std::vector<uint64_t> &full);

}  // namespace mclg
