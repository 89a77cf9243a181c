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
  // The same rows at a fixed stride of kFixedStride uint32 (when max_q allows):
  // row r = {k_first | q << 16, thresholds..., zero padding}, so that a row
  // is found from (N, |J|, n0) by arithmetic and read in one round of loads.
  std::vector<uint32_t> fixed;    // empty when not built
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

// LDS image of the hottest collision rows of one workload (a performance
// cache: every site it cannot decide goes to the exact global tables, so the
// results never depend on it).
//
// A row is addressed by (a', b, c') = (min(n_-1, n_+1), n_0, max(n_-1, n_+1)),
// which fixes N, |J| and n0.  With np pairs in the image, `dir` holds
// dim_a * dim_c + 2 entries: dir[a' * dim_c + c'] is the index p of an
// (a', c') pair, or np for an absent pair; the two extra entries are the
// "never" slot (np) and the "skip" slot (np + 1).  The record of (p, b) is
// records[p * nb + b - b_lo]: eight uint16, (b >> 1) - k_s as int16, then the
// top 16 bits of the full-fiber thresholds thr_{k_s - 1} .. thr_{k_s + 5}
// (thr_{-1} = 0, thr_{>= m - 1} = 2^32, clamped to 0xFFFF).  With
// rh = r >> 16 the draw is decided in LDS when T1 < rh < T7 and no inner T
// equals rh; then the outcome index is k_s + #{inner T < rh}, i.e. the
// site's n0 moves by -2 ((b >> 1) - k_s - #{inner T < rh}).  Records of the
// never slot (and of rows the tables do not hold) have T1 = 0xFFFF and
// decide nothing: the exact global row decides.  The one skip record,
// records[(np + 1) * nb], is (0x8000, 0xFFFF, 0, ...) and marks a site that
// does not collide.  Without room for any pair the image is just the
// directory's two slots and these records (np = 0, nb = 1).
struct LdsImage {
  uint32_t dim_a = 0, dim_c = 0, b_lo = 0, nb = 0;
  std::vector<uint16_t> dir;      // dim_a * dim_c + 2
  std::vector<uint16_t> records;  // 8 per record
  double coverage = 0.0;          // expected fraction of site updates decided in LDS
  // serialised: dir padded to 16 bytes, then the records
  std::vector<uint8_t> blob() const;
  uint32_t dir_bytes() const { return (uint32_t)(((dim_a * dim_c + 2) * 2 + 15) / 16 * 16); }
};

// Build the image for a lattice near the product-Poisson law at
// f^eq(rho, u) within `budget` bytes.
LdsImage build_image(const CollisionTables &tab, double rho, double u, uint32_t budget);

// Compacted form used on the device: n = k_first + #{thr[i] <= r}.
struct CompactLaw {
  uint32_t k_first = 0;
  std::vector<uint32_t> thr;  // q - 1 values, all < 2^32
};
CompactLaw compact(uint32_t k_lo, const std::vector<uint64_t> &full);

}  // namespace mclg
