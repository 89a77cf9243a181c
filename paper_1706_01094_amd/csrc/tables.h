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
  bool galilean = false;          // per-fiber lambda of galilean_lambda_q
  std::vector<uint32_t> rowbase;
  std::vector<uint32_t> rowdesc;  // pairs (offset, k_first | q << 16)
  std::vector<uint32_t> thr;
  uint32_t max_q = 0;             // largest number of outcomes in a row
  // The same rows at a fixed stride of kFixedStride uint32 (when max_q allows):
  // row r = {k_first | q << 16, thresholds..., zero padding}, so that a row
  // is found from (N, |J|, n0) by arithmetic and read in one round of loads.
  std::vector<uint32_t> fixed;    // empty when not built
  // The same rows as 64 bytes of 16-bit values: k_first, q, the top 16 bits
  // of the q - 1 thresholds, then 0xFFFF (when max_q <= 31).  A draw r whose
  // top 16 bits equal none of them is decided by the row alone: a threshold
  // with smaller top bits is <= r, one with larger top bits is > r.
  std::vector<uint16_t> row16;    // empty when not built
};

// Build (or fetch from the process cache) the tables for (C, lambda, n_max),
// with the Galilean-invariant per-fiber lambda when `galilean` is set.
// Returns nullptr for invalid parameters.
std::shared_ptr<const CollisionTables> collision_tables(int32_t C, uint32_t lam_p,
                                                        uint32_t lam_q, uint32_t n_max,
                                                        bool galilean);

// Full-fiber thresholds (uint64, 2^32 = "never") of one row, for inspection.
bool collision_row_full(int32_t C, uint32_t lam_p, uint32_t lam_q, bool galilean, uint32_t N,
                        uint32_t absJ, uint32_t n0, std::vector<uint64_t> &thr);

bool params_ok(int32_t C, uint32_t lam_p, uint32_t lam_q, uint32_t n_max, bool galilean);

// Galilean-invariant acceptance of fiber (N, |J|) for lambda~ = num / den, as
// a numerator over 2^32: floor(floor(2^32 N / sqrt(N^2 + 3 J^2)) num / den)
// (exact integer arithmetic; 2^32 num / den for J = 0).
uint64_t galilean_lambda_q(uint32_t num, uint32_t den, uint32_t N, uint32_t absJ);

// Equilibrium means of Eq. (D1Q3equil) with the stated IEEE evaluation order.
void feq(double rho, double u, double out[3]);

// Poisson(mu) thresholds of the initial-state rule (full list, uint64).
bool poisson_full(double mu, uint32_t &k_lo, std::vector<uint64_t> &thr);

// LDS image of the hottest collision rows of one workload (a performance
// cache: every site it cannot decide goes to the exact global tables, so the
// results never depend on it).
//
// A row is addressed by (a', b, c') = (min(n_-1, n_+1), n_0, max(n_-1, n_+1)),
// which fixes N, |J| and n0.  With np pairs in the image, records come in
// np + 1 rows of nb + 1: row p holds the pair's records for b = b_lo ..
// b_lo + nb - 1, then one never record; row np is all never records.  `dir`
// holds (dim_a + 1) x (dim_c + 1) entries: dir[a' (dim_c + 1) + c'] is the
// index of the first record of an (a', c') pair (in 16-byte units from the
// start of the image, whose directory comes first), that of row np for an
// absent pair, and row dim_a and column dim_c are absent pairs, so that a
// site's record is image16[dir[min(a', dim_a) (dim_c + 1) + min(c', dim_c)] +
// min(b - b_lo mod 2^16, nb)] without a range test.  A record is eight
// uint16: (b >> 1) - k_s as int16, then a lower bound L = ceil(thr_{k_s-1} /
// 2^16), the top 16 bits of thr_{k_s} .. thr_{k_s+4} (inner values), and the
// top 16 bits of thr_{k_s+5} as upper bound U (thr_{-1} = 0, thr_{>= m - 1} =
// 2^32; all clamped to 0xFFFF).  With rh = r >> 16 the draw is decided in LDS
// when L <= rh < U and no inner value equals rh; then the outcome index is
// k_s + #{inner value < rh}, i.e. the site's n0 moves by -2 ((b >> 1) - k_s -
// #{inner value < rh}).  Never records have L = 0xFFFF and U = 0 and decide
// nothing: the exact global row decides.  A pair with N < 2 (no collision)
// gets records (0, 0, 0xFFFF x 6): move 0 for every rh < 0xFFFF.  Without room
// for any pair the image is a one-entry directory and two never records
// (np = 0, nb = 1).
struct LdsImage {
  uint32_t dim_a = 0, dim_c = 0, b_lo = 0, nb = 0;
  std::vector<uint16_t> dir;      // (dim_a + 1) * (dim_c + 1)
  std::vector<uint16_t> records;  // 8 per record
  double coverage = 0.0;          // expected fraction of site updates decided in LDS
  // serialised: dir padded to 16 bytes, then the records
  std::vector<uint8_t> blob() const;
  uint32_t dir_bytes() const {
    return (uint32_t)(((dim_a + 1) * (dim_c + 1) * 2 + 15) / 16 * 16);
  }
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
