// D2Q9 contexts of the MCLG library (host side): layout, collision rules,
// launches.  The rules and the layout are described in mclg.h.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/mclg.h"
#include "device.h"
#include "moments.h"

namespace mclg {

struct D2Ctx {
  uint32_t n = 0, flags = 0, D = 0;
  int32_t C = 0;
  uint64_t seed = 0;
  int64_t t = 0;
  std::vector<uint64_t> Lx, Ly, rid, dense;
  std::vector<Rep9> reps;
  std::vector<Tile9> tiles;
  std::vector<uint32_t> rules;      // 81 x kRule9Words
  std::vector<uint32_t> rules_dev;  // 81 x kRule9DevWords
  uint64_t state_bytes = 0, ws_bytes = 0;
  uint64_t o_err = 0, o_reps = 0, o_tiles = 0, o_rules = 0, o_pdesc = 0, o_pool = 0,
           o_dense = 0;
  MomPlan mplan;  // moment kernels: segments and runs (one per replica)
  uint64_t o_mseg = 0, o_mrun = 0, o_mslot = 0, o_mpart = 0, o_mout = 0;
  uint16_t *state = nullptr;
  uint8_t *ws = nullptr;
  hipStream_t stream = nullptr;
  int last_hip = 0;
};

// Collision rule table of mclg.h for lambda9 (18 values); false when a
// lambda is not in [0, 1], D would reach 2^32, or a source's targets would
// add up to more than one.
bool build_rules9(const uint32_t *lambda9, std::vector<uint32_t> &rules, uint32_t &D);

// The rules as the step kernel reads them, per ordered source pair,
// kRule9DevWords uint32: words 0-3 the cumulative weights (as in the table
// of mclg.h); then, for q = 0..4, four words holding the change of the
// partial sums K_j = n_0 + ... + n_j (j = 0..7) as 16-bit two's-complement
// pairs, K_2m in the low and K_2m+1 in the high half.
constexpr uint32_t kRule9DevWords = 24;
std::vector<uint32_t> device_rules9(const std::vector<uint32_t> &rules);

// Validate a D2Q9 configuration and fill the layout (sizes and offsets).
int d2q9_layout(const mclg_config *cfg, D2Ctx &d);
int d2q9_init(D2Ctx &d, const mclg_config *cfg, const mclg_init_spec *init);
int d2q9_step(D2Ctx &d, uint64_t n_steps);
int d2q9_get_counts(D2Ctx &d, uint32_t r, uint16_t *out);
int d2q9_moments(D2Ctx &d, mclg_moments9_t *out);
int d2q9_check(D2Ctx &d);
int d2q9_histogram(D2Ctx &d, uint32_t n_bins, uint64_t *dev_hist);

}  // namespace mclg
