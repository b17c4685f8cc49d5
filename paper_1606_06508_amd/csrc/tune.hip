// Launch-configuration choice for the evaluation kernels.
#include "fh_internal.h"

namespace fhk {

EvalConfig choose_eval_config(int32_t prec, int64_t n, int32_t d, int64_t m, bool want_r,
                              bool want_l) {
  (void)prec; (void)n; (void)d; (void)want_r; (void)want_l;
  EvalConfig c;
  c.block = 256;
  // enough waves to fill 256 CUs x 4 SIMDs before raising points per lane
  const int64_t waves_p4 = (m + 255) / 256;
  c.points_per_lane = waves_p4 >= 4096 ? 4 : (m >= 256 * 1024 * 2 ? 2 : 1);
  return c;
}

}  // namespace fhk
