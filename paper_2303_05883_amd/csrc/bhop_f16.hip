// Batched hop kernels with FP16 storage (FP32 arithmetic) fields (see bhop.h).
#include "bhop.h"

namespace lq {

template <>
int launch_bhop<2>(const BHopArgs& a, const BShape& sh, int epi, int red, bool clov, hipStream_t s) {
  LQ_BHOP_LAUNCH_NB(2, 1)
  LQ_BHOP_LAUNCH_NB(2, 2)
  LQ_BHOP_LAUNCH_NB(2, 3)
  LQ_BHOP_LAUNCH_NB(2, 4)
  return set_error(LQCD_EINVAL, "unsupported right-hand sides per lane in the batched hop");
}

}  // namespace lq
