// Batched hop kernels with FP64 fields (see bhop.h).
#include "bhop.h"

namespace lq {

template <>
int launch_bhop<0>(const BHopArgs& a, const BShape& sh, int epi, int red, bool clov, hipStream_t s) {
  LQ_BHOP_LAUNCH_NB(0, 1)
  LQ_BHOP_LAUNCH_NB(0, 2)
  return set_error(LQCD_EINVAL, "unsupported right-hand sides per lane in the batched hop");
}

}  // namespace lq
