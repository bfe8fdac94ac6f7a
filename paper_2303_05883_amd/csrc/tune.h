// Hop launch-shape autotuner (tune.hip).
#pragma once

#include "internal.h"

namespace lq {

// Apply cached launch shapes for this lattice from $LQCD_TUNE_CACHE, if any.
int tune_load_defaults(lqcd_ctx* c);

}  // namespace lq
