// Hop launch-shape autotuner (tune.hip).
#pragma once

#include <string>

#include "internal.h"

namespace lq {

// Apply cached launch shapes for this lattice from $LQCD_TUNE_CACHE, if any.
int tune_load_defaults(lqcd_ctx* c);
// A tuner's entry under key in the LQCD_TUNE_CACHE file: four integers (kept
// in the fields block, split, remap, nt) and the time; get returns false when
// there is no cache or no entry, put does nothing without a cache.
bool tune_cache_get(const std::string& key, int v[4]);
int tune_cache_put(const std::string& key, const int v[4], double us);

}  // namespace lq
