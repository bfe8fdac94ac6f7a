// Batched solves over several lattices and right-hand sides.
#include "internal.h"

extern "C" int lqcd_solve_batch(lqcd_ctx* const* ctxs, const int* nrhs, const double* const* b, double* const* x,
                                int nlattices, const lqcd_solve_params* prm, lqcd_solve_stats* stats) {
  if (!ctxs || !nrhs || !b || !x || nlattices < 1) return lq::set_error(LQCD_EINVAL, "null argument");
  int idx = 0;
  for (int l = 0; l < nlattices; ++l) {
    const size_t n = (size_t)ctxs[l]->g.vh * 2 * 24;
    for (int r = 0; r < nrhs[l]; ++r, ++idx) {
      lqcd_solve_stats st{};
      const int s = lqcd_solve(ctxs[l], b[l] + r * n, x[l] + r * n, prm, &st);
      if (stats) stats[idx] = st;
      if (s != LQCD_OK) return s;
    }
  }
  return LQCD_OK;
}
