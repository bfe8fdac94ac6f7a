// Two-level aggregation multigrid (mg.hip).
#pragma once

#include "internal.h"

namespace lq {

// Aggregate extents a (x, y, z, t): each >= 2, dividing the lattice into an
// even number of aggregates per direction, at most 256 sites per aggregate.
bool mg_shape_ok(const Geom& g, const int a[4]);
// Test vectors from prm.nvec canonical FP64 device fields at start (back to
// back), prm.setup_iters rounds of SAP smoothing of D v = 0 (v <- v - M D v)
// and aggregate-wise orthonormalisation, then the coarse operator; replaces
// any earlier setup.
int mg_setup(lqcd_ctx* c, const lqcd_mg_params& prm, const double* start);
// complex entries of a coarse vector (0 without a setup)
size_t mg_coarse_size(lqcd_ctx* c);
// rc = P^dag r (FP32 native halves in, FP32 complex coarse vector out)
int mg_restrict(lqcd_ctx* c, const void* r_e, const void* r_o, void* rc);
// x = P ec (FP32 complex coarse vector in, FP32 native halves out)
int mg_prolong(lqcd_ctx* c, const void* ec, void* x_e, void* x_o);
// out = D_c in (FP32 complex coarse vectors)
int mg_coarse_apply(lqcd_ctx* c, const void* in, void* out);
// x = the two-level preconditioner applied to r (FP32 native halves)
int mg_precond(lqcd_ctx* c, const void* r_e, const void* r_o, void* x_e, void* x_o, int* coarse_iters);
// D x = b (FP64 native halves) by flexible BiCGStab with the two-level
// preconditioner; coarse_iters_total: coarse BiCGStab iterations summed
int solve_mg(lqcd_ctx* c, const lqcd_solve_params& prm, const void* b_e, const void* b_o, void* x_e, void* x_o,
             bool zero_x, lqcd_solve_stats& st, long* coarse_iters_total);
// coarse vectors: FP32 complex <-> complex128
int mg_coarse_convert(lqcd_ctx* c, const void* src, bool src_f64, void* dst, size_t n);

}  // namespace lq
