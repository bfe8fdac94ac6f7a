// Domain-wall operator and its normal-equation CG (dwf.hip).
#pragma once

#include "internal.h"

namespace lq {

// Bytes of a native 5-d field: two parity halves, each site-blocked over the
// 5-d index i Ls + s (i the 4-d checkerboard index), even half first.
size_t dwf_field_bytes(int prec, size_t vh, int Ls);
// canonical [s][t][z][y][x][spin][colour] complex128 <-> native 5-d field
int dwf_import(lqcd_ctx* c, int prec, int Ls, const double* canon, void* f5);
int dwf_export(lqcd_ctx* c, int prec, int Ls, const void* f5, double* canon);
// out = D in (dag 0) or D^dag in (dag 1); in != out; 1 <= Ls <= 256; tmp: a
// third 5-d field, needed (phi) by D with c5 != 0 only
int dwf_apply(lqcd_ctx* c, int prec, const lqcd_dwf_params& d, int dag, const void* in, void* out, void* tmp);
// D x = b (FP64 native 5-d fields, padding zero) by CG on D^dag D x = D^dag b
int dwf_solve(lqcd_ctx* c, const lqcd_dwf_params& d, const lqcd_solve_params& prm, const void* b, void* x,
              lqcd_solve_stats& st);

}  // namespace lq
