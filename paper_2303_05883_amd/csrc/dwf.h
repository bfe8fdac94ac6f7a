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
// third 5-d field, needed (phi) by D with c5 != 0 only; norm_partials: if
// given, the launch's workgroups write their partial sums of |out|^2 as
// (0, value) pairs, dwf_apply_groups of them; upd (D with c5 != 0 only): in
// is first replaced in place by upd + upd_beta in (a CG direction update)
int dwf_apply(lqcd_ctx* c, int prec, const lqcd_dwf_params& d, int dag, const void* in, void* out, void* tmp,
              double* norm_partials = nullptr, const void* upd = nullptr, double upd_beta = 0.0);
size_t dwf_apply_groups(const Geom& g, int prec, int Ls);
// Even-odd form (4-d parity): out_e = S_ee in_e (dag 0) or S_ee^dag in_e (dag
// 1), S_ee = M5op - Dhop_eo M5op^-1 Dhop_oe; only the even halves of in and
// out are used; tA, tB: scratch 5-d fields
int dwf_schur_apply(lqcd_ctx* c, int prec, const lqcd_dwf_params& d, int dag, const void* in, void* out, void* tA,
                    void* tB);
// D x = b (FP64 native 5-d fields) through S_ee and CG on its normal
// equations (FP64, or FP32 inner CG under FP64 defect correction when
// prm.inner_prec is F32), x_o rebuilt, stopping on the true residual of D
int dwf_solve_eo(lqcd_ctx* c, const lqcd_dwf_params& d, const lqcd_solve_params& prm, const void* b, void* x,
                 lqcd_solve_stats& st);
// D x = b (FP64 native 5-d fields, padding zero) by CG on D^dag D x = D^dag b
int dwf_solve(lqcd_ctx* c, const lqcd_dwf_params& d, const lqcd_solve_params& prm, const void* b, void* x,
              lqcd_solve_stats& st);

}  // namespace lq
