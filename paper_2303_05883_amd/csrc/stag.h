// Staggered operator and its even-odd CG (stag.hip).
#pragma once

#include "internal.h"

namespace lq {

// Bytes of one native staggered half field (3 complex per site, 64-site blocks).
size_t stag_field_bytes(int prec, size_t vh);
// canonical full-lattice [t, z, y, x, colour] complex128 <-> native half of one parity
int stag_import(lqcd_ctx* c, int prec, int parity, const double* canon, void* half);
int stag_export(lqcd_ctx* c, int prec, int parity, const void* half, double* canon);
// out = c_own own + c_hop H in at the sites of out_parity (own may be null);
// dot_partials (needs own): the workgroups' pairs (Re <own, out>, 0), one per
// 256 sites
int stag_hop(lqcd_ctx* c, int prec, int out_parity, const void* in, const void* own, double c_own, double c_hop,
             void* out, double* dot_partials = nullptr);
// out_e = (m^2 - H_eo H_oe) x_e; tmp_o is scratch; dot_partials as stag_hop's,
// for Re <x_e, out_e>
int stag_schur(lqcd_ctx* c, int prec, double mass, const void* x_e, void* tmp_o, void* out_e,
               double* dot_partials = nullptr);
// D x = b (FP64 native halves) by CG on the even-odd normal system (FP64, or
// FP32 inner CG under FP64 defect correction when prm.inner_prec is F32)
int stag_solve(lqcd_ctx* c, double mass, const lqcd_solve_params& prm, const void* b_e, const void* b_o, void* x_e,
               void* x_o, lqcd_solve_stats& st);

}  // namespace lq
