// SAP preconditioner and the SAP-preconditioned flexible BiCGStab (sap.hip).
#pragma once

#include <functional>

#include "internal.h"

namespace lq {

// Whether block extents b (x, y, z, t) tile the lattice with an even number of
// blocks per direction and 64, 128, 192 or 256 sites per block.
bool sap_shape_ok(const Geom& g, const int b[4]);
// psi = M eta on FP32 native half fields: ncy cycles over the two block
// colours, nmr minimal-residual iterations per block solve, from psi = 0.
// Uses the context's two FP32 SAP fields (block residuals and updates,
// allocated on first use); calls on one context must not overlap.
int sap_apply(lqcd_ctx* c, const int b[4], int ncy, int nmr, const void* eta_e, const void* eta_o, void* psi_e,
              void* psi_o);
// A right preconditioner for solve_flexible: FP64 native halves in and out.
using FlexPrecond = std::function<int(const void* in_e, const void* in_o, void* out_e, void* out_o)>;
// D x = b on the full lattice with FP64 flexible BiCGStab, pre on the right
// (an empty pre: plain BiCGStab on D); x starts at zero if zero_x; stops on the
// true residual.
int solve_flexible(lqcd_ctx* c, const lqcd_solve_params& prm, const FlexPrecond& pre, const char* name,
                   const void* b_e, const void* b_o, void* x_e, void* x_o, bool zero_x, lqcd_solve_stats& st);
// D x = b with FP64 flexible BiCGStab, SAP on the right; x starts at zero if zero_x.
int solve_sap(lqcd_ctx* c, const lqcd_solve_params& prm, const int b[4], int ncy, int nmr, const void* b_e,
              const void* b_o, void* x_e, void* x_o, bool zero_x, lqcd_solve_stats& st);

}  // namespace lq
