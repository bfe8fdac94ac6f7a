// Operator compositions on native half fields (ops.hip).
#pragma once

#include "internal.h"

namespace lq {

// clover slot of a precision (0: A_ee, 1: A_oo, 2: A_ee^-1, 3: A_oo^-1), null for Wilson (A = 1)
const void* clover_slot(lqcd_ctx* c, int prec, int slot);
// out = scale * H in, output parity out_parity
int op_hop(lqcd_ctx* c, int prec, int out_parity, const void* in, void* out, double scale);
// out = C own + scale * H in
int op_hop_xpay(lqcd_ctx* c, int prec, int out_parity, const void* in, const void* own, const void* clov, void* out,
                double scale);
// out = S in (even -> even) through tmp_odd; optional fused reduction (RED_DOT with w, or RED_TS)
int op_schur(lqcd_ctx* c, int prec, const void* in, void* out, void* tmp_odd, int red, const void* w,
             double* partials, const int* skip, int* nblocks);
// full D on a pair of half fields
int op_full(lqcd_ctx* c, int prec, const void* in_e, const void* in_o, void* out_e, void* out_o);
// one native operator (see lqcd_apply_native)
int op_native(lqcd_ctx* c, int op, int prec, const void* in, void* out, void* tmp_odd);

}  // namespace lq
