// Operator compositions on native half fields (Eq. (1) of the paper):
//   D_pq = -kappa P_p H P_q (one hop), D_pp = A_pp (site term),
//   S = D_ee - D_eo D_oo^-1 D_oe = A_ee - kappa^2 H_eo A_oo^-1 H_oe (two hops),
//   D^(eo) = D_ee^-1 S, and the full D on a pair of half fields.
// The site terms are fused into the hops' epilogues.
#include "blas.h"
#include "internal.h"
#include "ops.h"

namespace lq {

const void* clover_slot(lqcd_ctx* c, int prec, int slot) {
  if (c->is_wilson) return nullptr;
  return c->clov[prec][slot];
}

int op_hop(lqcd_ctx* c, int prec, int out_parity, const void* in, void* out, double scale) {
  HopCall h{};
  h.prec = prec;
  h.out_parity = out_parity;
  h.in = in;
  h.out = out;
  h.epi = EPI_SCALE;
  h.scale = scale;
  h.red = RED_NONE;
  return launch_hop(c, h, nullptr);
}

int op_hop_xpay(lqcd_ctx* c, int prec, int out_parity, const void* in, const void* own, const void* clov, void* out,
                double scale) {
  HopCall h{};
  h.prec = prec;
  h.out_parity = out_parity;
  h.in = in;
  h.out = out;
  h.epi = EPI_XPAY;
  h.scale = scale;
  h.clov = clov;
  h.xown = own;
  h.red = RED_NONE;
  return launch_hop(c, h, nullptr);
}

int op_schur(lqcd_ctx* c, int prec, const void* in, void* out, void* tmp_odd, int red, const void* w,
             double* partials, const int* skip, int* nblocks) {
  const double k = c->kappa;
  HopCall h1{};
  h1.prec = prec;
  h1.out_parity = 1;
  h1.in = in;
  h1.out = tmp_odd;
  h1.epi = EPI_SCALE_CLOV;
  h1.scale = 1.0;
  h1.clov = clover_slot(c, prec, 3);  // A_oo^-1
  h1.red = RED_NONE;
  h1.skip = skip;
  LQ_TRY(launch_hop(c, h1, nullptr));
  HopCall h2{};
  h2.prec = prec;
  h2.out_parity = 0;
  h2.in = tmp_odd;
  h2.out = out;
  h2.epi = EPI_XPAY;
  h2.scale = -k * k;
  h2.clov = clover_slot(c, prec, 0);  // A_ee
  h2.xown = in;
  h2.red = red;
  h2.w = w;
  h2.partials = partials;
  h2.skip = skip;
  return launch_hop(c, h2, nblocks);
}

int op_full(lqcd_ctx* c, int prec, const void* in_e, const void* in_o, void* out_e, void* out_o) {
  const double k = c->kappa;
  LQ_TRY(op_hop_xpay(c, prec, 0, in_o, in_e, clover_slot(c, prec, 0), out_e, -k));
  return op_hop_xpay(c, prec, 1, in_e, in_o, clover_slot(c, prec, 1), out_o, -k);
}

int op_native(lqcd_ctx* c, int op, int prec, const void* in, void* out, void* tmp_odd) {
  const double k = c->kappa;
  switch (op) {
    case LQCD_DEO: return op_hop(c, prec, 0, in, out, -k);
    case LQCD_DOE: return op_hop(c, prec, 1, in, out, -k);
    case LQCD_HOP_EO: return op_hop(c, prec, 0, in, out, 1.0);
    case LQCD_HOP_OE: return op_hop(c, prec, 1, in, out, 1.0);
    case LQCD_DEE: return launch_site(c, prec, clover_slot(c, prec, 0), in, out);
    case LQCD_DOO: return launch_site(c, prec, clover_slot(c, prec, 1), in, out);
    case LQCD_DEE_INV: return launch_site(c, prec, clover_slot(c, prec, 2), in, out);
    case LQCD_DOO_INV: return launch_site(c, prec, clover_slot(c, prec, 3), in, out);
    case LQCD_DPREC_SCHUR: return op_schur(c, prec, in, out, tmp_odd, RED_NONE, nullptr, nullptr, nullptr, nullptr);
    case LQCD_DPREC_PAPER:
      return set_error(LQCD_EINVAL, "DPREC_PAPER is available through lqcd_apply only");
  }
  return set_error(LQCD_EINVAL, "unknown operator");
}

}  // namespace lq
