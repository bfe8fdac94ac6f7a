// Solver scalars kept in device memory and the launchers of the fused vector
// kernels (blas.hip).
#pragma once

#include "internal.h"

namespace lq {

// One BiCGStab's scalars, resident on the device. Complex values are (re, im).
struct Scal {
  double rho_r, rho_i;
  double alpha_r, alpha_i;
  double omega_r, omega_i;
  double beta_r, beta_i;
  double rr;        // ||r||^2 of the iterated residual
  double target2;   // stop when rr <= target2
  int done;         // set when converged, broken down or out of iterations
  int breakdown;
  int iters;        // iterations since the last (re)start
  int max_iters;
  double pad[2];
};

int blas_blocks(size_t vh);
int blas_p_update(lqcd_ctx* c, int prec, const void* r, void* p, const void* v, const Scal* sc);
int blas_s_update(lqcd_ctx* c, int prec, const void* r, const void* v, void* s, const Scal* sc);
int blas_xr_update(lqcd_ctx* c, int prec, int xprec, void* x, const void* p, const void* s, const void* t, void* r,
                   const void* rhat, const Scal* sc, double* partials);
int blas_dot_norm(lqcd_ctx* c, int prec, const void* a, const void* b, double* partials);
int blas_sub_norm(lqcd_ctx* c, const void* a, const void* b, void* out, double* partials);
int blas_scale_down(lqcd_ctx* c, int dprec, const void* src, void* dst, const double* dscale, double hscale);
int blas_accum_up(lqcd_ctx* c, int sprec, void* x, const void* e, const double* dscale);
int blas_copy(lqcd_ctx* c, int prec, const void* src, void* dst);
int blas_zero(lqcd_ctx* c, int prec, void* dst);

int blas_scale2(lqcd_ctx* c, int prec, void* p, void* v, double f);
int fin_reliable(lqcd_ctx* c, Scal* sc, const double* partials, int n, double target2);
int fin_alpha(lqcd_ctx* c, Scal* sc, const double* partials, int n);
int fin_omega(lqcd_ctx* c, Scal* sc, const double* partials, int n);
int fin_rho(lqcd_ctx* c, Scal* sc, const double* partials, int n);
int fin_init(lqcd_ctx* c, Scal* sc, const double* partials, int n, double target2, int max_iters);
// out[0] = sum, out[1] = 1/sqrt(sum), out[2] = sqrt(sum)
int fin_norm(lqcd_ctx* c, double* out, const double* partials, int n, int width, int comp);

}  // namespace lq
