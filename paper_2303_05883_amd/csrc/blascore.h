// Per-site bodies of the BiCGStab vector updates, shared by the single-field
// kernels (blas.hip) and the batched ones (batch.hip). Scalars come from the
// solve's device-resident Scal.
#pragma once

#include "blas.h"
#include "fieldio.h"

namespace lq {

template <typename T>
__device__ inline cx<T> ld_scalar(const double* re_im) {
  return {(T)re_im[0], (T)re_im[1]};
}

// p = r + beta (p - omega v)
template <int P>
__device__ inline void p_update_site(const void* r, void* p, const void* v, const Scal* sc, size_t i) {
  using T = typename IO<P>::T;
  const cx<T> beta = ld_scalar<T>(&sc->beta_r), omega = ld_scalar<T>(&sc->omega_r);
  cx<T> a[12], b[12], c[12];
  IO<P>::load_spinor(r, i, a);
  IO<P>::load_spinor(p, i, b);
  IO<P>::load_spinor(v, i, c);
#pragma unroll
  for (int k = 0; k < 12; ++k) b[k] = a[k] + beta * (b[k] - omega * c[k]);
  IO<P>::store_spinor(p, i, b);
}

// s = r - alpha v
template <int P>
__device__ inline void s_update_site(const void* r, const void* v, void* s, const Scal* sc, size_t i) {
  using T = typename IO<P>::T;
  const cx<T> alpha = ld_scalar<T>(&sc->alpha_r);
  cx<T> a[12], c[12];
  IO<P>::load_spinor(r, i, a);
  IO<P>::load_spinor(v, i, c);
#pragma unroll
  for (int k = 0; k < 12; ++k) a[k] = a[k] - alpha * c[k];
  IO<P>::store_spinor(s, i, a);
}

// x += alpha p + omega s (x in precision PX); r = s - omega t; red += <rhat, r>, <r, r>
template <int P, int PX>
__device__ inline void xr_update_site(void* x, const void* p, const void* s, const void* t, void* r, const void* rhat,
                                      const Scal* sc, size_t i, double red[3]) {
  using T = typename IO<P>::T;
  using TX = typename IO<PX>::T;
  const cx<T> omega = ld_scalar<T>(&sc->omega_r);
  const cx<TX> alx = ld_scalar<TX>(&sc->alpha_r), omx = ld_scalar<TX>(&sc->omega_r);
  cx<T> pv[12], sv[12], tv[12];
  cx<TX> xv[12];
  IO<P>::load_spinor(p, i, pv);
  IO<P>::load_spinor(s, i, sv);
  IO<PX>::load_spinor(x, i, xv);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const cx<TX> pk = {(TX)pv[k].r, (TX)pv[k].i}, sk = {(TX)sv[k].r, (TX)sv[k].i};
    xv[k] = xv[k] + alx * pk + omx * sk;
  }
  IO<PX>::store_spinor(x, i, xv);
  IO<P>::load_spinor(t, i, tv);
#pragma unroll
  for (int k = 0; k < 12; ++k) sv[k] = sv[k] - omega * tv[k];
  IO<P>::store_spinor(r, i, sv);
  // FP16 codes round the stored value: reduce what was stored
  if (P == 2) IO<P>::load_spinor(r, i, sv);
  IO<P>::load_spinor(rhat, i, tv);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const cx<T> d = cmulc(tv[k], sv[k]);
    red[0] += (double)d.r;
    red[1] += (double)d.i;
    red[2] += (double)sv[k].r * (double)sv[k].r + (double)sv[k].i * (double)sv[k].i;
  }
}

// red += <a, b>, <b, b>
template <int P>
__device__ inline void dot_norm_site(const void* a, const void* b, size_t i, double red[3]) {
  using T = typename IO<P>::T;
  cx<T> av[12], bv[12];
  IO<P>::load_spinor(a, i, av);
  IO<P>::load_spinor(b, i, bv);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const cx<T> d = cmulc(av[k], bv[k]);
    red[0] += (double)d.r;
    red[1] += (double)d.i;
    red[2] += (double)bv[k].r * (double)bv[k].r + (double)bv[k].i * (double)bv[k].i;
  }
}

template <int P>
__device__ inline void copy_site(const void* src, void* dst, size_t i) {
  using T = typename IO<P>::T;
  cx<T> a[12];
  IO<P>::load_spinor(src, i, a);
  IO<P>::store_spinor(dst, i, a);
}

template <int P>
__device__ inline void zero_site(void* dst, size_t i) {
  using T = typename IO<P>::T;
  cx<T> a[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) a[k] = {T(0), T(0)};
  IO<P>::store_spinor(dst, i, a);
}

__device__ inline void cdiv(double ar, double ai, double br, double bi, double& cr, double& ci) {
  const double d = br * br + bi * bi;
  cr = (ar * br + ai * bi) / d;
  ci = (ai * br - ar * bi) / d;
}

// Sum n partial records of W doubles in a fixed order; every thread of the block
// receives the totals in out.
template <int W>
__device__ inline void sum_partials(const double* partials, int n, double out[W]) {
  // four independent partial sums per thread keep four loads in flight; the
  // order of additions is fixed by (n, blockDim), so the result is reproducible
  double v[4][W];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int k = 0; k < W; ++k) v[u][k] = 0.0;
  const int step = blockDim.x;
  int j = threadIdx.x;
  for (; j + 3 * step < n; j += 4 * step)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < W; ++k) v[u][k] += partials[(size_t)(j + u * step) * W + k];
  for (; j < n; j += step)
#pragma unroll
    for (int k = 0; k < W; ++k) v[0][k] += partials[(size_t)j * W + k];
#pragma unroll
  for (int k = 0; k < W; ++k) v[0][k] = (v[0][k] + v[1][k]) + (v[2][k] + v[3][k]);
  __shared__ double res[W];
  double tmp[W];
#pragma unroll
  for (int k = 0; k < W; ++k) tmp[k] = v[0][k];
  block_reduce<W>(tmp, res);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < W; ++k) out[k] = res[k];
  __syncthreads();
}

// The scalar updates of one BiCGStab (thread 0 of the block calls them).
__device__ inline void scal_alpha(Scal* sc, const double v[2]) {
  if (v[0] == 0.0 && v[1] == 0.0) {
    sc->breakdown = 1;
    sc->done = 1;
    return;
  }
  cdiv(sc->rho_r, sc->rho_i, v[0], v[1], sc->alpha_r, sc->alpha_i);
}

__device__ inline void scal_omega(Scal* sc, const double v[3]) {
  if (v[2] == 0.0) {
    sc->omega_r = 0.0;
    sc->omega_i = 0.0;
  } else {
    sc->omega_r = v[0] / v[2];
    sc->omega_i = v[1] / v[2];
  }
}

__device__ inline void scal_rho(Scal* sc, const double v[3]) {
  sc->iters += 1;
  sc->rr = v[2];
  if (v[2] <= sc->target2 || !(v[2] == v[2])) {
    sc->done = 1;
    if (!(v[2] == v[2])) sc->breakdown = 1;
    return;
  }
  if ((v[0] == 0.0 && v[1] == 0.0) || (sc->omega_r == 0.0 && sc->omega_i == 0.0)) {
    sc->breakdown = 1;
    sc->done = 1;
    return;
  }
  double qr, qi, ar, ai;
  cdiv(v[0], v[1], sc->rho_r, sc->rho_i, qr, qi);
  cdiv(sc->alpha_r, sc->alpha_i, sc->omega_r, sc->omega_i, ar, ai);
  sc->beta_r = qr * ar - qi * ai;
  sc->beta_i = qr * ai + qi * ar;
  sc->rho_r = v[0];
  sc->rho_i = v[1];
  if (sc->iters >= sc->max_iters) sc->done = 1;
}

__device__ inline void scal_init(Scal* sc, const double v[3], double target2, int max_iters) {
  sc->rho_r = v[0];
  sc->rho_i = v[1];
  sc->rr = v[2];
  sc->alpha_r = 1.0;
  sc->alpha_i = 0.0;
  sc->omega_r = 1.0;
  sc->omega_i = 0.0;
  sc->beta_r = 0.0;
  sc->beta_i = 0.0;
  sc->target2 = target2;
  sc->done = (v[2] <= target2) ? 1 : 0;
  sc->breakdown = 0;
  sc->max_iters = max_iters;
  sc->iters = 0;
}

// After a reliable update replaced r: rho = <rhat, r>, rr = <r, r>, new
// target; alpha, omega and the iteration count carry on.
__device__ inline void scal_reliable(Scal* sc, const double v[3], double target2) {
  sc->rho_r = v[0];
  sc->rho_i = v[1];
  sc->rr = v[2];
  sc->target2 = target2;
  sc->breakdown = 0;
  sc->done = (v[2] <= target2 || sc->iters >= sc->max_iters) ? 1 : 0;
}

}  // namespace lq
