// Fused vector kernels and deterministic reductions of the BiCGStab solver.
//
// Every update kernel reads the solver's scalars (alpha, beta, omega) from
// device memory, so an iteration needs no host round trip and can be replayed
// from a captured graph; every kernel first checks the solve's "done" flag and
// returns at once when it is set. Reductions are FP64: each block writes its
// partial sums in a fixed slot, and a one-block finalize kernel adds them in a
// fixed order, so repeated FP64 runs are bitwise identical. The finalize
// kernels also compute the next scalars (the solver's global reductions, of up
// to three values at once, the pattern the paper credits for solver
// efficiency in Sec. 3).
#include "blas.h"
#include "fieldio.h"

namespace lq {

namespace {

constexpr int BS = 256;
constexpr int FBS = 1024;  // threads of the one-block finalize kernels

__device__ inline bool is_done(const Scal* s) { return s && s->done; }

template <typename T>
__device__ inline cx<T> ld(const double* re_im) {
  return {(T)re_im[0], (T)re_im[1]};
}

// p = r + beta (p - omega v)
template <int P>
__global__ void __launch_bounds__(BS) k_p_update(const void* r, void* p, const void* v, const Scal* sc, size_t vh) {
  using T = typename IO<P>::T;
  if (is_done(sc)) return;
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x;
  if (i >= vh) return;
  const cx<T> beta = ld<T>(&sc->beta_r), omega = ld<T>(&sc->omega_r);
  cx<T> a[12], b[12], c[12];
  IO<P>::load_spinor(r, vh, i, a);
  IO<P>::load_spinor(p, vh, i, b);
  IO<P>::load_spinor(v, vh, i, c);
#pragma unroll
  for (int k = 0; k < 12; ++k) b[k] = a[k] + beta * (b[k] - omega * c[k]);
  IO<P>::store_spinor(p, vh, i, b);
}

// s = r - alpha v
template <int P>
__global__ void __launch_bounds__(BS) k_s_update(const void* r, const void* v, void* s, const Scal* sc, size_t vh) {
  using T = typename IO<P>::T;
  if (is_done(sc)) return;
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x;
  if (i >= vh) return;
  const cx<T> alpha = ld<T>(&sc->alpha_r);
  cx<T> a[12], c[12];
  IO<P>::load_spinor(r, vh, i, a);
  IO<P>::load_spinor(v, vh, i, c);
#pragma unroll
  for (int k = 0; k < 12; ++k) a[k] = a[k] - alpha * c[k];
  IO<P>::store_spinor(s, vh, i, a);
}

// x += alpha p + omega s (x in precision PX); r = s - omega t; partials <rhat, r>, <r, r>
template <int P, int PX>
__global__ void __launch_bounds__(BS) k_xr_update(void* x, const void* p, const void* s, const void* t, void* r,
                                                  const void* rhat, const Scal* sc, double* partials, size_t vh) {
  using T = typename IO<P>::T;
  using TX = typename IO<PX>::T;
  if (is_done(sc)) return;
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x;
  double red[3] = {0.0, 0.0, 0.0};
  if (i < vh) {
    const cx<T> alpha = ld<T>(&sc->alpha_r), omega = ld<T>(&sc->omega_r);
    const cx<TX> alx = ld<TX>(&sc->alpha_r), omx = ld<TX>(&sc->omega_r);
    cx<T> pv[12], sv[12], tv[12];
    cx<TX> xv[12];
    IO<P>::load_spinor(p, vh, i, pv);
    IO<P>::load_spinor(s, vh, i, sv);
    IO<PX>::load_spinor(x, vh, i, xv);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const cx<TX> pk = {(TX)pv[k].r, (TX)pv[k].i}, sk = {(TX)sv[k].r, (TX)sv[k].i};
      xv[k] = xv[k] + alx * pk + omx * sk;
    }
    IO<PX>::store_spinor(x, vh, i, xv);
    IO<P>::load_spinor(t, vh, i, tv);
#pragma unroll
    for (int k = 0; k < 12; ++k) sv[k] = sv[k] - omega * tv[k];
    IO<P>::store_spinor(r, vh, i, sv);
    // FP16 codes round the stored value: reduce what was stored
    if (P == 2) IO<P>::load_spinor(r, vh, i, sv);
    IO<P>::load_spinor(rhat, vh, i, tv);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const cx<T> d = cmulc(tv[k], sv[k]);
      red[0] += (double)d.r;
      red[1] += (double)d.i;
      red[2] += (double)sv[k].r * (double)sv[k].r + (double)sv[k].i * (double)sv[k].i;
    }
  }
  block_reduce<3>(red, partials + (size_t)blockIdx.x * 3);
}

// partials <a, b> (re, im) and <b, b>
template <int P>
__global__ void __launch_bounds__(BS) k_dot_norm(const void* a, const void* b, double* partials, size_t vh) {
  using T = typename IO<P>::T;
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x;
  double red[3] = {0.0, 0.0, 0.0};
  if (i < vh) {
    cx<T> av[12], bv[12];
    IO<P>::load_spinor(a, vh, i, av);
    IO<P>::load_spinor(b, vh, i, bv);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const cx<T> d = cmulc(av[k], bv[k]);
      red[0] += (double)d.r;
      red[1] += (double)d.i;
      red[2] += (double)bv[k].r * (double)bv[k].r + (double)bv[k].i * (double)bv[k].i;
    }
  }
  block_reduce<3>(red, partials + (size_t)blockIdx.x * 3);
}

// out = a - b (FP64), partial ||out||^2
__global__ void __launch_bounds__(BS) k_sub_norm(const void* a, const void* b, void* out, double* partials, size_t vh) {
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x;
  double red[1] = {0.0};
  if (i < vh) {
    cx<double> av[12], bv[12];
    IO<0>::load_spinor(a, vh, i, av);
    IO<0>::load_spinor(b, vh, i, bv);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      av[k] = av[k] - bv[k];
      red[0] += av[k].r * av[k].r + av[k].i * av[k].i;
    }
    IO<0>::store_spinor(out, vh, i, av);
  }
  block_reduce<1>(red, partials + blockIdx.x);
}

// dst (precision PD) = scale * src (FP64); scale read from device (1 / ||r||) or given
template <int PD>
__global__ void __launch_bounds__(BS) k_scale_down(const void* src, void* dst, const double* dscale, double hscale,
                                                   size_t vh) {
  using TD = typename IO<PD>::T;
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x;
  if (i >= vh) return;
  const double s = dscale ? *dscale : hscale;
  cx<double> a[12];
  cx<TD> d[12];
  IO<0>::load_spinor(src, vh, i, a);
#pragma unroll
  for (int k = 0; k < 12; ++k) d[k] = {(TD)(s * a[k].r), (TD)(s * a[k].i)};
  IO<PD>::store_spinor(dst, vh, i, d);
}

// x64 += scale * e (e in precision PS)
template <int PS>
__global__ void __launch_bounds__(BS) k_accum_up(void* x, const void* e, const double* dscale, size_t vh) {
  using TS = typename IO<PS>::T;
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x;
  if (i >= vh) return;
  const double s = *dscale;
  cx<double> a[12];
  cx<TS> b[12];
  IO<0>::load_spinor(x, vh, i, a);
  IO<PS>::load_spinor(e, vh, i, b);
#pragma unroll
  for (int k = 0; k < 12; ++k) a[k] = a[k] + s * cx<double>{(double)b[k].r, (double)b[k].i};
  IO<0>::store_spinor(x, vh, i, a);
}

template <int P>
__global__ void __launch_bounds__(BS) k_copy(const void* src, void* dst, size_t vh) {
  using T = typename IO<P>::T;
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x;
  if (i >= vh) return;
  cx<T> a[12];
  IO<P>::load_spinor(src, vh, i, a);
  IO<P>::store_spinor(dst, vh, i, a);
}

template <int P>
__global__ void __launch_bounds__(BS) k_zero(void* dst, size_t vh) {
  using T = typename IO<P>::T;
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x;
  if (i >= vh) return;
  cx<T> a[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) a[k] = {T(0), T(0)};
  IO<P>::store_spinor(dst, vh, i, a);
}

// Sum n partial records of `width` doubles in a fixed order into out[0..width).
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
}

__device__ inline void cdiv(double ar, double ai, double br, double bi, double& cr, double& ci) {
  const double d = br * br + bi * bi;
  cr = (ar * br + ai * bi) / d;
  ci = (ai * br - ar * bi) / d;
}

// alpha = rho / <rhat, v>
__global__ void __launch_bounds__(FBS) k_fin_alpha(Scal* sc, const double* partials, int n) {
  if (sc->done) return;
  double v[2];
  sum_partials<2>(partials, n, v);
  if (threadIdx.x == 0) {
    if (v[0] == 0.0 && v[1] == 0.0) {
      sc->breakdown = 1;
      sc->done = 1;
      return;
    }
    cdiv(sc->rho_r, sc->rho_i, v[0], v[1], sc->alpha_r, sc->alpha_i);
  }
}

// omega = <t, s> / <t, t>
__global__ void __launch_bounds__(FBS) k_fin_omega(Scal* sc, const double* partials, int n) {
  if (sc->done) return;
  double v[3];
  sum_partials<3>(partials, n, v);
  if (threadIdx.x == 0) {
    if (v[2] == 0.0) {
      sc->omega_r = 0.0;
      sc->omega_i = 0.0;
    } else {
      sc->omega_r = v[0] / v[2];
      sc->omega_i = v[1] / v[2];
    }
  }
}

// rho_new = <rhat, r>, rr = <r, r>; beta = (rho_new / rho)(alpha / omega); convergence test
__global__ void __launch_bounds__(FBS) k_fin_rho(Scal* sc, const double* partials, int n) {
  if (sc->done) return;
  double v[3];
  sum_partials<3>(partials, n, v);
  if (threadIdx.x == 0) {
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
}

// Start of a (re)start: rho = <rhat, r>, rr = <r, r>, alpha = omega = 1.
__global__ void __launch_bounds__(FBS) k_fin_init(Scal* sc, const double* partials, int n, double target2,
                                                 int max_iters) {
  double v[3];
  sum_partials<3>(partials, n, v);
  if (threadIdx.x == 0) {
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
}

// out[0] = sum of n partials (width 1 or 3, component `comp`); out[1] = 1/sqrt(out[0]) (0 if out[0] == 0)
__global__ void __launch_bounds__(FBS) k_fin_norm(double* out, const double* partials, int n, int width, int comp) {
  double v = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) v += partials[(size_t)j * width + comp];
  double tmp[1] = {v};
  __shared__ double res[1];
  block_reduce<1>(tmp, res);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = res[0];
    out[1] = res[0] > 0.0 ? 1.0 / sqrt(res[0]) : 0.0;
    out[2] = sqrt(res[0]);
  }
}

inline int nblk(size_t vh) { return (int)((vh + BS - 1) / BS); }

}  // namespace

int blas_blocks(size_t vh) { return nblk(vh); }

#define LQ_PREC_SWITCH(prec, CALL)                             \
  switch (prec) {                                              \
    case 0: { constexpr int P = 0; CALL; } break;              \
    case 1: { constexpr int P = 1; CALL; } break;              \
    case 2: { constexpr int P = 2; CALL; } break;              \
    default: return set_error(LQCD_EINVAL, "bad precision");   \
  }

int blas_p_update(lqcd_ctx* c, int prec, const void* r, void* p, const void* v, const Scal* sc) {
  const size_t vh = c->g.vh;
  LQ_PREC_SWITCH(prec, hipLaunchKernelGGL(k_p_update<P>, dim3(nblk(vh)), dim3(BS), 0, c->stream, r, p, v, sc, vh));
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int blas_s_update(lqcd_ctx* c, int prec, const void* r, const void* v, void* s, const Scal* sc) {
  const size_t vh = c->g.vh;
  LQ_PREC_SWITCH(prec, hipLaunchKernelGGL(k_s_update<P>, dim3(nblk(vh)), dim3(BS), 0, c->stream, r, v, s, sc, vh));
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int blas_xr_update(lqcd_ctx* c, int prec, int xprec, void* x, const void* p, const void* s, const void* t, void* r,
                   const void* rhat, const Scal* sc, double* partials) {
  const size_t vh = c->g.vh;
  const dim3 g(nblk(vh)), b(BS);
  if (prec == 0 && xprec == 0)
    hipLaunchKernelGGL((k_xr_update<0, 0>), g, b, 0, c->stream, x, p, s, t, r, rhat, sc, partials, vh);
  else if (prec == 1 && xprec == 1)
    hipLaunchKernelGGL((k_xr_update<1, 1>), g, b, 0, c->stream, x, p, s, t, r, rhat, sc, partials, vh);
  else if (prec == 2 && xprec == 1)
    hipLaunchKernelGGL((k_xr_update<2, 1>), g, b, 0, c->stream, x, p, s, t, r, rhat, sc, partials, vh);
  else if (prec == 2 && xprec == 2)
    hipLaunchKernelGGL((k_xr_update<2, 2>), g, b, 0, c->stream, x, p, s, t, r, rhat, sc, partials, vh);
  else
    return set_error(LQCD_EINVAL, "unsupported precision pair for x/r update");
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int blas_dot_norm(lqcd_ctx* c, int prec, const void* a, const void* b, double* partials) {
  const size_t vh = c->g.vh;
  LQ_PREC_SWITCH(prec, hipLaunchKernelGGL(k_dot_norm<P>, dim3(nblk(vh)), dim3(BS), 0, c->stream, a, b, partials, vh));
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int blas_sub_norm(lqcd_ctx* c, const void* a, const void* b, void* out, double* partials) {
  const size_t vh = c->g.vh;
  hipLaunchKernelGGL(k_sub_norm, dim3(nblk(vh)), dim3(BS), 0, c->stream, a, b, out, partials, vh);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int blas_scale_down(lqcd_ctx* c, int dprec, const void* src, void* dst, const double* dscale, double hscale) {
  const size_t vh = c->g.vh;
  LQ_PREC_SWITCH(dprec, hipLaunchKernelGGL(k_scale_down<P>, dim3(nblk(vh)), dim3(BS), 0, c->stream, src, dst, dscale,
                                           hscale, vh));
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int blas_accum_up(lqcd_ctx* c, int sprec, void* x, const void* e, const double* dscale) {
  const size_t vh = c->g.vh;
  LQ_PREC_SWITCH(sprec, hipLaunchKernelGGL(k_accum_up<P>, dim3(nblk(vh)), dim3(BS), 0, c->stream, x, e, dscale, vh));
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int blas_copy(lqcd_ctx* c, int prec, const void* src, void* dst) {
  const size_t vh = c->g.vh;
  LQ_PREC_SWITCH(prec, hipLaunchKernelGGL(k_copy<P>, dim3(nblk(vh)), dim3(BS), 0, c->stream, src, dst, vh));
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int blas_zero(lqcd_ctx* c, int prec, void* dst) {
  const size_t vh = c->g.vh;
  LQ_PREC_SWITCH(prec, hipLaunchKernelGGL(k_zero<P>, dim3(nblk(vh)), dim3(BS), 0, c->stream, dst, vh));
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int fin_alpha(lqcd_ctx* c, Scal* sc, const double* partials, int n) {
  hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(FBS), 0, c->stream, sc, partials, n);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}
int fin_omega(lqcd_ctx* c, Scal* sc, const double* partials, int n) {
  hipLaunchKernelGGL(k_fin_omega, dim3(1), dim3(FBS), 0, c->stream, sc, partials, n);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}
int fin_rho(lqcd_ctx* c, Scal* sc, const double* partials, int n) {
  hipLaunchKernelGGL(k_fin_rho, dim3(1), dim3(FBS), 0, c->stream, sc, partials, n);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}
int fin_init(lqcd_ctx* c, Scal* sc, const double* partials, int n, double target2, int max_iters) {
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(FBS), 0, c->stream, sc, partials, n, target2, max_iters);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}
int fin_norm(lqcd_ctx* c, double* out, const double* partials, int n, int width, int comp) {
  hipLaunchKernelGGL(k_fin_norm, dim3(1), dim3(FBS), 0, c->stream, out, partials, n, width, comp);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

}  // namespace lq
