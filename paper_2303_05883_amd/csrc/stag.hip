// Staggered fermions: the hopping term with staggered phases on the
// checkerboarded, site-blocked layout, the even-odd normal system and CG
// (one of the fermion kinds the paper lists for Bridge++, Sec. 2):
//   D = m + H,  (H psi)(x) = 1/2 sum_mu eta_mu(x) [U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu)],
//   eta_x = 1, eta_y = (-1)^x, eta_z = (-1)^(x+y), eta_t = (-1)^(x+y+z),
// cross-boundary t hops times the fermion boundary factor; H is anti-Hermitian,
// so on the even sites m^2 - H_eo H_oe = m^2 + H_eo H_eo^dag is Hermitian
// positive definite and CG solves it (in FP64, or as FP32 inner solves under
// FP64 defect correction); x_o = (b_o - H_oe x_e) / m.
//
// Field layout: 3 complex per site in 64-site blocks, word k = colour k
// (FP64 double2, FP32 float2). The links are the context's 12-real links.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>

#include "fieldio.h"
#include "internal.h"
#include "stag.h"

namespace lq {
namespace {

constexpr int SBS = 256;

template <int P>
struct SIO;
template <>
struct SIO<0> {
  using T = double;
  __device__ static inline void load(const void* f, size_t i, cx<T> v[3]) {
    const double2* b = reinterpret_cast<const double2*>(f);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double2 w = b[widx(i, k, 3)];
      v[k] = {w.x, w.y};
    }
  }
  __device__ static inline void store(void* f, size_t i, const cx<T> v[3]) {
    double2* b = reinterpret_cast<double2*>(f);
#pragma unroll
    for (int k = 0; k < 3; ++k) b[widx(i, k, 3)] = make_double2(v[k].r, v[k].i);
  }
};
template <>
struct SIO<1> {
  using T = float;
  __device__ static inline void load(const void* f, size_t i, cx<T> v[3]) {
    const float2* b = reinterpret_cast<const float2*>(f);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float2 w = b[widx(i, k, 3)];
      v[k] = {w.x, w.y};
    }
  }
  __device__ static inline void store(void* f, size_t i, const cx<T> v[3]) {
    float2* b = reinterpret_cast<float2*>(f);
#pragma unroll
    for (int k = 0; k < 3; ++k) b[widx(i, k, 3)] = make_float2(v[k].r, v[k].i);
  }
};

struct StagArgs {
  Geom g;
  int p;               // output parity
  const char* gauge;   // links of this precision, 2 parities x 4 directions
  size_t link_stride;
  const void* in;      // parity 1 - p
  const void* own;     // parity p, or null
  void* out;
  double c_own, c_hop;  // out = c_own own + c_hop H in
  double* dot_partials;  // if set (with own): per-workgroup pairs (Re <own, out>, 0)
};

// out = c_own own + c_hop (H in) at site i of parity p; with dot_partials,
// Re <own, out> at the site into red[0]
template <int P>
__device__ inline void stag_hop_site(const StagArgs& a, size_t i, double red[2]) {
  using T = typename SIO<P>::T;
  const Geom& g = a.g;
  const int ii = (int)i;
  const int xh = ii % g.lxh;
  int r = ii / g.lxh;
  const int y = r % g.ly;
  r /= g.ly;
  const int z = r % g.lz;
  const int t = r / g.lz;
  const int x = 2 * xh + ((y + z + t + a.p) & 1);
  const int row = ii - xh;
  const int yl = g.lxh, zl = g.lxh * g.ly, tl = g.lxh * g.ly * g.lz;
  const int nf[4] = {row + (((x + 1 == g.lx) ? 0 : x + 1) >> 1), ii + ((y + 1 == g.ly) ? -(g.ly - 1) * yl : yl),
                     ii + ((z + 1 == g.lz) ? -(g.lz - 1) * zl : zl), ii + ((t + 1 == g.lt) ? -(g.lt - 1) * tl : tl)};
  const int nb[4] = {row + (((x == 0) ? g.lx - 1 : x - 1) >> 1), ii + ((y == 0) ? (g.ly - 1) * yl : -yl),
                     ii + ((z == 0) ? (g.lz - 1) * zl : -zl), ii + ((t == 0) ? (g.lt - 1) * tl : -tl)};
  const T eta[4] = {T(1), (x & 1) ? T(-1) : T(1), ((x + y) & 1) ? T(-1) : T(1), ((x + y + z) & 1) ? T(-1) : T(1)};
  const T sf = (g.t_bc < 0 && t + 1 == g.lt) ? T(-1) : T(1);
  const T sb = (g.t_bc < 0 && t == 0) ? T(-1) : T(1);
  const char* gf = a.gauge + (size_t)(a.p * 4) * a.link_stride;
  const char* gb = a.gauge + (size_t)((1 - a.p) * 4) * a.link_stride;
  cx<T> acc[3] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    cx<T> u[6], r2[3], v[3];
    // forward: + eta U_mu(x) psi(x + mu)
    IO<P>::template load_link<true>(gf + mu * a.link_stride, i, u);
    reconstruct(u, r2);
    SIO<P>::load(a.in, (size_t)nf[mu], v);
    const cx<T> M[9] = {u[0], u[1], u[2], u[3], u[4], u[5], r2[0], r2[1], r2[2]};
    const T ef = eta[mu] * (mu == 3 ? sf : T(1));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cx<T> s = M[3 * c] * v[0];
      s = s + M[3 * c + 1] * v[1];
      s = s + M[3 * c + 2] * v[2];
      acc[c] = acc[c] + ef * s;
    }
    // backward: - eta U_mu(x - mu)^dag psi(x - mu)
    IO<P>::template load_link<true>(gb + mu * a.link_stride, (size_t)nb[mu], u);
    reconstruct(u, r2);
    SIO<P>::load(a.in, (size_t)nb[mu], v);
    const cx<T> N[9] = {u[0], u[1], u[2], u[3], u[4], u[5], r2[0], r2[1], r2[2]};
    const T eb = -eta[mu] * (mu == 3 ? sb : T(1));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cx<T> s = cmulc(N[c], v[0]);
      s = s + cmulc(N[3 + c], v[1]);
      s = s + cmulc(N[6 + c], v[2]);
      acc[c] = acc[c] + eb * s;
    }
  }
  cx<T> out[3];
  const T ch = (T)(0.5 * a.c_hop);
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c] = ch * acc[c];
  if (a.own) {
    cx<T> o[3];
    SIO<P>::load(a.own, i, o);
    const T co = (T)a.c_own;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = out[c] + co * o[c];
    if (a.dot_partials) {
#pragma unroll
      for (int c = 0; c < 3; ++c) red[0] += (double)o[c].r * (double)out[c].r + (double)o[c].i * (double)out[c].i;
    }
  }
  SIO<P>::store(a.out, i, out);
}

template <int P>
__global__ void __launch_bounds__(SBS) k_stag_hop(StagArgs a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double red[2] = {0.0, 0.0};
  if (i < (size_t)a.g.vh) stag_hop_site<P>(a, i, red);
  if (a.dot_partials) block_reduce<2>(red, a.dot_partials + (size_t)blockIdx.x * 2);  // uniform over the launch
}

// canonical full-lattice [t, z, y, x, colour] complex128 <-> native half of one parity
template <int P>
__global__ void __launch_bounds__(SBS) k_stag_import(Geom g, int p, const double* canon, void* half) {
  using T = typename SIO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)g.vh) return;
  const int ii = (int)i, xh = ii % g.lxh;
  int r = ii / g.lxh;
  const int y = r % g.ly;
  r /= g.ly;
  const int z = r % g.lz, t = r / g.lz;
  const int x = 2 * xh + ((y + z + t + p) & 1);
  const size_t s = (size_t)x + (size_t)g.lx * (y + (size_t)g.ly * (z + (size_t)g.lz * t));
  cx<T> v[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = {(T)canon[6 * s + 2 * k], (T)canon[6 * s + 2 * k + 1]};
  SIO<P>::store(half, i, v);
}

template <int P>
__global__ void __launch_bounds__(SBS) k_stag_export(Geom g, int p, const void* half, double* canon) {
  using T = typename SIO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)g.vh) return;
  const int ii = (int)i, xh = ii % g.lxh;
  int r = ii / g.lxh;
  const int y = r % g.ly;
  r /= g.ly;
  const int z = r % g.lz, t = r / g.lz;
  const int x = 2 * xh + ((y + z + t + p) & 1);
  const size_t s = (size_t)x + (size_t)g.lx * (y + (size_t)g.ly * (z + (size_t)g.lz * t));
  cx<T> v[3];
  SIO<P>::load(half, i, v);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    canon[6 * s + 2 * k] = (double)v[k].r;
    canon[6 * s + 2 * k + 1] = (double)v[k].i;
  }
}

// Fields of precision P: out = ca a + cb b (b may be null)
template <int P>
__global__ void __launch_bounds__(SBS) k_stag_axpby(void* out, const void* a, double ca, const void* b, double cb,
                                                    size_t vh) {
  using T = typename SIO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vh) return;
  cx<T> va[3], w[3];
  SIO<P>::load(a, i, va);
  const T fa = (T)ca, fb = (T)cb;
#pragma unroll
  for (int k = 0; k < 3; ++k) w[k] = fa * va[k];
  if (b) {
    SIO<P>::load(b, i, va);
#pragma unroll
    for (int k = 0; k < 3; ++k) w[k] = w[k] + fb * va[k];
  }
  SIO<P>::store(out, i, w);
}

// per-workgroup partial sums (FP64) of Re <a, b> and <b, b>
template <int P>
__global__ void __launch_bounds__(SBS) k_stag_dot(const void* a, const void* b, double* partials, size_t vh) {
  using T = typename SIO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (i < vh) {
    cx<T> x[3], y[3];
    SIO<P>::load(a, i, x);
    SIO<P>::load(b, i, y);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v[0] += (double)x[k].r * (double)y[k].r + (double)x[k].i * (double)y[k].i;
      v[1] += (double)y[k].r * (double)y[k].r + (double)y[k].i * (double)y[k].i;
    }
  }
  block_reduce<2>(v, partials + (size_t)blockIdx.x * 2);
}

// CG update in one pass: x += alpha p, r -= alpha q, per-workgroup pairs
// (0, |r|^2) of the updated r (FP64 sums)
template <int P>
__global__ void __launch_bounds__(SBS) k_stag_xr(void* x, const void* p, void* r, const void* q, double alpha,
                                                 double* partials, size_t vh) {
  using T = typename SIO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (i < vh) {
    const T al = (T)alpha, mal = (T)(-alpha);
    cx<T> a[3], b[3];
    SIO<P>::load(x, i, a);
    SIO<P>::load(p, i, b);
#pragma unroll
    for (int k = 0; k < 3; ++k) a[k] = a[k] + al * b[k];
    SIO<P>::store(x, i, a);
    SIO<P>::load(r, i, a);
    SIO<P>::load(q, i, b);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a[k] = a[k] + mal * b[k];
      v[1] += (double)a[k].r * (double)a[k].r + (double)a[k].i * (double)a[k].i;
    }
    SIO<P>::store(r, i, a);
  }
  block_reduce<2>(v, partials + (size_t)blockIdx.x * 2);
}

// FP64 field rounded to FP32, and x (FP64) += e (FP32)
__global__ void __launch_bounds__(SBS) k_stag_down(const void* in64, void* out32, size_t vh) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vh) return;
  cx<double> a[3];
  cx<float> b[3];
  SIO<0>::load(in64, i, a);
#pragma unroll
  for (int k = 0; k < 3; ++k) b[k] = {(float)a[k].r, (float)a[k].i};
  SIO<1>::store(out32, i, b);
}

__global__ void __launch_bounds__(SBS) k_stag_accum_up(void* x64, const void* e32, size_t vh) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vh) return;
  cx<double> a[3];
  cx<float> b[3];
  SIO<0>::load(x64, i, a);
  SIO<1>::load(e32, i, b);
#pragma unroll
  for (int k = 0; k < 3; ++k) a[k] = a[k] + cx<double>{(double)b[k].r, (double)b[k].i};
  SIO<0>::store(x64, i, a);
}

int grid_for_sites(size_t n) { return (int)((n + SBS - 1) / SBS); }

}  // namespace

size_t stag_field_bytes(int prec, size_t vh) { return (size_t)(prec == 0 ? 48 : 24) * padded_sites(vh); }

int stag_import(lqcd_ctx* c, int prec, int parity, const double* canon, void* half) {
  const int nb = grid_for_sites(c->g.vh);
  if (prec == 0) hipLaunchKernelGGL(k_stag_import<0>, dim3(nb), dim3(SBS), 0, c->stream, c->g, parity, canon, half);
  else hipLaunchKernelGGL(k_stag_import<1>, dim3(nb), dim3(SBS), 0, c->stream, c->g, parity, canon, half);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int stag_export(lqcd_ctx* c, int prec, int parity, const void* half, double* canon) {
  const int nb = grid_for_sites(c->g.vh);
  if (prec == 0) hipLaunchKernelGGL(k_stag_export<0>, dim3(nb), dim3(SBS), 0, c->stream, c->g, parity, half, canon);
  else hipLaunchKernelGGL(k_stag_export<1>, dim3(nb), dim3(SBS), 0, c->stream, c->g, parity, half, canon);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int stag_hop(lqcd_ctx* c, int prec, int out_parity, const void* in, const void* own, double c_own, double c_hop,
             void* out, double* dot_partials) {
  if (dot_partials && !own) return set_error(LQCD_EINVAL, "staggered hop: a dot product with no own field");
  StagArgs a;
  a.g = c->g;
  a.p = out_parity;
  a.gauge = reinterpret_cast<const char*>(c->gauge[prec]);
  a.link_stride = link_bytes(prec, c->g.vh);
  a.in = in;
  a.own = own;
  a.out = out;
  a.c_own = c_own;
  a.c_hop = c_hop;
  a.dot_partials = dot_partials;
  const int nb = grid_for_sites(c->g.vh);
  if (prec == 0) hipLaunchKernelGGL(k_stag_hop<0>, dim3(nb), dim3(SBS), 0, c->stream, a);
  else hipLaunchKernelGGL(k_stag_hop<1>, dim3(nb), dim3(SBS), 0, c->stream, a);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

namespace {

struct SWork {
  std::vector<void*> mem;
  double* partials = nullptr;
  std::vector<double> host;
  ~SWork() {
    for (void* p : mem) (void)hipFree(p);
    if (partials) (void)hipFree(partials);
  }
  int alloc(size_t bytes, void** p) {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(LQCD_ENOMEM, "staggered solver workspace allocation failed");
    }
    mem.push_back(*p);
    return LQCD_OK;
  }
};

// The vector operations on half fields of precision prec (0 FP64, 1 FP32)
int axpby(lqcd_ctx* c, void* out, const void* a, double ca, const void* b = nullptr, double cb = 0.0, int prec = 0) {
  const dim3 grid(grid_for_sites(c->g.vh));
  const size_t vh = c->g.vh;
  if (prec == 0) hipLaunchKernelGGL(k_stag_axpby<0>, grid, dim3(SBS), 0, c->stream, out, a, ca, b, cb, vh);
  else hipLaunchKernelGGL(k_stag_axpby<1>, grid, dim3(SBS), 0, c->stream, out, a, ca, b, cb, vh);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

// the sums of the pairs of the last reduction (one pair per workgroup of a
// site-parallel launch), on the host in a fixed order
int sum_pairs(lqcd_ctx* c, SWork& w, double* ab, double* bb) {
  const int nb = grid_for_sites(c->g.vh);
  w.host.resize((size_t)nb * 2);
  LQ_HIP(hipMemcpyAsync(w.host.data(), w.partials, w.host.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  double s0 = 0.0, s1 = 0.0;
  for (size_t k = 0; k < w.host.size(); k += 2) {
    s0 += w.host[k];
    s1 += w.host[k + 1];
  }
  if (ab) *ab = s0;
  if (bb) *bb = s1;
  return LQCD_OK;
}

// Re <a, b> and <b, b>
int dot(lqcd_ctx* c, SWork& w, const void* a, const void* b, double* ab, double* bb, int prec = 0) {
  const int nb = grid_for_sites(c->g.vh);
  const size_t vh = c->g.vh;
  if (prec == 0) hipLaunchKernelGGL(k_stag_dot<0>, dim3(nb), dim3(SBS), 0, c->stream, a, b, w.partials, vh);
  else hipLaunchKernelGGL(k_stag_dot<1>, dim3(nb), dim3(SBS), 0, c->stream, a, b, w.partials, vh);
  LQ_HIP(hipGetLastError());
  return sum_pairs(c, w, ab, bb);
}

// x += alpha p, r -= alpha q, *rr = |r|^2 after the update
int xr_update(lqcd_ctx* c, SWork& w, void* x, const void* p, void* r, const void* q, double alpha, double* rr,
              int prec = 0) {
  const int nb = grid_for_sites(c->g.vh);
  const size_t vh = c->g.vh;
  if (prec == 0) hipLaunchKernelGGL(k_stag_xr<0>, dim3(nb), dim3(SBS), 0, c->stream, x, p, r, q, alpha, w.partials, vh);
  else hipLaunchKernelGGL(k_stag_xr<1>, dim3(nb), dim3(SBS), 0, c->stream, x, p, r, q, alpha, w.partials, vh);
  LQ_HIP(hipGetLastError());
  return sum_pairs(c, w, nullptr, rr);
}

int down(lqcd_ctx* c, const void* in64, void* out32) {
  hipLaunchKernelGGL(k_stag_down, dim3(grid_for_sites(c->g.vh)), dim3(SBS), 0, c->stream, in64, out32,
                     (size_t)c->g.vh);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int accum_up(lqcd_ctx* c, void* x64, const void* e32) {
  hipLaunchKernelGGL(k_stag_accum_up, dim3(grid_for_sites(c->g.vh)), dim3(SBS), 0, c->stream, x64, e32,
                     (size_t)c->g.vh);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

}  // namespace

int stag_schur(lqcd_ctx* c, int prec, double mass, const void* x_e, void* tmp_o, void* out_e, double* dot_partials) {
  LQ_TRY(stag_hop(c, prec, 1, x_e, nullptr, 0.0, 1.0, tmp_o));                     // H_oe x
  return stag_hop(c, prec, 0, tmp_o, x_e, mass * mass, -1.0, out_e, dot_partials);  // m^2 x - H_eo H_oe x
}

int stag_solve(lqcd_ctx* c, double mass, const lqcd_solve_params& prm, const void* b_e, const void* b_o, void* x_e,
               void* x_o, lqcd_solve_stats& st) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  SWork w;
  const size_t bytes = stag_field_bytes(0, c->g.vh);
  void *be2, *r, *p, *q, *t;
  for (void** f : {&be2, &r, &p, &q, &t}) LQ_TRY(w.alloc(bytes, f));
  // mixed precision: the inner CG in FP32 on its own fields
  const bool mixed = prm.inner_prec == LQCD_F32;
  const double delta = prm.inner_tol > 0.0 && prm.inner_tol < 1.0 ? prm.inner_tol : 1e-6;
  void *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *t32 = nullptr, *e32 = nullptr;
  if (mixed)
    for (void** f : {&r32, &p32, &q32, &t32, &e32}) LQ_TRY(w.alloc(stag_field_bytes(1, c->g.vh), f));
  LQ_HIP(hipMalloc(&w.partials, (size_t)grid_for_sites(c->g.vh) * 2 * sizeof(double)));
  // full-lattice |b|
  double bb_e = 0.0, bb_o = 0.0;
  LQ_TRY(dot(c, w, b_e, b_e, nullptr, &bb_e));
  LQ_TRY(dot(c, w, b_o, b_o, nullptr, &bb_o));
  const double bnorm = std::sqrt(bb_e + bb_o);
  st = lqcd_solve_stats{};
  const auto t1 = clk::now();
  st.seconds_setup = std::chrono::duration<double>(t1 - t0).count();
  if (bnorm == 0.0) {
    LQ_TRY(axpby(c, x_e, b_e, 0.0));
    LQ_TRY(axpby(c, x_o, b_o, 0.0));
    return LQCD_OK;
  }
  // even-odd source b' = m b_e - H_eo b_o
  LQ_TRY(stag_hop(c, 0, 0, b_o, b_e, mass, -1.0, be2));
  double bb2 = 0.0;
  LQ_TRY(dot(c, w, be2, be2, nullptr, &bb2));
  LQ_TRY(axpby(c, x_e, be2, 0.0));
  // CG on the normal system, to a residual that leaves room for the reconstruction
  const double target = 0.1 * prm.tol * bnorm * mass;
  int iters = 0, restarts = 0, status = LQCD_OK;
  double rr = 0.0, true_rel = 0.0;
  for (;;) {
    LQ_TRY(stag_schur(c, 0, mass, x_e, t, q));
    LQ_TRY(axpby(c, r, be2, 1.0, q, -1.0));
    LQ_TRY(dot(c, w, r, r, nullptr, &rr));
    // reconstruction and the true residual of D x = b
    LQ_TRY(stag_hop(c, 0, 1, x_e, b_o, 1.0 / mass, -1.0 / mass, x_o));  // x_o = (b_o - H_oe x_e) / m
    LQ_TRY(stag_hop(c, 0, 0, x_o, x_e, mass, 1.0, q));                  // (D x)_e
    LQ_TRY(axpby(c, q, q, 1.0, b_e, -1.0));
    double re = 0.0, ro = 0.0;
    LQ_TRY(dot(c, w, q, q, nullptr, &re));
    LQ_TRY(stag_hop(c, 0, 1, x_e, x_o, mass, 1.0, q));                  // (D x)_o
    LQ_TRY(axpby(c, q, q, 1.0, b_o, -1.0));
    LQ_TRY(dot(c, w, q, q, nullptr, &ro));
    true_rel = std::sqrt(re + ro) / bnorm;
    if (log_level() >= 1)
      std::fprintf(stderr, "[lqcd] staggered CG pass %d: %d iterations, |b - D x|/|b| %.3e\n", restarts, iters,
                   true_rel);
    if (true_rel <= prm.tol) break;
    if (!(true_rel == true_rel)) {
      status = set_error(LQCD_EBREAKDOWN, "staggered CG produced NaN");
      break;
    }
    if (iters >= prm.max_iter || restarts >= prm.max_outer) {
      status = set_error(LQCD_ENOCONV, "staggered CG did not reach the tolerance");
      break;
    }
    ++restarts;
    if (mixed) {
      // defect correction: (m^2 - H_eo H_oe) e = r by CG in FP32 from e = 0
      // until the iterated residual has dropped by delta (or reached the
      // target), then x_e += e in FP64 and the next pass starts from the true
      // residual
      LQ_TRY(down(c, r, r32));
      LQ_TRY(axpby(c, e32, r32, 0.0, nullptr, 0.0, 1));
      LQ_TRY(axpby(c, p32, r32, 1.0, nullptr, 0.0, 1));
      double rr32 = 0.0;
      LQ_TRY(dot(c, w, r32, r32, nullptr, &rr32, 1));
      const double tgt32 = std::max(delta * std::sqrt(rr32), target);
      while (iters < prm.max_iter) {
        LQ_TRY(stag_schur(c, 1, mass, p32, t32, q32, w.partials));
        double pq = 0.0;
        LQ_TRY(sum_pairs(c, w, &pq, nullptr));
        if (!(pq > 0.0)) break;
        const double alpha = rr32 / pq;
        double rn = 0.0;
        LQ_TRY(xr_update(c, w, e32, p32, r32, q32, alpha, &rn, 1));
        ++iters;
        if (std::sqrt(rn) <= tgt32) break;
        LQ_TRY(axpby(c, p32, r32, 1.0, p32, rn / rr32, 1));
        rr32 = rn;
      }
      LQ_TRY(accum_up(c, x_e, e32));
      continue;
    }
    LQ_TRY(axpby(c, p, r, 1.0));
    const double tgt = std::min(target, 0.5 * std::sqrt(rr));
    while (iters < prm.max_iter) {
      LQ_TRY(stag_schur(c, 0, mass, p, t, q, w.partials));  // q = (m^2 - H_eo H_oe) p, with Re <p, q>
      double pq = 0.0;
      LQ_TRY(sum_pairs(c, w, &pq, nullptr));
      if (!(pq > 0.0)) break;
      const double alpha = rr / pq;
      double rr_new = 0.0;
      LQ_TRY(xr_update(c, w, x_e, p, r, q, alpha, &rr_new));
      ++iters;
      if (std::sqrt(rr_new) <= tgt) {
        rr = rr_new;
        break;
      }
      LQ_TRY(axpby(c, p, r, 1.0, p, rr_new / rr));
      rr = rr_new;
    }
  }
  st.outer_iters = restarts;
  st.inner_iters = iters;
  st.restarts = restarts > 0 ? restarts - 1 : 0;
  st.true_rel_resid = true_rel;
  st.seconds_solve = std::chrono::duration<double>(clk::now() - t1).count();
  return status;
}

}  // namespace lq
