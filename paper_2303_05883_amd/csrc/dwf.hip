// Domain-wall fermions (Shamir form; one of the operator kinds the paper
// lists and benchmarks for Bridge++, Sec. 2-3):
//   (D psi)_s = (5 - M5) psi_s - 1/2 H psi_s - P_- psi_{s+1} - P_+ psi_{s-1},
//   P_+- = (1 +- gamma5)/2, psi_{Ls} -> -m_f psi_0, psi_{-1} -> -m_f psi_{Ls-1},
// H the Wilson hopping term of hopcore.h. D^dag = (5 - M5) - 1/2 gamma5 H
// gamma5 - P_+ S_+ - P_- S_- (same walls). Solved by CG on the normal
// equations D^dag D x = D^dag b in FP64.
//
// A 5-d field is 2 Ls native half fields, slice s and parity p at index
// 2 s + p, back to back; as all have the same padded size, the whole 5-d field
// is also one valid site-blocked field of 2 Ls padded half volumes, which the
// vector kernels below use. The hop runs on 4 slices per thread so that each
// link load serves 4 slices (the hop_site_multi core of the batched solver).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>

#include "dwf.h"
#include "hopcore.h"
#include "internal.h"

namespace lq {
namespace {

constexpr int DBS = 128;
constexpr int NS = 4;  // slices per thread in the hop

template <int P>
__global__ void __launch_bounds__(DBS) k_dwf_hop(HopArgs a, const char* in5, char* out5, size_t hb, int Ls) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s0 = blockIdx.y * NS;
  MultiPtrs<NS> m;
  m.act = 0;
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int s = s0 + r < Ls ? s0 + r : Ls - 1;
    m.in[r] = in5 + (size_t)(2 * s + 1 - a.p) * hb;
    m.out[r] = out5 + (size_t)(2 * s + a.p) * hb;
    m.own[r] = nullptr;
    m.w[r] = nullptr;
    if (s0 + r < Ls) m.act |= 1u << r;
  }
  double red[NS][3];
  if (i < (size_t)a.g.vh) hop_site_multi<P, EPI_SCALE, false, RED_NONE, true, NS>(a, m, i, red);
}

// gamma5 of the Dirac-Pauli basis: (gamma5 v)_{0,1} = -v_{2,3}, (gamma5 v)_{2,3} = -v_{0,1}
template <typename T>
__device__ inline void g5(const cx<T> v[12], cx<T> o[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    o[k] = T(-1) * v[6 + k];
    o[6 + k] = T(-1) * v[k];
  }
}

// out_s = (5 - M5) in_s + hop_s (gamma5 hop_s if DAG) - P_a in_{s+1} - P_b in_{s-1}
// with (P_a, P_b) = (P_-, P_+) for D and (P_+, P_-) for D^dag; walls carry -m_f
template <int P, bool DAG>
__global__ void __launch_bounds__(DBS) k_dwf_s(const char* in5, const char* hop5, char* out5, size_t hb, int Ls,
                                               int vh, double diag, double mf) {
  using T = typename IO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)vh) return;
  const int s = blockIdx.y >> 1, p = blockIdx.y & 1;
  const int su = s + 1 < Ls ? s + 1 : 0, sd = s > 0 ? s - 1 : Ls - 1;
  const T wu = s + 1 < Ls ? T(1) : T(-mf), wd = s > 0 ? T(1) : T(-mf);
  cx<T> v[12], h[12], u[12], d[12], o[12];
  IO<P>::load_spinor(in5 + (size_t)(2 * s + p) * hb, i, v);
  IO<P>::load_spinor(hop5 + (size_t)(2 * s + p) * hb, i, h);
  IO<P>::load_spinor(in5 + (size_t)(2 * su + p) * hb, i, u);
  IO<P>::load_spinor(in5 + (size_t)(2 * sd + p) * hb, i, d);
  if (DAG) {
    cx<T> t[12];
    g5(h, t);
#pragma unroll
    for (int k = 0; k < 12; ++k) h[k] = t[k];
  }
  const T dg = (T)diag, half = T(0.5);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    // P_+ w: upper = (w_u - w_l)/2, lower = -upper; P_- w: upper = (w_u + w_l)/2, lower = upper
    const cx<T> up_p = half * (u[k] - u[6 + k]), up_m = half * (u[k] + u[6 + k]);
    const cx<T> dn_p = half * (d[k] - d[6 + k]), dn_m = half * (d[k] + d[6 + k]);
    // D: - P_- u - P_+ d;  D^dag: - P_+ u - P_- d
    const cx<T> a_up = DAG ? up_p : up_m, a_lo = DAG ? T(-1) * up_p : up_m;
    const cx<T> b_up = DAG ? dn_m : dn_p, b_lo = DAG ? dn_m : T(-1) * dn_p;
    o[k] = dg * v[k] + h[k] - wu * a_up - wd * b_up;
    o[6 + k] = dg * v[6 + k] + h[6 + k] - wu * a_lo - wd * b_lo;
  }
  IO<P>::store_spinor(out5 + (size_t)(2 * s + p) * hb, i, o);
}

// gamma5 on every site of a flat field of n sites
template <int P>
__global__ void __launch_bounds__(DBS) k_dwf_g5(const void* in, void* out, size_t n) {
  using T = typename IO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cx<T> v[12], o[12];
  IO<P>::load_spinor(in, i, v);
  g5(v, o);
  IO<P>::store_spinor(out, i, o);
}

// FP64 flat fields: out = a + cb b
__global__ void __launch_bounds__(256) k_flat_axpy(void* out, const void* a, const void* b, double cb, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cx<double> x[12], y[12];
  IO<0>::load_spinor(a, i, x);
  IO<0>::load_spinor(b, i, y);
#pragma unroll
  for (int k = 0; k < 12; ++k) x[k] = x[k] + cb * y[k];
  IO<0>::store_spinor(out, i, x);
}

// per-workgroup partial sums of Re <a, b> and <b, b>
__global__ void __launch_bounds__(256) k_flat_dot(const void* a, const void* b, double* partials, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (i < n) {
    cx<double> x[12], y[12];
    IO<0>::load_spinor(a, i, x);
    IO<0>::load_spinor(b, i, y);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      v[0] += x[k].r * y[k].r + x[k].i * y[k].i;
      v[1] += y[k].r * y[k].r + y[k].i * y[k].i;
    }
  }
  block_reduce<2>(v, partials + (size_t)blockIdx.x * 2);
}

}  // namespace

size_t dwf_field_bytes(int prec, size_t vh, int Ls) { return (size_t)2 * Ls * spinor_bytes(prec, vh); }

int dwf_import(lqcd_ctx* c, int prec, int Ls, const double* canon, void* f5) {
  const size_t hb = spinor_bytes(prec, c->g.vh), vol = (size_t)c->g.vh * 2;
  for (int s = 0; s < Ls; ++s)
    for (int p = 0; p < 2; ++p)
      LQ_TRY(launch_import_spinor(c, prec, p, canon + (size_t)s * vol * 24,
                                  reinterpret_cast<char*>(f5) + (size_t)(2 * s + p) * hb));
  return LQCD_OK;
}

int dwf_export(lqcd_ctx* c, int prec, int Ls, const void* f5, double* canon) {
  const size_t hb = spinor_bytes(prec, c->g.vh), vol = (size_t)c->g.vh * 2;
  for (int s = 0; s < Ls; ++s)
    for (int p = 0; p < 2; ++p)
      LQ_TRY(launch_export_spinor(c, prec, p, reinterpret_cast<const char*>(f5) + (size_t)(2 * s + p) * hb,
                                  canon + (size_t)s * vol * 24));
  return LQCD_OK;
}

// out = D in (dag = 0) or D^dag in (dag = 1) on native 5-d fields; tmp: one
// 5-d scratch field (two when dag: gamma5 in, then the hop)
int dwf_apply(lqcd_ctx* c, int prec, const lqcd_dwf_params& d, int dag, const void* in, void* out, void* tmp,
              void* tmp2) {
  if (!c->gauge[prec]) return set_error(LQCD_ESTATE, "gauge field not set");
  const size_t hb = spinor_bytes(prec, c->g.vh), n = (size_t)2 * d.Ls * padded_sites(c->g.vh);
  const char* src = reinterpret_cast<const char*>(in);
  const int nbx = (int)((c->g.vh + DBS - 1) / DBS);
  if (dag) {
    const int nb = (int)((n + DBS - 1) / DBS);
    if (prec == 0) hipLaunchKernelGGL(k_dwf_g5<0>, dim3(nb), dim3(DBS), 0, c->stream, in, tmp2, n);
    else if (prec == 1) hipLaunchKernelGGL(k_dwf_g5<1>, dim3(nb), dim3(DBS), 0, c->stream, in, tmp2, n);
    else return set_error(LQCD_EINVAL, "domain-wall operator: precision must be F64 or F32");
    src = reinterpret_cast<const char*>(tmp2);
  }
  HopArgs a{};
  a.gauge = reinterpret_cast<const char*>(c->gauge[prec]);
  a.link_stride = link_bytes(prec, c->g.vh);
  a.scale = -0.5;
  a.g = c->g;
  a.remap = 0;
  const dim3 gh(nbx, (d.Ls + NS - 1) / NS);
  for (int p = 0; p < 2; ++p) {
    a.p = p;
    if (prec == 0)
      hipLaunchKernelGGL(k_dwf_hop<0>, gh, dim3(DBS), 0, c->stream, a, src, reinterpret_cast<char*>(tmp), hb, d.Ls);
    else if (prec == 1)
      hipLaunchKernelGGL(k_dwf_hop<1>, gh, dim3(DBS), 0, c->stream, a, src, reinterpret_cast<char*>(tmp), hb, d.Ls);
    else return set_error(LQCD_EINVAL, "domain-wall operator: precision must be F64 or F32");
  }
  const dim3 gs(nbx, 2 * d.Ls);
  const double diag = 5.0 - d.M5;
  const char* i5 = reinterpret_cast<const char*>(in);
  const char* h5 = reinterpret_cast<const char*>(tmp);
  char* o5 = reinterpret_cast<char*>(out);
  if (prec == 0) {
    if (dag) hipLaunchKernelGGL((k_dwf_s<0, true>), gs, dim3(DBS), 0, c->stream, i5, h5, o5, hb, d.Ls, c->g.vh, diag, d.mf);
    else hipLaunchKernelGGL((k_dwf_s<0, false>), gs, dim3(DBS), 0, c->stream, i5, h5, o5, hb, d.Ls, c->g.vh, diag, d.mf);
  } else {
    if (dag) hipLaunchKernelGGL((k_dwf_s<1, true>), gs, dim3(DBS), 0, c->stream, i5, h5, o5, hb, d.Ls, c->g.vh, diag, d.mf);
    else hipLaunchKernelGGL((k_dwf_s<1, false>), gs, dim3(DBS), 0, c->stream, i5, h5, o5, hb, d.Ls, c->g.vh, diag, d.mf);
  }
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

namespace {

struct DWork {
  std::vector<void*> mem;
  double* partials = nullptr;
  std::vector<double> host;
  ~DWork() {
    for (void* p : mem) (void)hipFree(p);
    if (partials) (void)hipFree(partials);
  }
  int alloc(lqcd_ctx* c, size_t bytes, void** p) {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(LQCD_ENOMEM, "domain-wall solver workspace allocation failed");
    }
    mem.push_back(*p);
    // padding sites must read as zero in the flat vector kernels
    LQ_HIP(hipMemsetAsync(*p, 0, bytes, c->stream));
    return LQCD_OK;
  }
};

int axpy(lqcd_ctx* c, size_t n, void* out, const void* a, const void* b, double cb) {
  hipLaunchKernelGGL(k_flat_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, out, a, b, cb, n);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int dot(lqcd_ctx* c, DWork& w, size_t n, const void* a, const void* b, double* ab, double* bb) {
  const int nb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_flat_dot, dim3(nb), dim3(256), 0, c->stream, a, b, w.partials, n);
  LQ_HIP(hipGetLastError());
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

}  // namespace

int dwf_solve(lqcd_ctx* c, const lqcd_dwf_params& d, const lqcd_solve_params& prm, const void* b, void* x,
              lqcd_solve_stats& st) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  DWork w;
  const size_t bytes = dwf_field_bytes(0, c->g.vh, d.Ls), n = (size_t)2 * d.Ls * padded_sites(c->g.vh);
  void *bn, *r, *p, *q, *t, *t1, *t2;
  for (void** f : {&bn, &r, &p, &q, &t, &t1, &t2}) LQ_TRY(w.alloc(c, bytes, f));
  LQ_HIP(hipMalloc(&w.partials, (size_t)((n + 255) / 256) * 2 * sizeof(double)));
  double bb = 0.0;
  LQ_TRY(dot(c, w, n, b, b, nullptr, &bb));
  const double bnorm = std::sqrt(bb);
  st = lqcd_solve_stats{};
  const auto ts = clk::now();
  st.seconds_setup = std::chrono::duration<double>(ts - t0).count();
  LQ_HIP(hipMemsetAsync(x, 0, bytes, c->stream));  // x = 0 (padding included)
  if (bnorm == 0.0) return LQCD_OK;
  LQ_TRY(dwf_apply(c, 0, d, 1, b, bn, t1, t2));  // D^dag b
  double bnn = 0.0;
  LQ_TRY(dot(c, w, n, bn, bn, nullptr, &bnn));
  int iters = 0, passes = 0, status = LQCD_OK;
  double true_rel = 1.0, rr = 0.0;
  double target = 0.1 * prm.tol * std::sqrt(bnn);
  for (;;) {
    // true residual of D x = b, and the normal-equation residual
    LQ_TRY(dwf_apply(c, 0, d, 0, x, q, t1, t2));
    LQ_TRY(axpy(c, n, t, b, q, -1.0));
    double tt = 0.0;
    LQ_TRY(dot(c, w, n, t, t, nullptr, &tt));
    true_rel = std::sqrt(tt) / bnorm;
    if (log_level() >= 1)
      std::fprintf(stderr, "[lqcd] domain-wall CG pass %d: %d iterations, |b - D x|/|b| %.3e\n", passes, iters, true_rel);
    if (true_rel <= prm.tol) break;
    if (!(true_rel == true_rel)) {
      status = set_error(LQCD_EBREAKDOWN, "domain-wall CG produced NaN");
      break;
    }
    if (iters >= prm.max_iter || passes >= prm.max_outer) {
      status = set_error(LQCD_ENOCONV, "domain-wall CG did not reach the tolerance");
      break;
    }
    ++passes;
    LQ_TRY(dwf_apply(c, 0, d, 1, t, r, t1, t2));  // r = D^dag (b - D x)
    LQ_TRY(dot(c, w, n, r, r, nullptr, &rr));
    LQ_TRY(axpy(c, n, p, r, r, 0.0));             // p = r
    const double tgt = std::min(target, 0.5 * std::sqrt(rr));
    while (iters < prm.max_iter) {
      LQ_TRY(dwf_apply(c, 0, d, 0, p, t, t1, t2));
      LQ_TRY(dwf_apply(c, 0, d, 1, t, q, t1, t2));  // q = D^dag D p
      double pq = 0.0;
      LQ_TRY(dot(c, w, n, p, q, &pq, nullptr));
      if (!(pq > 0.0)) break;
      const double alpha = rr / pq;
      LQ_TRY(axpy(c, n, x, x, p, alpha));
      LQ_TRY(axpy(c, n, r, r, q, -alpha));
      double rn = 0.0;
      LQ_TRY(dot(c, w, n, r, r, nullptr, &rn));
      ++iters;
      if (std::sqrt(rn) <= tgt) {
        rr = rn;
        break;
      }
      LQ_TRY(axpy(c, n, p, r, p, rn / rr));
      rr = rn;
    }
    // the next pass iterates on the recomputed residual to a tighter normal target if needed
    target *= 0.5;
  }
  st.outer_iters = passes;
  st.inner_iters = iters;
  st.restarts = passes > 0 ? passes - 1 : 0;
  st.true_rel_resid = true_rel;
  st.seconds_solve = std::chrono::duration<double>(clk::now() - ts).count();
  return status;
}

}  // namespace lq
