// Schwarz alternating procedure (SAP) preconditioner and the flexible
// BiCGStab around it (the smoother / preconditioner of the paper's multigrid
// solver, Sec. 3: checkerboard-coloured blocks, the Dirac equation restricted
// to each block with the hops that leave it removed, a fixed number of
// minimal-residual block iterations, the two colours in turn; outer flexible
// BiCGStab).
//
// One workgroup per block of the colour being updated, one lane per block
// site. The lane forms the block right-hand side rho = eta - D psi at its
// site, then the block's minimal-residual iterations run on chip: the block
// residual and the block's internal forward links sit in LDS, q = D_B r takes
// its neighbours from LDS, the block dot products <q, r> and <q, q> are
// workgroup reductions, and psi += delta goes back to memory.
// The right-hand side is kept up to date instead of recomputed: after a
// colour's update its residual eta - D psi on its own sites is exactly the
// blocks' final MR residual r = rho - D_B delta (the neighbouring blocks are
// of the other colour, so no hop of the update lands on its own colour), and
// the other colour's update changes it only through the hops that cross the
// block faces, by +kappa H delta_other. So each launch stores r and delta, and
// the next launch of the colour starts from r plus those face hops (the
// first launch from eta alone, psi being zero) - no clover term and no
// interior hops from memory.
// The preconditioner works in FP32; the outer solve in FP64.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>

#include "blas.h"
#include "hopcore.h"
#include "internal.h"
#include "ops.h"
#include "sap.h"

namespace lq {
namespace {

struct SapArgs {
  Geom g;
  int b[4];        // block extents
  int nb[4];       // blocks per direction (even)
  int colour;
  int nmr;
  float kappa;
  const char* gauge;  // FP32 links, 2 parities x 4 directions
  size_t link_stride;
  const void* clov[2];  // FP32 A on even / odd sites, or null (Wilson: A = 1)
  const void* base[2];   // eta (first cycle) or the stored block residuals
  const void* dother[2]; // the other colour's last update delta, or null (first launch)
  void* res[2];          // this launch's final block residuals
  void* dout[2];         // this launch's delta
  void* psi[2];
};

// (1 -+ gamma_mu) U h-projection of a full spinor s for the hop in direction MU
template <int MU, bool FWD>
__device__ inline void project_any(const cx<float> s[12], cx<float> h[6]) {
  if (MU == 3) {  // (1 - gamma_t) s = 2 (0, 0, s2, s3); (1 + gamma_t) s = 2 (s0, s1, 0, 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) h[k] = 2.f * s[(FWD ? 6 : 0) + k];
  } else {
    project<MU, FWD>(s, h);
  }
}

// acc += f (1 -+ gamma_mu) U s for a neighbour spinor s and link u given
template <int MU, bool FWD>
__device__ inline void hop_given(const cx<float> s[12], const cx<float> u[6], float f, cx<float> acc[12]) {
  cx<float> h[6], w[6];
  project_any<MU, FWD>(s, h);
#pragma unroll
  for (int k = 0; k < 6; ++k) h[k] = f * h[k];
  link_mul<FWD>(u, h, w);
  expand<MU, FWD>(acc, w);
}

__device__ inline void lds_put12(float4* L, int n, int slot, const cx<float> s[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) L[k * n + slot] = make_float4(s[2 * k].r, s[2 * k].i, s[2 * k + 1].r, s[2 * k + 1].i);
}
__device__ inline void lds_get12(const float4* L, int n, int slot, cx<float> s[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float4 v = L[k * n + slot];
    s[2 * k] = {v.x, v.y};
    s[2 * k + 1] = {v.z, v.w};
  }
}
__device__ inline void lds_put6(float4* L, int n, int slot, const cx<float> u[6]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) L[k * n + slot] = make_float4(u[2 * k].r, u[2 * k].i, u[2 * k + 1].r, u[2 * k + 1].i);
}
__device__ inline void lds_get6(const float4* L, int n, int slot, cx<float> u[6]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float4 v = L[k * n + slot];
    u[2 * k] = {v.x, v.y};
    u[2 * k + 1] = {v.z, v.w};
  }
}

// Sum of NV doubles over the workgroup, returned to every lane (wave
// butterflies, then the wave sums added in wave order by every lane).
template <int NV>
__device__ inline void group_sum(double v[NV], double (*red)[NV]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    v[k] = x;
  }
  __syncthreads();  // the previous use of red is over
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wave][k] = v[k];
  __syncthreads();
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w][k];
    v[k] = s;
  }
}

__global__ void __launch_bounds__(256) k_sap_block(SapArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ double red[4][3];
  const int n = blockDim.x;  // block sites
  float4* Lr = reinterpret_cast<float4*>(lds_raw);  // residual, 6 words x n
  float4* Lu = Lr + 6 * n;                          // forward links, 4 directions x 3 words x n
  const Geom& g = a.g;
  // the blockIdx-th block of this colour: rows of nb[0] blocks alternate colours
  const int hx = a.nb[0] / 2;
  const int q = blockIdx.x % hx, row = blockIdx.x / hx;
  const int by = row % a.nb[1], bz = (row / a.nb[1]) % a.nb[2], bt = row / (a.nb[1] * a.nb[2]);
  const int bx = 2 * q + ((by + bz + bt + a.colour) & 1);
  // this lane's site
  const int l = threadIdx.x;
  const int lx = l % a.b[0], ly = (l / a.b[0]) % a.b[1], lz = (l / (a.b[0] * a.b[1])) % a.b[2],
            lt = l / (a.b[0] * a.b[1] * a.b[2]);
  const int x = bx * a.b[0] + lx, y = by * a.b[1] + ly, z = bz * a.b[2] + lz, t = bt * a.b[3] + lt;
  const int p = (x + y + z + t) & 1;
  const int lxh = g.lxh;
  auto hidx = [&](int xx, int yy, int zz, int tt) -> size_t {
    return (size_t)(xx >> 1) + (size_t)lxh * (yy + (size_t)g.ly * (zz + (size_t)g.lz * tt));
  };
  const size_t i = hidx(x, y, z, t);
  const char* gf = a.gauge + (size_t)(p * 4) * a.link_stride;        // U_mu(x), parity p
  const char* gb = a.gauge + (size_t)((1 - p) * 4) * a.link_stride;  // U_mu(x - mu), parity 1-p
  const size_t ls = a.link_stride;
  const int c[4] = {x, y, z, t}, L[4] = {g.lx, g.ly, g.lz, g.lt};
  const int lc[4] = {lx, ly, lz, lt};
  const int stride[4] = {1, a.b[0], a.b[0] * a.b[1], a.b[0] * a.b[1] * a.b[2]};

  // ---- rho = base + kappa (H delta_other) over the hops that cross the block
  // faces (neighbours from memory; the interior hops are in base)
  cx<float> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = {0.f, 0.f};
  if (a.dother[1 - p]) {
    const void* pin = a.dother[1 - p];
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      int f[4] = {c[0], c[1], c[2], c[3]}, bk[4] = {c[0], c[1], c[2], c[3]};
      f[mu] = c[mu] + 1 == L[mu] ? 0 : c[mu] + 1;
      bk[mu] = c[mu] == 0 ? L[mu] - 1 : c[mu] - 1;
      const size_t jf = hidx(f[0], f[1], f[2], f[3]), jb = hidx(bk[0], bk[1], bk[2], bk[3]);
      const bool ff = mu == 3 && g.t_bc < 0 && c[3] + 1 == L[3];
      const bool fb = mu == 3 && g.t_bc < 0 && c[3] == 0;
      const bool face_f = lc[mu] + 1 == a.b[mu], face_b = lc[mu] == 0;
      switch (mu) {
        case 0:
          if (face_f) hop_dir<1, 0, true, false>(pin, gf + 0 * ls, 0, jf, i, false, acc);
          if (face_b) hop_dir<1, 0, false, false>(pin, gb + 0 * ls, 0, jb, jb, false, acc);
          break;
        case 1:
          if (face_f) hop_dir<1, 1, true, false>(pin, gf + 1 * ls, 0, jf, i, false, acc);
          if (face_b) hop_dir<1, 1, false, false>(pin, gb + 1 * ls, 0, jb, jb, false, acc);
          break;
        case 2:
          if (face_f) hop_dir<1, 2, true, false>(pin, gf + 2 * ls, 0, jf, i, false, acc);
          if (face_b) hop_dir<1, 2, false, false>(pin, gb + 2 * ls, 0, jb, jb, false, acc);
          break;
        default:
          if (face_f) hop_dir<1, 3, true, false>(pin, gf + 3 * ls, 0, jf, i, ff, acc);
          if (face_b) hop_dir<1, 3, false, false>(pin, gb + 3 * ls, 0, jb, jb, fb, acc);
          break;
      }
    }
  }
  cx<float> r[12];
  IO<1>::load_spinor(a.base[p], i, r);
#pragma unroll
  for (int k = 0; k < 12; ++k) r[k] = r[k] + a.kappa * acc[k];

  // ---- the block's internal forward links into LDS
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    cx<float> u[6];
    IO<1>::template load_link<false>(gf + mu * ls, i, u);
    lds_put6(Lu + mu * 3 * n, n, l, u);
  }

  // ---- minimal-residual iterations on the block
  cx<float> delta[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) delta[k] = {0.f, 0.f};
  for (int it = 0; it < a.nmr; ++it) {
    __syncthreads();  // the previous residual has been read
    lds_put12(Lr, n, l, r);
    __syncthreads();
    // q = D_B r = A r - kappa sum of the hops that stay in the block
    cx<float> qv[12];
    if (a.clov[p]) clover_apply<1>(a.clov[p], i, r, qv);
    else
#pragma unroll
      for (int k = 0; k < 12; ++k) qv[k] = r[k];
    const float mk = -a.kappa;
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {  // not unrolled: one direction's LDS data live at a time
      cx<float> sp[12], u[6];
      if (lc[mu] + 1 < a.b[mu]) {
        lds_get12(Lr, n, l + stride[mu], sp);
        lds_get6(Lu + mu * 3 * n, n, l, u);
        switch (mu) {
          case 0: hop_given<0, true>(sp, u, mk, qv); break;
          case 1: hop_given<1, true>(sp, u, mk, qv); break;
          case 2: hop_given<2, true>(sp, u, mk, qv); break;
          default: hop_given<3, true>(sp, u, mk, qv); break;
        }
      }
      if (lc[mu] > 0) {
        lds_get12(Lr, n, l - stride[mu], sp);
        lds_get6(Lu + mu * 3 * n, n, l - stride[mu], u);
        switch (mu) {
          case 0: hop_given<0, false>(sp, u, mk, qv); break;
          case 1: hop_given<1, false>(sp, u, mk, qv); break;
          case 2: hop_given<2, false>(sp, u, mk, qv); break;
          default: hop_given<3, false>(sp, u, mk, qv); break;
        }
      }
    }
    double dv[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const cx<float> d = cmulc(qv[k], r[k]);
      dv[0] += (double)d.r;
      dv[1] += (double)d.i;
      dv[2] += (double)qv[k].r * qv[k].r + (double)qv[k].i * qv[k].i;
    }
    group_sum<3>(dv, red);
    const cx<float> alpha = dv[2] > 0.0 ? cx<float>{(float)(dv[0] / dv[2]), (float)(dv[1] / dv[2])}
                                        : cx<float>{0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      delta[k] = delta[k] + alpha * r[k];
      r[k] = r[k] - alpha * qv[k];
    }
  }
  // ---- psi += delta on this block; the residual and delta for the next launches
  IO<1>::store_spinor(a.res[p], i, r);
  IO<1>::store_spinor(a.dout[p], i, delta);
  cx<float> ps[12];
  IO<1>::load_spinor(a.psi[p], i, ps);
#pragma unroll
  for (int k = 0; k < 12; ++k) ps[k] = ps[k] + delta[k];
  IO<1>::store_spinor(a.psi[p], i, ps);
}

}  // namespace

bool sap_shape_ok(const Geom& g, const int b[4]) {
  const int L[4] = {g.lx, g.ly, g.lz, g.lt};
  int vol = 1;
  for (int d = 0; d < 4; ++d) {
    if (b[d] < 1 || L[d] % b[d] != 0 || (L[d] / b[d]) % 2 != 0) return false;
    vol *= b[d];
  }
  return vol >= 64 && vol <= 256 && vol % 64 == 0;
}

// psi = M eta on FP32 native half fields (eta, psi: even and odd halves).
int sap_apply(lqcd_ctx* c, const int b[4], int ncy, int nmr, const void* eta_e, const void* eta_o, void* psi_e,
              void* psi_o) {
  if (!sap_shape_ok(c->g, b)) return set_error(LQCD_EINVAL, "bad SAP block shape");
  if (ncy < 1 || nmr < 1) return set_error(LQCD_EINVAL, "SAP needs at least one cycle and one block iteration");
  SapArgs a{};
  a.g = c->g;
  const int L[4] = {c->g.lx, c->g.ly, c->g.lz, c->g.lt};
  int vol = 1, nblocks = 1;
  for (int d = 0; d < 4; ++d) {
    a.b[d] = b[d];
    a.nb[d] = L[d] / b[d];
    vol *= b[d];
    nblocks *= a.nb[d];
  }
  a.nmr = nmr;
  a.kappa = (float)c->kappa;
  a.gauge = reinterpret_cast<const char*>(c->gauge[1]);
  a.link_stride = link_bytes(1, c->g.vh);
  a.clov[0] = clover_slot(c, 1, 0);
  a.clov[1] = clover_slot(c, 1, 1);
  const size_t hb = spinor_bytes(1, c->g.vh);
  for (void** f : {&c->sap_res, &c->sap_delta})
    if (!*f && hipMalloc(f, 2 * hb) != hipSuccess) {
      *f = nullptr;
      (void)hipGetLastError();
      return set_error(LQCD_ENOMEM, "SAP workspace allocation failed");
    }
  char* res = static_cast<char*>(c->sap_res);
  char* del = static_cast<char*>(c->sap_delta);
  a.psi[0] = psi_e;
  a.psi[1] = psi_o;
  a.res[0] = res;
  a.res[1] = res + hb;
  a.dout[0] = del;
  a.dout[1] = del + hb;
  LQ_TRY(blas_zero(c, 1, psi_e));
  LQ_TRY(blas_zero(c, 1, psi_o));
  const size_t lds = (size_t)vol * (6 + 12) * 16;
  for (int cy = 0; cy < ncy; ++cy)
    for (int colour = 0; colour < 2; ++colour) {
      a.colour = colour;
      // right-hand side: eta on the first cycle, then this colour's stored
      // residual; plus the face hops of the other colour's last update (none
      // before the first update)
      a.base[0] = cy == 0 ? eta_e : res;
      a.base[1] = cy == 0 ? eta_o : res + hb;
      const bool none = cy == 0 && colour == 0;
      a.dother[0] = none ? nullptr : del;
      a.dother[1] = none ? nullptr : del + hb;
      hipLaunchKernelGGL(k_sap_block, dim3(nblocks / 2), dim3(vol), lds, c->stream, a);
    }
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

}  // namespace lq

// ------------------------------------------------------------------ flexible BiCGStab (FP64)
namespace lq {
namespace {

constexpr int LBS = 256;

// out = ca a + cb b + cc c on FP64 half fields (b, c may be null)
__global__ void __launch_bounds__(LBS) k_lin3(void* out, const void* a, cx<double> ca, const void* b, cx<double> cb,
                                              const void* cc_f, cx<double> cc, size_t vh) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vh) return;
  cx<double> va[12], w[12];
  IO<0>::load_spinor(a, i, va);
#pragma unroll
  for (int k = 0; k < 12; ++k) w[k] = ca * va[k];
  if (b) {
    IO<0>::load_spinor(b, i, va);
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = w[k] + cb * va[k];
  }
  if (cc_f) {
    IO<0>::load_spinor(cc_f, i, va);
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = w[k] + cc * va[k];
  }
  IO<0>::store_spinor(out, i, w);
}

// per-workgroup partial sums of <a, b> (re, im) and <b, b> on FP64 half fields
__global__ void __launch_bounds__(LBS) k_dot(const void* a, const void* b, double* partials, size_t vh) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (i < vh) {
    cx<double> x[12], y[12];
    IO<0>::load_spinor(a, i, x);
    IO<0>::load_spinor(b, i, y);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const cx<double> d = cmulc(x[k], y[k]);
      v[0] += d.r;
      v[1] += d.i;
      v[2] += y[k].r * y[k].r + y[k].i * y[k].i;
    }
  }
  block_reduce<3>(v, partials + (size_t)blockIdx.x * 3);
}

struct Pair {
  void* h[2] = {nullptr, nullptr};
};

struct FWork {
  std::vector<void*> mem;
  double* partials = nullptr;
  std::vector<double> host;
  ~FWork() {
    for (void* p : mem) (void)hipFree(p);
    if (partials) (void)hipFree(partials);
  }
  int alloc(size_t bytes, void** p) {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(LQCD_ENOMEM, "SAP solver workspace allocation failed");
    }
    mem.push_back(*p);
    return LQCD_OK;
  }
};

int grid_of(size_t n) { return (int)((n + LBS - 1) / LBS); }

int lin3(lqcd_ctx* c, Pair out, cx<double> ca, Pair a, cx<double> cb = {0, 0}, const Pair* b = nullptr,
         cx<double> cc = {0, 0}, const Pair* cf = nullptr) {
  const size_t vh = c->g.vh;
  for (int h = 0; h < 2; ++h)
    hipLaunchKernelGGL(k_lin3, dim3(grid_of(vh)), dim3(LBS), 0, c->stream, out.h[h], a.h[h], ca, b ? b->h[h] : nullptr,
                       cb, cf ? cf->h[h] : nullptr, cc, vh);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

// <a, b> and ||b||^2 over both halves, summed on the host in a fixed order
int dot(lqcd_ctx* c, FWork& w, Pair a, Pair b, cx<double>* ab, double* bb) {
  const size_t vh = c->g.vh;
  const int nb = grid_of(vh);
  for (int h = 0; h < 2; ++h)
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(LBS), 0, c->stream, a.h[h], b.h[h], w.partials + (size_t)h * nb * 3, vh);
  LQ_HIP(hipGetLastError());
  w.host.resize((size_t)2 * nb * 3);
  LQ_HIP(hipMemcpyAsync(w.host.data(), w.partials, w.host.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  double s[3] = {0.0, 0.0, 0.0};
  for (size_t k = 0; k < w.host.size(); k += 3)
    for (int j = 0; j < 3; ++j) s[j] += w.host[k + j];
  if (ab) *ab = {s[0], s[1]};
  if (bb) *bb = s[2];
  return LQCD_OK;
}

inline cx<double> cdivd(cx<double> a, cx<double> b) {
  const double d = b.r * b.r + b.i * b.i;
  return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

}  // namespace

// D x = b on the full lattice (FP64 native halves) by flexible BiCGStab with
// the preconditioner pre on the right (FP64 halves in, FP64 halves out; it may
// vary between calls); stops on the true residual. name labels the log lines.
int solve_flexible(lqcd_ctx* c, const lqcd_solve_params& prm, const FlexPrecond& pre, const char* name,
                   const void* b_e, const void* b_o, void* x_e, void* x_o, bool zero_x, lqcd_solve_stats& st) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  FWork w;
  const size_t b64 = spinor_bytes(0, c->g.vh);
  Pair r, rh, p, v, s, t, ph, sh, ax;
  for (Pair* q : {&r, &rh, &p, &v, &s, &t, &ax})
    for (auto& h : q->h) LQ_TRY(w.alloc(b64, &h));
  // without a preconditioner (plain BiCGStab) the preconditioned vectors are
  // the vectors themselves: p_hat aliases p and s_hat aliases s
  const bool ident = !pre;
  if (ident) {
    ph = p;
    sh = s;
  } else {
    for (Pair* q : {&ph, &sh})
      for (auto& h : q->h) LQ_TRY(w.alloc(b64, &h));
  }
  LQ_HIP(hipMalloc(&w.partials, (size_t)2 * grid_of(c->g.vh) * 3 * sizeof(double)));
  Pair b, x;
  b.h[0] = const_cast<void*>(b_e);
  b.h[1] = const_cast<void*>(b_o);
  x.h[0] = x_e;
  x.h[1] = x_o;
  if (zero_x) {
    LQ_TRY(blas_zero(c, 0, x_e));
    LQ_TRY(blas_zero(c, 0, x_o));
  }
  auto apply = [&](Pair in, Pair out) -> int { return op_full(c, 0, in.h[0], in.h[1], out.h[0], out.h[1]); };
  int napply = 0;
  auto precond = [&](Pair in, Pair out) -> int {
    if (ident) return LQCD_OK;
    LQ_TRY(pre(in.h[0], in.h[1], out.h[0], out.h[1]));
    ++napply;
    return LQCD_OK;
  };
  double bb = 0.0;
  LQ_TRY(dot(c, w, b, b, nullptr, &bb));
  const double bnorm = std::sqrt(bb);
  st = lqcd_solve_stats{};
  const auto t1 = clk::now();
  st.seconds_setup = std::chrono::duration<double>(t1 - t0).count();
  if (bnorm == 0.0) {
    LQ_TRY(blas_zero(c, 0, x_e));
    LQ_TRY(blas_zero(c, 0, x_o));
    st.true_rel_resid = 0.0;
    return LQCD_OK;
  }
  const double target = prm.tol * bnorm;
  int iters = 0, restarts = 0, status = LQCD_OK;
  double rnorm = 0.0;
  for (;;) {
    // true residual r = b - D x
    LQ_TRY(apply(x, ax));
    LQ_TRY(lin3(c, r, {1, 0}, b, {-1, 0}, &ax));
    double rr = 0.0;
    LQ_TRY(dot(c, w, r, r, nullptr, &rr));
    rnorm = std::sqrt(rr);
    if (log_level() >= 1)
      std::fprintf(stderr, "[lqcd] %s-FBiCGStab restart %d: %d iterations, |r|/|b| %.3e\n", name, restarts, iters,
                   rnorm / bnorm);
    if (rnorm <= target) break;
    if (!(rnorm == rnorm)) {
      status = set_error(LQCD_EBREAKDOWN, "preconditioned flexible BiCGStab produced NaN");
      break;
    }
    if (iters >= prm.max_iter || restarts > prm.max_outer) {
      status = set_error(LQCD_ENOCONV, "preconditioned flexible BiCGStab did not reach the tolerance");
      break;
    }
    LQ_TRY(lin3(c, rh, {1, 0}, r));
    cx<double> rho_old{1, 0}, alpha{1, 0}, omega{1, 0};
    LQ_TRY(blas_zero(c, 0, v.h[0]));
    LQ_TRY(blas_zero(c, 0, v.h[1]));
    LQ_TRY(blas_zero(c, 0, p.h[0]));
    LQ_TRY(blas_zero(c, 0, p.h[1]));
    // rho = <rhat, r>; later iterations take it from the residual-norm pass
    cx<double> rho;
    LQ_TRY(dot(c, w, rh, r, &rho, nullptr));
    while (iters < prm.max_iter) {
      if (rho.r == 0.0 && rho.i == 0.0) break;
      const cx<double> beta = cdivd(rho, rho_old) * cdivd(alpha, omega);
      // p = r + beta (p - omega v)
      LQ_TRY(lin3(c, p, {1, 0}, r, beta, &p, {-(beta * omega).r, -(beta * omega).i}, &v));
      LQ_TRY(precond(p, ph));
      LQ_TRY(apply(ph, v));
      cx<double> rv;
      LQ_TRY(dot(c, w, rh, v, &rv, nullptr));
      if (rv.r == 0.0 && rv.i == 0.0) break;
      alpha = cdivd(rho, rv);
      LQ_TRY(lin3(c, s, {1, 0}, r, {-alpha.r, -alpha.i}, &v));
      LQ_TRY(precond(s, sh));
      LQ_TRY(apply(sh, t));
      // one pass: <s, t> (its conjugate is <t, s>) and <t, t>
      cx<double> st;
      double tt = 0.0;
      LQ_TRY(dot(c, w, s, t, &st, &tt));
      omega = tt != 0.0 ? cx<double>{st.r / tt, -st.i / tt} : cx<double>{0, 0};
      LQ_TRY(lin3(c, x, {1, 0}, x, alpha, &ph, omega, &sh));
      LQ_TRY(lin3(c, r, {1, 0}, s, {-omega.r, -omega.i}, &t));
      rho_old = rho;
      ++iters;
      // one pass: the next rho = <rhat, r> and |r|^2
      double rn2 = 0.0;
      LQ_TRY(dot(c, w, rh, r, &rho, &rn2));
      if (log_level() >= 2)
        std::fprintf(stderr, "[lqcd] %s-FBiCGStab iteration %d: |r|/|b| %.3e\n", name, iters, std::sqrt(rn2) / bnorm);
      if (std::sqrt(rn2) <= target || (omega.r == 0.0 && omega.i == 0.0)) break;
    }
    ++restarts;
  }
  st.outer_iters = iters;
  st.inner_iters = napply;
  st.restarts = restarts > 0 ? restarts - 1 : 0;
  st.true_rel_resid = rnorm / bnorm;
  st.seconds_solve = std::chrono::duration<double>(clk::now() - t1).count();
  return status;
}

// D x = b with FP64 flexible BiCGStab, the FP32 SAP preconditioner on the right.
int solve_sap(lqcd_ctx* c, const lqcd_solve_params& prm, const int blk[4], int ncy, int nmr, const void* b_e,
              const void* b_o, void* x_e, void* x_o, bool zero_x, lqcd_solve_stats& st) {
  if (!sap_shape_ok(c->g, blk)) return set_error(LQCD_EINVAL, "bad SAP block shape");
  const size_t b32 = spinor_bytes(1, c->g.vh);
  FWork w;
  Pair e32, q32;
  for (Pair* q : {&e32, &q32})
    for (auto& h : q->h) LQ_TRY(w.alloc(b32, &h));
  FlexPrecond pre = [&](const void* ie, const void* io, void* oe, void* oo) -> int {
    LQ_TRY(launch_convert_field(c, 0, ie, 1, e32.h[0]));
    LQ_TRY(launch_convert_field(c, 0, io, 1, e32.h[1]));
    LQ_TRY(sap_apply(c, blk, ncy, nmr, e32.h[0], e32.h[1], q32.h[0], q32.h[1]));
    LQ_TRY(launch_convert_field(c, 1, q32.h[0], 0, oe));
    LQ_TRY(launch_convert_field(c, 1, q32.h[1], 0, oo));
    return LQCD_OK;
  };
  return solve_flexible(c, prm, pre, "SAP", b_e, b_o, x_e, x_o, zero_x, st);
}

}  // namespace lq
