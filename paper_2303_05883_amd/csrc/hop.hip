// Even-odd hopping term ("Dslash") for gfx950, with fused epilogues.
//
// For an output site x of parity p it computes (Sec. 2 and Eq. (1) of the
// paper: the hop is the off-diagonal block D_pq = -kappa P_p H P_q)
//
//   (H psi)(x) = sum_mu eta (1 - gamma_mu) U_mu(x) psi(x+mu) + eta (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)
//
// One thread per output site. Per direction the neighbour spinor is projected
// to a half spinor h (2 spins x 3 colours), using (1 -+ gamma_mu) psi =
// (h, -+ i sigma_mu h) for spatial mu in the Dirac-Pauli basis and
// (1 -+ gamma_t) = 2 diag(0,0,1,1) / 2 diag(1,1,0,0) in time (so a t hop
// reads only half of the neighbour). The link's third row is rebuilt from
// the two stored rows, U (or U^dag) multiplies the two colour vectors of h, and
// the result is expanded back to 4 spins into the accumulator. eta = t_bc on
// t hops that cross the boundary.
//
// Epilogues (out at the output site):
//   EPI_SCALE       out = a H psi
//   EPI_SCALE_CLOV  out = C (a H psi)            C = clover slot of the output parity
//   EPI_XPAY        out = C x + a H psi          C x = x when no clover slot is given
// Fused reductions (per-block FP64 partial sums, reduced later in fixed order):
//   RED_DOT         <w, out>                      (2 doubles: re, im)
//   RED_TS          <out, x>, <out, out>          (3 doubles)
#include "fieldio.h"
#include "internal.h"

namespace lq {

// Spin projection for direction MU; FWD: (1 - gamma_mu), else (1 + gamma_mu).
// s: 12 complex (3*spin + colour), or for MU == 3 only the 6 needed (see below).
template <int MU, bool FWD, typename T>
__device__ inline void project(const cx<T> s[12], cx<T> h[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<T> s0 = s[c], s1 = s[3 + c], s2 = s[6 + c], s3 = s[9 + c];
    if (MU == 0) {  // h = u +- i sigma_x l
      h[c] = FWD ? s0 + mul_i(s3) : s0 - mul_i(s3);
      h[3 + c] = FWD ? s1 + mul_i(s2) : s1 - mul_i(s2);
    } else if (MU == 1) {  // i sigma_y l = (l1, -l0)
      h[c] = FWD ? s0 + s3 : s0 - s3;
      h[3 + c] = FWD ? s1 - s2 : s1 + s2;
    } else if (MU == 2) {  // i sigma_z l = (i l0, -i l1)
      h[c] = FWD ? s0 + mul_i(s2) : s0 - mul_i(s2);
      h[3 + c] = FWD ? s1 - mul_i(s3) : s1 + mul_i(s3);
    }
  }
}

// Accumulate the expanded spinor of w = U h (two colour vectors w[0..2], w[3..5]).
template <int MU, bool FWD, typename T>
__device__ inline void expand(cx<T> acc[12], const cx<T> w[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<T> w0 = w[c], w1 = w[3 + c];
    if (MU == 3) {
      if (FWD) {  // (1 - gamma_t): lower spins
        acc[6 + c] = acc[6 + c] + w0;
        acc[9 + c] = acc[9 + c] + w1;
      } else {
        acc[c] = acc[c] + w0;
        acc[3 + c] = acc[3 + c] + w1;
      }
      continue;
    }
    acc[c] = acc[c] + w0;
    acc[3 + c] = acc[3 + c] + w1;
    if (MU == 0) {  // lower = -+ i sigma_x w = -+ i (w1, w0)
      acc[6 + c] = acc[6 + c] + (FWD ? mul_mi(w1) : mul_i(w1));
      acc[9 + c] = acc[9 + c] + (FWD ? mul_mi(w0) : mul_i(w0));
    } else if (MU == 1) {  // -+ i sigma_y w = -+ (w1, -w0)
      acc[6 + c] = FWD ? acc[6 + c] - w1 : acc[6 + c] + w1;
      acc[9 + c] = FWD ? acc[9 + c] + w0 : acc[9 + c] - w0;
    } else {  // -+ i sigma_z w = -+ (i w0, -i w1)
      acc[6 + c] = acc[6 + c] + (FWD ? mul_mi(w0) : mul_i(w0));
      acc[9 + c] = acc[9 + c] + (FWD ? mul_i(w1) : mul_mi(w1));
    }
  }
}

// w = U h (FWD) or U^dag h, for both colour vectors of h.
template <bool FWD, typename T>
__device__ inline void link_mul(const cx<T> u[6], const cx<T> h[6], cx<T> w[6]) {
  cx<T> r2[3];
  reconstruct(u, r2);
  const cx<T> m[9] = {u[0], u[1], u[2], u[3], u[4], u[5], r2[0], r2[1], r2[2]};
#pragma unroll
  for (int v = 0; v < 2; ++v) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<T> s;
      if (FWD) {
        s = m[3 * a] * h[3 * v];
        s = s + m[3 * a + 1] * h[3 * v + 1];
        s = s + m[3 * a + 2] * h[3 * v + 2];
      } else {
        s = cmulc(m[a], h[3 * v]);
        s = s + cmulc(m[3 + a], h[3 * v + 1]);
        s = s + cmulc(m[6 + a], h[3 * v + 2]);
      }
      w[3 * v + a] = s;
    }
  }
}

template <int P, int MU, bool FWD>
__device__ inline void hop_dir(const void* in, const void* links, size_t vh, size_t nbr, size_t lidx, bool flip,
                               cx<typename IO<P>::T> acc[12]) {
  using T = typename IO<P>::T;
  cx<T> h[6];
  if (MU == 3) {
    // (1 - gamma_t) psi = 2 (0, 0, psi_2, psi_3); (1 + gamma_t) psi = 2 (psi_0, psi_1, 0, 0)
    cx<T> half[6];
    IO<P>::load_half(in, vh, nbr, !FWD, half);
    const T two = flip ? T(-2) : T(2);
#pragma unroll
    for (int k = 0; k < 6; ++k) h[k] = two * half[k];
  } else {
    cx<T> s[12];
    IO<P>::load_spinor(in, vh, nbr, s);
    project<MU, FWD>(s, h);
  }
  cx<T> u[6], w[6];
  IO<P>::load_link(links, vh, lidx, u);
  link_mul<FWD>(u, h, w);
  expand<MU, FWD>(acc, w);
}

struct HopArgs {
  const void* in;
  void* out;
  const char* gauge;   // base of the 2 x 4 link blocks of this precision
  size_t link_stride;  // bytes of one (parity, mu) link block
  const void* clov;
  const void* xown;
  const void* w;
  double* partials;
  const int* skip;
  double scale;
  Geom g;
  int p;
  int remap;
};

template <int P, int EPI, bool CLOV, int RED>
__global__ void __launch_bounds__(256) k_hop(HopArgs a) {
  using T = typename IO<P>::T;
  if (a.skip && *a.skip) return;
  const size_t vh = (size_t)a.g.vh;
  const int blk = logical_block(a.remap);
  const size_t i = (size_t)blk * blockDim.x + threadIdx.x;
  constexpr int NR = RED == RED_DOT ? 2 : (RED == RED_TS ? 3 : 0);
  double red[3] = {0.0, 0.0, 0.0};
  if (i < vh) {
    const Geom& g = a.g;
    const int ii = (int)i;
    const int xh = ii % g.lxh;
    int r = ii / g.lxh;
    const int y = r % g.ly;
    r /= g.ly;
    const int z = r % g.lz;
    const int t = r / g.lz;
    const int x = 2 * xh + ((y + z + t + a.p) & 1);
    const int row = ii - xh;  // index of the (y, z, t) row
    const int xf = (x + 1 == g.lx) ? 0 : x + 1;
    const int xb = (x == 0) ? g.lx - 1 : x - 1;
    const int yl = g.lxh, zl = g.lxh * g.ly, tl = g.lxh * g.ly * g.lz;
    const int iyf = ii + ((y + 1 == g.ly) ? -(g.ly - 1) * yl : yl);
    const int iyb = ii + ((y == 0) ? (g.ly - 1) * yl : -yl);
    const int izf = ii + ((z + 1 == g.lz) ? -(g.lz - 1) * zl : zl);
    const int izb = ii + ((z == 0) ? (g.lz - 1) * zl : -zl);
    const int itf = ii + ((t + 1 == g.lt) ? -(g.lt - 1) * tl : tl);
    const int itb = ii + ((t == 0) ? (g.lt - 1) * tl : -tl);
    const bool flipf = (g.t_bc < 0) && (t + 1 == g.lt);
    const bool flipb = (g.t_bc < 0) && (t == 0);

    const char* gf = a.gauge + (size_t)(a.p * 4) * a.link_stride;        // U_mu(x), parity p
    const char* gb = a.gauge + (size_t)((1 - a.p) * 4) * a.link_stride;  // U_mu(x - mu), parity 1-p
    const size_t ls = a.link_stride;

    cx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};

    hop_dir<P, 0, true>(a.in, gf + 0 * ls, vh, (size_t)(row + (xf >> 1)), i, false, acc);
    hop_dir<P, 0, false>(a.in, gb + 0 * ls, vh, (size_t)(row + (xb >> 1)), (size_t)(row + (xb >> 1)), false, acc);
    hop_dir<P, 1, true>(a.in, gf + 1 * ls, vh, (size_t)iyf, i, false, acc);
    hop_dir<P, 1, false>(a.in, gb + 1 * ls, vh, (size_t)iyb, (size_t)iyb, false, acc);
    hop_dir<P, 2, true>(a.in, gf + 2 * ls, vh, (size_t)izf, i, false, acc);
    hop_dir<P, 2, false>(a.in, gb + 2 * ls, vh, (size_t)izb, (size_t)izb, false, acc);
    hop_dir<P, 3, true>(a.in, gf + 3 * ls, vh, (size_t)itf, i, flipf, acc);
    hop_dir<P, 3, false>(a.in, gb + 3 * ls, vh, (size_t)itb, (size_t)itb, flipb, acc);

    const T sc = (T)a.scale;
    cx<T> out[12];
    if (EPI == EPI_SCALE) {
#pragma unroll
      for (int k = 0; k < 12; ++k) out[k] = sc * acc[k];
    } else if (EPI == EPI_SCALE_CLOV) {
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = sc * acc[k];
      clover_apply<P>(a.clov, vh, i, acc, out);
    } else {
      cx<T> xo[12];
      IO<P>::load_spinor(a.xown, vh, i, xo);
      if (CLOV) {
        cx<T> cxo[12];
        clover_apply<P>(a.clov, vh, i, xo, cxo);
#pragma unroll
        for (int k = 0; k < 12; ++k) out[k] = cxo[k] + sc * acc[k];
      } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) out[k] = xo[k] + sc * acc[k];
      }
      if (RED == RED_TS) {
        // <out, x> and <out, out>
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          const cx<T> d = cmulc(out[k], xo[k]);
          red[0] += (double)d.r;
          red[1] += (double)d.i;
          red[2] += (double)out[k].r * (double)out[k].r + (double)out[k].i * (double)out[k].i;
        }
      }
    }
    IO<P>::store_spinor(a.out, vh, i, out);
    if (RED == RED_DOT) {
      cx<T> wv[12];
      IO<P>::load_spinor(a.w, vh, i, wv);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const cx<T> d = cmulc(wv[k], out[k]);
        red[0] += (double)d.r;
        red[1] += (double)d.i;
      }
    }
  }
  if constexpr (NR > 0) block_reduce<NR>(red, a.partials + (size_t)blk * NR);
}

template <int P>
__global__ void __launch_bounds__(256) k_site(const void* clov, const void* in, void* out, size_t vh) {
  using T = typename IO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vh) return;
  cx<T> s[12], o[12];
  IO<P>::load_spinor(in, vh, i, s);
  if (clov) {
    clover_apply<P>(clov, vh, i, s, o);
    IO<P>::store_spinor(out, vh, i, o);
  } else {
    IO<P>::store_spinor(out, vh, i, s);
  }
}

int hop_blocks(lqcd_ctx* c, int prec) {
  const int bs = c->hop_block[prec];
  return (c->g.vh + bs - 1) / bs;
}

template <int P, int EPI, bool CLOV, int RED>
static void launch_t(const HopArgs& a, int nb, int bs, hipStream_t s) {
  hipLaunchKernelGGL((k_hop<P, EPI, CLOV, RED>), dim3(nb), dim3(bs), 0, s, a);
}

template <int P>
static int dispatch(lqcd_ctx* c, const HopCall& h, HopArgs& a, int nb, int bs) {
  const bool cl = h.clov != nullptr;
  hipStream_t s = c->stream;
  if (h.epi == EPI_SCALE && h.red == RED_NONE) {
    launch_t<P, EPI_SCALE, false, RED_NONE>(a, nb, bs, s);
  } else if (h.epi == EPI_SCALE && h.red == RED_DOT) {
    launch_t<P, EPI_SCALE, false, RED_DOT>(a, nb, bs, s);
  } else if (h.epi == EPI_SCALE_CLOV && h.red == RED_NONE) {
    if (cl) launch_t<P, EPI_SCALE_CLOV, true, RED_NONE>(a, nb, bs, s);
    else launch_t<P, EPI_SCALE, false, RED_NONE>(a, nb, bs, s);
  } else if (h.epi == EPI_XPAY) {
    if (h.red == RED_NONE) {
      if (cl) launch_t<P, EPI_XPAY, true, RED_NONE>(a, nb, bs, s);
      else launch_t<P, EPI_XPAY, false, RED_NONE>(a, nb, bs, s);
    } else if (h.red == RED_DOT) {
      if (cl) launch_t<P, EPI_XPAY, true, RED_DOT>(a, nb, bs, s);
      else launch_t<P, EPI_XPAY, false, RED_DOT>(a, nb, bs, s);
    } else {
      if (cl) launch_t<P, EPI_XPAY, true, RED_TS>(a, nb, bs, s);
      else launch_t<P, EPI_XPAY, false, RED_TS>(a, nb, bs, s);
    }
  } else {
    return set_error(LQCD_EINVAL, "unsupported hop epilogue/reduction combination");
  }
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int launch_hop(lqcd_ctx* c, const HopCall& h, int* nblocks_out) {
  if (!c->gauge[h.prec]) return set_error(LQCD_ESTATE, "gauge field not set");
  const int bs = c->hop_block[h.prec];
  if (bs % 64 != 0 || bs < 64 || bs > 256) return set_error(LQCD_EINVAL, "hop block size must be 64..256, multiple of 64");
  const int nb = hop_blocks(c, h.prec);
  if (nblocks_out) *nblocks_out = nb;
  if (h.red != RED_NONE && !h.partials) return set_error(LQCD_EINVAL, "reduction without a partials buffer");
  HopArgs a;
  a.in = h.in;
  a.out = h.out;
  a.gauge = reinterpret_cast<const char*>(c->gauge[h.prec]);
  a.link_stride = link_bytes(h.prec, c->g.vh);
  a.clov = h.clov;
  a.xown = h.xown;
  a.w = h.w;
  a.partials = h.partials;
  a.skip = h.skip;
  a.scale = h.scale;
  a.g = c->g;
  a.p = h.out_parity;
  a.remap = c->hop_remap[h.prec];
  switch (h.prec) {
    case 0: return dispatch<0>(c, h, a, nb, bs);
    case 1: return dispatch<1>(c, h, a, nb, bs);
    case 2: return dispatch<2>(c, h, a, nb, bs);
  }
  return set_error(LQCD_EINVAL, "bad precision");
}

int launch_site(lqcd_ctx* c, int prec, const void* clov, const void* in, void* out) {
  const size_t vh = c->g.vh;
  const int bs = 256;
  const int nb = (int)((vh + bs - 1) / bs);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_site<0>, dim3(nb), dim3(bs), 0, c->stream, clov, in, out, vh); break;
    case 1: hipLaunchKernelGGL(k_site<1>, dim3(nb), dim3(bs), 0, c->stream, clov, in, out, vh); break;
    case 2: hipLaunchKernelGGL(k_site<2>, dim3(nb), dim3(bs), 0, c->stream, clov, in, out, vh); break;
    default: return set_error(LQCD_EINVAL, "bad precision");
  }
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

}  // namespace lq
