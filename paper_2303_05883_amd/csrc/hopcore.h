// Device code shared by the single-field hop kernels (hop.hip) and the
// batched persistent hop (batch.hip): spin projection, link multiply, the
// per-direction hop, the launch-shape site mapping and the epilogues.
#pragma once

#include "fieldio.h"
#include "internal.h"

namespace lq {

// Fused multiply-add forms of the complex arithmetic (four FMAs per complex
// multiply-accumulate), used where the hop is bounded by vector issue: the
// multi-RHS hop and the FP16 hop (conversions on top of the arithmetic).
__device__ inline float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// c + a b and c + conj(a) b
template <typename T>
__device__ inline cx<T> cmadd(cx<T> a, cx<T> b, cx<T> c) {
  return {fmat(-a.i, b.i, fmat(a.r, b.r, c.r)), fmat(a.i, b.r, fmat(a.r, b.i, c.i))};
}
template <typename T>
__device__ inline cx<T> cmaddc(cx<T> a, cx<T> b, cx<T> c) {
  return {fmat(a.i, b.i, fmat(a.r, b.r, c.r)), fmat(-a.i, b.r, fmat(a.r, b.i, c.i))};
}
// c + f z, c + f (i z), c - f (i z) for a real factor f
template <typename T>
__device__ inline cx<T> caxpy(T f, cx<T> z, cx<T> c) {
  return {fmat(f, z.r, c.r), fmat(f, z.i, c.i)};
}
template <typename T>
__device__ inline cx<T> caxpy_i(T f, cx<T> z, cx<T> c) {
  return {fmat(-f, z.i, c.r), fmat(f, z.r, c.i)};
}
template <typename T>
__device__ inline cx<T> caxpy_mi(T f, cx<T> z, cx<T> c) {
  return {fmat(f, z.i, c.r), fmat(-f, z.r, c.i)};
}

// acc += f * (the four-spinor of w = U h for direction MU), f real: the
// projection's factor (2 and the boundary sign in t) and the FP16 scale.
template <int MU, bool FWD, typename T>
__device__ inline void expand_f(cx<T> acc[12], const cx<T> w[6], T f) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<T> w0 = w[c], w1 = w[3 + c];
    if (MU == 3) {
      if (FWD) {
        acc[6 + c] = caxpy(f, w0, acc[6 + c]);
        acc[9 + c] = caxpy(f, w1, acc[9 + c]);
      } else {
        acc[c] = caxpy(f, w0, acc[c]);
        acc[3 + c] = caxpy(f, w1, acc[3 + c]);
      }
      continue;
    }
    acc[c] = caxpy(f, w0, acc[c]);
    acc[3 + c] = caxpy(f, w1, acc[3 + c]);
    if (MU == 0) {  // lower = -+ i sigma_x w = -+ i (w1, w0)
      acc[6 + c] = FWD ? caxpy_mi(f, w1, acc[6 + c]) : caxpy_i(f, w1, acc[6 + c]);
      acc[9 + c] = FWD ? caxpy_mi(f, w0, acc[9 + c]) : caxpy_i(f, w0, acc[9 + c]);
    } else if (MU == 1) {  // -+ i sigma_y w = -+ (w1, -w0)
      acc[6 + c] = caxpy(FWD ? -f : f, w1, acc[6 + c]);
      acc[9 + c] = caxpy(FWD ? f : -f, w0, acc[9 + c]);
    } else {  // -+ i sigma_z w = -+ (i w0, -i w1)
      acc[6 + c] = FWD ? caxpy_mi(f, w0, acc[6 + c]) : caxpy_i(f, w0, acc[6 + c]);
      acc[9 + c] = FWD ? caxpy_i(f, w1, acc[9 + c]) : caxpy_mi(f, w1, acc[9 + c]);
    }
  }
}

// y = M x (M Hermitian 6x6 in the 18-slot packed form), fused multiply-adds.
template <typename T>
__device__ inline void herm6_mul_fma(const cx<T> m[18], const cx<T> x[6], cx<T> y[6]) {
  const T d[6] = {m[0].r, m[0].i, m[1].r, m[1].i, m[2].r, m[2].i};
#pragma unroll
  for (int a = 0; a < 6; ++a) y[a] = d[a] * x[a];
  int k = 3;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
#pragma unroll
    for (int b = a + 1; b < 6; ++b) {
      const cx<T> c = m[k++];
      y[a] = cmadd(c, x[b], y[a]);
      y[b] = cmaddc(c, x[a], y[b]);
    }
  }
}

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

// G5: the hop acts on gamma5 psi instead of psi (gamma5 of the Dirac-Pauli
// basis swaps the upper and lower spin pairs with a minus sign).
template <int P, int MU, bool FWD, bool NT, bool G5 = false>
__device__ inline void hop_dir(const void* in, const void* links, size_t vh, size_t nbr, size_t lidx, bool flip,
                               cx<typename IO<P>::T> acc[12]) {
  using T = typename IO<P>::T;
  cx<T> h[6];
  if (MU == 3) {
    // (1 - gamma_t) psi = 2 (0, 0, psi_2, psi_3); (1 + gamma_t) psi = 2 (psi_0, psi_1, 0, 0)
    cx<T> half[6];
    IO<P>::load_half(in, nbr, G5 ? FWD : !FWD, half);
    const T two = (flip != G5) ? T(-2) : T(2);
#pragma unroll
    for (int k = 0; k < 6; ++k) h[k] = two * half[k];
  } else {
    cx<T> s[12];
    IO<P>::load_spinor(in, nbr, s);
    if (G5) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const cx<T> u = s[k];
        s[k] = T(-1) * s[6 + k];
        s[6 + k] = T(-1) * u;
      }
    }
    project<MU, FWD>(s, h);
  }
  cx<T> u[6], w[6];
  IO<P>::template load_link<NT>(links, lidx, u);
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
  int remap;  // 0: linear, 1: XCD-contiguous ranges, 2: XCD z-slabs (see map_site)
  int hz;     // z extent of one XCD slab (remap 2)
};

// Site of this thread (local = index among the block's sites, spb sites per
// block). remap 2 gives XCD k (blocks are dealt to the 8 XCDs round-robin) the
// slab z in [k hz, (k+1) hz) and walks it x, y fastest, then z, then t, so that
// the z and t neighbours of the sites in flight were read shortly before and
// are still in that XCD's L2. Returns false for threads past the slab's end.
__device__ inline bool map_site(const HopArgs& a, int spb, int local, size_t& i) {
  if (a.remap == 2) {
    const int k = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int xy = a.g.lxh * a.g.ly;
    const int q = j * spb + local;
    if (q >= xy * a.hz * a.g.lt) return false;
    const int xyi = q % xy, rest = q / xy;
    const int zin = rest % a.hz, t = rest / a.hz;
    i = (size_t)xyi + (size_t)xy * ((size_t)(k * a.hz + zin) + (size_t)a.g.lz * t);
    return true;
  }
  i = (size_t)logical_block(a.remap) * spb + local;
  return i < (size_t)a.g.vh;
}


// The epilogue shared by the hop kernels: out from the hop sum acc at site i,
// plus the fused reductions of this site added into red.
template <int P, int EPI, bool CLOV, int RED>
__device__ inline void hop_epilogue(const HopArgs& a, size_t i, cx<typename IO<P>::T> acc[12],
                                    cx<typename IO<P>::T> out[12], double red[3]) {
  using T = typename IO<P>::T;
  const T sc = (T)a.scale;
  if (EPI == EPI_SCALE) {
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = sc * acc[k];
  } else if (EPI == EPI_SCALE_CLOV) {
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = sc * acc[k];
    clover_apply<P>(a.clov, i, acc, out);
  } else {
    cx<T> xo[12];
    IO<P>::load_spinor(a.xown, i, xo);
    if (CLOV) {
      cx<T> cxo[12];
      clover_apply<P>(a.clov, i, xo, cxo);
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
  if (RED == RED_DOT) {
    cx<T> wv[12];
    IO<P>::load_spinor(a.w, i, wv);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const cx<T> d = cmulc(wv[k], out[k]);
      red[0] += (double)d.r;
      red[1] += (double)d.i;
    }
  }
}


// One output site of the 1-lane hop: H psi at site i, the epilogue, the store,
// and this site's share of the fused reductions added into red.
template <int P, int EPI, bool CLOV, int RED, bool NT>
__device__ inline void hop_site(const HopArgs& a, size_t i, double red[3]) {
  using T = typename IO<P>::T;
  const size_t vh = (size_t)a.g.vh;
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

  hop_dir<P, 0, true, NT>(a.in, gf + 0 * ls, vh, (size_t)(row + (xf >> 1)), i, false, acc);
  hop_dir<P, 0, false, NT>(a.in, gb + 0 * ls, vh, (size_t)(row + (xb >> 1)), (size_t)(row + (xb >> 1)), false, acc);
  hop_dir<P, 1, true, NT>(a.in, gf + 1 * ls, vh, (size_t)iyf, i, false, acc);
  hop_dir<P, 1, false, NT>(a.in, gb + 1 * ls, vh, (size_t)iyb, (size_t)iyb, false, acc);
  hop_dir<P, 2, true, NT>(a.in, gf + 2 * ls, vh, (size_t)izf, i, false, acc);
  hop_dir<P, 2, false, NT>(a.in, gb + 2 * ls, vh, (size_t)izb, (size_t)izb, false, acc);
  hop_dir<P, 3, true, NT>(a.in, gf + 3 * ls, vh, (size_t)itf, i, flipf, acc);
  hop_dir<P, 3, false, NT>(a.in, gb + 3 * ls, vh, (size_t)itb, (size_t)itb, flipb, acc);

  cx<T> out[12];
  hop_epilogue<P, EPI, CLOV, RED>(a, i, acc, out, red);
  IO<P>::store_spinor(a.out, i, out);
}

// ------------------------------------------------------------------ several right-hand sides
// NB right-hand sides of one lattice at one site: each link (and its rebuilt
// third row) is loaded once per direction and applied to every right-hand
// side, so the link traffic per site-RHS falls by NB. act has bit r set for
// the right-hand sides to compute (uniform over a wavefront). The arithmetic is
// written as fused multiply-adds (four per complex multiply-accumulate): with
// the links shared, the multiply-RHS hop is bounded by vector issue as much as
// by memory.
template <int NB>
struct MultiPtrs {
  const void* in[NB];
  void* out[NB];
  const void* own[NB];
  const void* w[NB];
  unsigned act;
};

template <int P, int MU, bool FWD, bool NT, int NB>
__device__ inline void hop_dir_multi(const MultiPtrs<NB>& m, const void* links, size_t nbr, size_t lidx, bool flip,
                                     cx<typename IO<P>::T> acc[NB][12]) {
  using T = typename IO<P>::T;
  cx<T> u[6], r2[3];
  IO<P>::template load_link<NT>(links, lidx, u);
  reconstruct(u, r2);
  const cx<T> M[9] = {u[0], u[1], u[2], u[3], u[4], u[5], r2[0], r2[1], r2[2]};
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    if (!((m.act >> r) & 1u)) continue;
    cx<T> h[6];
    T f;
    if (MU == 3) {
      // (1 - gamma_t) psi = 2 (0, 0, psi_2, psi_3); (1 + gamma_t) psi = 2 (psi_0, psi_1, 0, 0)
      IO<P>::load_half_codes(m.in[r], nbr, !FWD, h, f);
      f = flip ? T(-2) * f : T(2) * f;
    } else {
      cx<T> s[12];
      IO<P>::load_spinor_codes(m.in[r], nbr, s, f);
      project<MU, FWD>(s, h);
    }
    cx<T> w[6];
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cx<T> q;
        if (FWD) {
          q = M[3 * a] * h[3 * v];
          q = cmadd(M[3 * a + 1], h[3 * v + 1], q);
          q = cmadd(M[3 * a + 2], h[3 * v + 2], q);
        } else {
          q = cmulc(M[a], h[3 * v]);
          q = cmaddc(M[3 + a], h[3 * v + 1], q);
          q = cmaddc(M[6 + a], h[3 * v + 2], q);
        }
        w[3 * v + a] = q;
      }
    expand_f<MU, FWD>(acc[r], w, f);
  }
}

template <int P, int EPI, bool CLOV, int RED, bool NT, int NB>
__device__ inline void hop_site_multi(const HopArgs& a, const MultiPtrs<NB>& m, size_t i, double red[NB][3]) {
  using T = typename IO<P>::T;
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
  const char* gf = a.gauge + (size_t)(a.p * 4) * a.link_stride;
  const char* gb = a.gauge + (size_t)((1 - a.p) * 4) * a.link_stride;
  const size_t ls = a.link_stride;

  cx<T> acc[NB][12];
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[q][k] = {T(0), T(0)};

  hop_dir_multi<P, 0, true, NT, NB>(m, gf + 0 * ls, (size_t)(row + (xf >> 1)), i, false, acc);
  hop_dir_multi<P, 0, false, NT, NB>(m, gb + 0 * ls, (size_t)(row + (xb >> 1)), (size_t)(row + (xb >> 1)), false,
                                     acc);
  hop_dir_multi<P, 1, true, NT, NB>(m, gf + 1 * ls, (size_t)iyf, i, false, acc);
  hop_dir_multi<P, 1, false, NT, NB>(m, gb + 1 * ls, (size_t)iyb, (size_t)iyb, false, acc);
  hop_dir_multi<P, 2, true, NT, NB>(m, gf + 2 * ls, (size_t)izf, i, false, acc);
  hop_dir_multi<P, 2, false, NT, NB>(m, gb + 2 * ls, (size_t)izb, (size_t)izb, false, acc);
  hop_dir_multi<P, 3, true, NT, NB>(m, gf + 3 * ls, (size_t)itf, i, flipf, acc);
  hop_dir_multi<P, 3, false, NT, NB>(m, gb + 3 * ls, (size_t)itb, (size_t)itb, flipb, acc);

  if (EPI == EPI_SCALE_CLOV) {
    // out = A (scale acc): each chiral block of A is loaded once and applied
    // to every right-hand side (acc[q] holds c_+ in 0..5 and c_- in 6..11,
    // then A_+ c_+ in 0..5 while the second block is applied)
    const T sc = (T)a.scale;
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const cx<T> u = acc[q][k], l = acc[q][k + 6];
        acc[q][k] = sc * (u - l);
        acc[q][k + 6] = sc * (u + l);
      }
    cx<T> mb[18];
    IO<P>::template load_clover_block<NT>(a.clov, i, 0, mb);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (!((m.act >> q) & 1u)) continue;
      cx<T> yv[6];
      herm6_mul_fma(mb, acc[q], yv);
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[q][k] = yv[k];
    }
    IO<P>::template load_clover_block<NT>(a.clov, i, 1, mb);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (!((m.act >> q) & 1u)) continue;
      cx<T> yv[6], out[12];
      herm6_mul_fma(mb, acc[q] + 6, yv);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        out[k] = acc[q][k] + yv[k];
        out[k + 6] = yv[k] - acc[q][k];
      }
      IO<P>::store_spinor(m.out[q], i, out);
    }
    return;
  }
  if (EPI == EPI_XPAY && CLOV) {
    // out = A x_own + scale acc, the chiral blocks of A loaded once for all
    // right-hand sides: xo[q] holds c_+, c_- of x_own, then A_+ c_+ in 0..5
    const T sc = (T)a.scale;
    cx<T> xo[NB][12];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (!((m.act >> q) & 1u)) continue;
      IO<P>::load_spinor(m.own[q], i, xo[q]);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const cx<T> u = xo[q][k], l = xo[q][k + 6];
        xo[q][k] = u - l;
        xo[q][k + 6] = u + l;
      }
    }
    cx<T> mb[18];
    IO<P>::template load_clover_block<NT>(a.clov, i, 0, mb);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (!((m.act >> q) & 1u)) continue;
      cx<T> yv[6];
      herm6_mul_fma(mb, xo[q], yv);
#pragma unroll
      for (int k = 0; k < 6; ++k) xo[q][k] = yv[k];
    }
    IO<P>::template load_clover_block<NT>(a.clov, i, 1, mb);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (!((m.act >> q) & 1u)) continue;
      cx<T> yv[6], out[12];
      herm6_mul_fma(mb, xo[q] + 6, yv);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        out[k] = caxpy(sc, acc[q][k], xo[q][k] + yv[k]);
        out[k + 6] = caxpy(sc, acc[q][k + 6], yv[k] - xo[q][k]);
      }
      if (RED == RED_TS) {
        // <out, x_own> and <out, out> (x_own read again, from the cache)
        cx<T> x0[12];
        IO<P>::load_spinor(m.own[q], i, x0);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          const cx<T> d = cmulc(out[k], x0[k]);
          red[q][0] += (double)d.r;
          red[q][1] += (double)d.i;
          red[q][2] += (double)out[k].r * (double)out[k].r + (double)out[k].i * (double)out[k].i;
        }
      } else if (RED == RED_DOT) {
        cx<T> wv[12];
        IO<P>::load_spinor(m.w[q], i, wv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          const cx<T> d = cmulc(wv[k], out[k]);
          red[q][0] += (double)d.r;
          red[q][1] += (double)d.i;
        }
      }
      IO<P>::store_spinor(m.out[q], i, out);
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (!((m.act >> q) & 1u)) continue;
    HopArgs aq = a;
    aq.xown = m.own[q];
    aq.w = m.w[q];
    cx<T> out[12];
    hop_epilogue<P, EPI, CLOV, RED>(aq, i, acc[q], out, red[q]);
    IO<P>::store_spinor(m.out[q], i, out);
  }
}

}  // namespace lq
