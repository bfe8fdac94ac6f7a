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

#include "hopcore.h"

namespace lq {

template <int P, int EPI, bool CLOV, int RED, bool NT>
__global__ void __launch_bounds__(256) k_hop(HopArgs a) {
  if (a.skip && *a.skip) return;
  const int blk = blockIdx.x;
  size_t i = 0;
  const bool active = map_site(a, blockDim.x, threadIdx.x, i);
  constexpr int NR = RED == RED_DOT ? 2 : (RED == RED_TS ? 3 : 0);
  double red[3] = {0.0, 0.0, 0.0};
  if (active) hop_site<P, EPI, CLOV, RED, NT>(a, i, red);
  if constexpr (NR > 0) block_reduce<NR>(red, a.partials + (size_t)blk * NR);
}

// Direction-split hop: four lanes of a quad share one output site, lane mu
// taking the forward and backward hops in direction mu. Every lane issues its
// two neighbour loads and two link loads before any arithmetic, so a site has
// all of its 16 reads in flight at once with a quarter of the registers per
// lane; the four partial sums are added with quad DPP exchanges. The lanes run
// one instruction stream: the direction enters only through the coefficients
// of the spin projection and reconstruction, (1 -+ gamma_mu) psi = (h, P h)
// with h = a u + c0 l_{j0}, ... (see below). The epilogue is computed by all
// four lanes; the stores are split between them.
template <int P, int EPI, bool CLOV, int RED, bool NT>
__global__ void __launch_bounds__(256) k_hop4(HopArgs a) {
  using T = typename IO<P>::T;
  if (a.skip && *a.skip) return;
  const int blk = blockIdx.x;
  const int mu = threadIdx.x & 3;
  size_t i = 0;
  const bool active = map_site(a, blockDim.x >> 2, threadIdx.x >> 2, i);
  constexpr int NR = RED == RED_DOT ? 2 : (RED == RED_TS ? 3 : 0);
  double red[3] = {0.0, 0.0, 0.0};
  if (active) {
    const Geom& g = a.g;
    const int ii = (int)i;
    const int xh = ii % g.lxh;
    int r = ii / g.lxh;
    const int y = r % g.ly;
    r /= g.ly;
    const int z = r % g.lz;
    const int t = r / g.lz;
    const int x = 2 * xh + ((y + z + t + a.p) & 1);
    // neighbour indices in direction mu, computed without branching: for
    // mu = 0 the checkerboarded x index moves within the row, otherwise the
    // index moves by the direction's stride with a periodic wrap
    const bool tdir = mu == 3;
    const int c = mu == 1 ? y : (mu == 2 ? z : t);
    const int L = mu == 1 ? g.ly : (mu == 2 ? g.lz : g.lt);
    const int st = mu == 1 ? g.lxh : (mu == 2 ? g.lxh * g.ly : g.lxh * g.ly * g.lz);
    const int row = ii - xh;
    const int xnf = row + (((x + 1 == g.lx) ? 0 : x + 1) >> 1);
    const int xnb = row + (((x == 0) ? g.lx - 1 : x - 1) >> 1);
    const int nf = mu == 0 ? xnf : ii + ((c + 1 == L) ? -(L - 1) * st : st);
    const int nb = mu == 0 ? xnb : ii + ((c == 0) ? (L - 1) * st : -st);
    const bool flipf = tdir && (g.t_bc < 0) && (t + 1 == g.lt);
    const bool flipb = tdir && (g.t_bc < 0) && (t == 0);
    // loads first, the same instructions in every lane: a t lane needs one
    // half of each neighbour and reads it into both halves (its other half is
    // multiplied by zero below)
    cx<T> sf[12], sb[12], uf[6], ub[6];
    const char* lf = a.gauge + (size_t)(a.p * 4 + mu) * a.link_stride;
    const char* lb = a.gauge + (size_t)((1 - a.p) * 4 + mu) * a.link_stride;
    IO<P>::template load_link<NT>(lf, i, uf);
    IO<P>::template load_link<NT>(lb, (size_t)nb, ub);
    IO<P>::load_spinor_sel(a.in, (size_t)nf, tdir ? 2 : 0, sf);
    IO<P>::load_spinor_sel(a.in, (size_t)nb, tdir ? 1 : 0, sb);
    // projection h0 = A s0 + C0 s_{j0}, h1 = A s1 + C1 s_{j1} (j0, j1 = 3, 2 for
    // x and y, 2, 3 for z and t); expansion upper += B w, lower0 += D0 w_{m0},
    // lower1 += D1 w_{m1} (m0, m1 = 1, 0 for x and y, 0, 1 for z and t).
    // Backward hops negate C and D; in t the forward hop is (0, 2 l), the
    // backward one (2 u, 0); eta = -1 flips h.
    const bool sw = mu < 2;
    const T c0r = mu == 1 ? T(1) : (tdir ? T(2) : T(0));
    const T c0i = (mu == 0 || mu == 2) ? T(1) : T(0);
    const T c1r = mu == 1 ? T(-1) : (tdir ? T(2) : T(0));
    const T c1i = mu == 0 ? T(1) : (mu == 2 ? T(-1) : T(0));
    const T d0r = mu == 1 ? T(-1) : (tdir ? T(1) : T(0));
    const T d0i = (mu == 0 || mu == 2) ? T(-1) : T(0);
    const T d1r = (mu == 1 || tdir) ? T(1) : T(0);
    const T d1i = mu == 0 ? T(-1) : (mu == 2 ? T(1) : T(0));
    cx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      const bool fwd = dir == 0;
      const cx<T>* s = fwd ? sf : sb;
      const T e = (fwd ? flipf : flipb) ? T(-1) : T(1);
      const T A = e * (tdir ? (fwd ? T(0) : T(2)) : T(1));
      const T sg = fwd ? e : -e;  // sign of C for this hop (backward negates; eta flips)
      const T C0r = tdir && !fwd ? T(0) : sg * c0r, C0i = sg * c0i;
      const T C1r = tdir && !fwd ? T(0) : sg * c1r, C1i = sg * c1i;
      cx<T> h[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cx<T> l0 = sw ? s[9 + c] : s[6 + c];
        const cx<T> l1 = sw ? s[6 + c] : s[9 + c];
        h[c] = {A * s[c].r + C0r * l0.r - C0i * l0.i, A * s[c].i + C0r * l0.i + C0i * l0.r};
        h[3 + c] = {A * s[3 + c].r + C1r * l1.r - C1i * l1.i, A * s[3 + c].i + C1r * l1.i + C1i * l1.r};
      }
      cx<T> w[6];
      if (fwd) link_mul<true>(uf, h, w);
      else link_mul<false>(ub, h, w);
      const T B = tdir && fwd ? T(0) : T(1);
      const T ds = fwd ? T(1) : T(-1);
      const T D0r = tdir ? (fwd ? T(1) : T(0)) : ds * d0r, D0i = ds * d0i;
      const T D1r = tdir ? (fwd ? T(1) : T(0)) : ds * d1r, D1i = ds * d1i;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cx<T> w0 = w[c], w1 = w[3 + c];
        const cx<T> m0 = sw ? w1 : w0, m1 = sw ? w0 : w1;
        acc[c] = acc[c] + B * w0;
        acc[3 + c] = acc[3 + c] + B * w1;
        acc[6 + c] = acc[6 + c] + cx<T>{D0r * m0.r - D0i * m0.i, D0r * m0.i + D0i * m0.r};
        acc[9 + c] = acc[9 + c] + cx<T>{D1r * m1.r - D1i * m1.i, D1r * m1.i + D1i * m1.r};
      }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {quad_sum(acc[k].r), quad_sum(acc[k].i)};
    cx<T> out[12];
    hop_epilogue<P, EPI, CLOV, RED>(a, i, acc, out, red);
    if (mu != 0) red[0] = red[1] = red[2] = 0.0;
    IO<P>::store_part(a.out, i, out, mu, 4);
  }
  if constexpr (NR > 0) block_reduce<NR>(red, a.partials + (size_t)blk * NR);
}


// Pair-split hop: two lanes share one output site, one taking the four
// forward hops and the other the four backward ones, in one instruction
// stream (the two differ only in signs, the neighbour and link they read, and
// U against U^dag). Lanes 0..31 of a wavefront take the forward hops of 32
// consecutive sites and lanes 32..63 the backward hops of the same sites, so
// every load instruction still reads whole contiguous runs (two 512-byte runs)
// and the partial sums meet with one cross-half lane swap. A CU then holds
// half as many sites in flight as with one lane per site for the same bytes in
// flight, so more of the z and t neighbours of those sites are still in the
// XCD's L2. The loads of HOP2_PF directions are issued ahead of the arithmetic
// of the current one.
#ifndef HOP2_PF
#define HOP2_PF 2
#endif

template <int P>
struct PairIn {
  cx<typename IO<P>::T> u[6], s[12];
};

template <int P, int MU, bool NT>
__device__ inline void pair_load(const void* in, const char* links, size_t vh, size_t nbr, size_t lidx, bool fwd,
                                 PairIn<P>& d) {
  IO<P>::template load_link<NT>(links, lidx, d.u);
  if (MU == 3) IO<P>::load_spinor_sel(in, nbr, fwd ? 2 : 1, d.s);  // the needed half, in both halves
  else IO<P>::load_spinor(in, nbr, d.s);
}

template <int P, int MU>
__device__ inline void pair_compute(const PairIn<P>& d, bool fwd, bool flip, cx<typename IO<P>::T> acc[12]) {
  using T = typename IO<P>::T;
  const cx<T>* s = d.s;
  const T sg = fwd ? T(1) : T(-1);
  cx<T> h[6];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (MU == 3) {  // the FP16 load brings the whole spinor, the others the selected half twice
      const T two = flip ? T(-2) : T(2);
      h[c] = two * ((P == 2 && fwd) ? s[6 + c] : s[c]);
      h[3 + c] = two * ((P == 2 && fwd) ? s[9 + c] : s[3 + c]);
    } else if (MU == 0) {  // h = u + sg i sigma_x l = (s0 + sg i s3, s1 + sg i s2)
      h[c] = s[c] + sg * mul_i(s[9 + c]);
      h[3 + c] = s[3 + c] + sg * mul_i(s[6 + c]);
    } else if (MU == 1) {  // i sigma_y l = (s3, -s2)
      h[c] = s[c] + sg * s[9 + c];
      h[3 + c] = s[3 + c] - sg * s[6 + c];
    } else {  // i sigma_z l = (i s2, -i s3)
      h[c] = s[c] + sg * mul_i(s[6 + c]);
      h[3 + c] = s[3 + c] - sg * mul_i(s[9 + c]);
    }
  }
  cx<T> r2[3];
  reconstruct(d.u, r2);
  const cx<T> U9[9] = {d.u[0], d.u[1], d.u[2], d.u[3], d.u[4], d.u[5], r2[0], r2[1], r2[2]};
  cx<T> M[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[3 * a + b] = fwd ? U9[3 * a + b] : conj(U9[3 * b + a]);
  cx<T> w[6];
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<T> q = M[3 * a] * h[3 * v];
      q = q + M[3 * a + 1] * h[3 * v + 1];
      q = q + M[3 * a + 2] * h[3 * v + 2];
      w[3 * v + a] = q;
    }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<T> w0 = w[c], w1 = w[3 + c];
    if (MU == 3) {  // forward: lower spins; backward: upper spins
      const T fw = fwd ? T(1) : T(0), bw = fwd ? T(0) : T(1);
      acc[c] = acc[c] + bw * w0;
      acc[3 + c] = acc[3 + c] + bw * w1;
      acc[6 + c] = acc[6 + c] + fw * w0;
      acc[9 + c] = acc[9 + c] + fw * w1;
    } else {
      acc[c] = acc[c] + w0;
      acc[3 + c] = acc[3 + c] + w1;
      if (MU == 0) {  // lower += -sg i sigma_x w = -sg (i w1, i w0)
        acc[6 + c] = acc[6 + c] - sg * mul_i(w1);
        acc[9 + c] = acc[9 + c] - sg * mul_i(w0);
      } else if (MU == 1) {  // -sg (w1, -w0)
        acc[6 + c] = acc[6 + c] - sg * w1;
        acc[9 + c] = acc[9 + c] + sg * w0;
      } else {  // -sg (i w0, -i w1)
        acc[6 + c] = acc[6 + c] - sg * mul_i(w0);
        acc[9 + c] = acc[9 + c] + sg * mul_i(w1);
      }
    }
  }
}

template <int P, int EPI, bool CLOV, int RED, bool NT>
__global__ void __launch_bounds__(256) k_hop2(HopArgs a) {
  using T = typename IO<P>::T;
  if (a.skip && *a.skip) return;
  const size_t vh = (size_t)a.g.vh;
  const int blk = blockIdx.x;
  const int half = (threadIdx.x >> 5) & 1;
  const bool fwd = half == 0;
  size_t i = 0;
  const bool active = map_site(a, blockDim.x >> 1, ((threadIdx.x >> 6) << 5) | (threadIdx.x & 31), i);
  constexpr int NR = RED == RED_DOT ? 2 : (RED == RED_TS ? 3 : 0);
  double red[3] = {0.0, 0.0, 0.0};
  if (active) {
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
    // this lane's neighbour in each direction: forward or backward
    size_t nb[4];
    nb[0] = (size_t)(row + ((fwd ? ((x + 1 == g.lx) ? 0 : x + 1) : ((x == 0) ? g.lx - 1 : x - 1)) >> 1));
    nb[1] = (size_t)(fwd ? ii + ((y + 1 == g.ly) ? -(g.ly - 1) * yl : yl) : ii + ((y == 0) ? (g.ly - 1) * yl : -yl));
    nb[2] = (size_t)(fwd ? ii + ((z + 1 == g.lz) ? -(g.lz - 1) * zl : zl) : ii + ((z == 0) ? (g.lz - 1) * zl : -zl));
    nb[3] = (size_t)(fwd ? ii + ((t + 1 == g.lt) ? -(g.lt - 1) * tl : tl) : ii + ((t == 0) ? (g.lt - 1) * tl : -tl));
    const bool flip = (g.t_bc < 0) && (fwd ? (t + 1 == g.lt) : (t == 0));
    // forward hops read U_mu(x) (parity p, index i); backward hops U_mu(x - mu) (parity 1-p)
    const char* gl = a.gauge + (size_t)((fwd ? a.p : 1 - a.p) * 4) * a.link_stride;
    const size_t ls = a.link_stride;
    cx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
#define LD(MU, B) pair_load<P, MU, NT>(a.in, gl + MU * ls, vh, nb[MU], fwd ? i : nb[MU], fwd, d[B])
#define CP(MU, B) pair_compute<P, MU>(d[B], fwd, MU == 3 && flip, acc)
#if HOP2_PF >= 4
    PairIn<P> d[4];
    LD(0, 0); LD(1, 1); LD(2, 2); LD(3, 3);
    CP(0, 0); CP(1, 1); CP(2, 2); CP(3, 3);
#elif HOP2_PF == 3
    PairIn<P> d[3];
    LD(0, 0); LD(1, 1); LD(2, 2);
    CP(0, 0); LD(3, 0); CP(1, 1); CP(2, 2); CP(3, 0);
#elif HOP2_PF == 2
    PairIn<P> d[2];
    LD(0, 0); LD(1, 1);
    CP(0, 0); LD(2, 0); CP(1, 1); LD(3, 1); CP(2, 0); CP(3, 1);
#else
    PairIn<P> d[1];
    LD(0, 0); CP(0, 0); LD(1, 0); CP(1, 0); LD(2, 0); CP(2, 0); LD(3, 0); CP(3, 0);
#endif
#undef LD
#undef CP
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {half_sum(acc[k].r), half_sum(acc[k].i)};
    cx<T> out[12];
    hop_epilogue<P, EPI, CLOV, RED>(a, i, acc, out, red);
    if (half != 0) red[0] = red[1] = red[2] = 0.0;
    IO<P>::store_part(a.out, i, out, half, 2);
  }
  if constexpr (NR > 0) block_reduce<NR>(red, a.partials + (size_t)blk * NR);
}

// ------------------------------------------------------------------ plane march
// One workgroup per (tile of `ty` full rows of the xy plane, chunk of `zc`
// planes in z, t). Lane (xh, y) computes the outputs of its column (xh, y) for
// the zc planes in turn. At each z the input spinors of the tile's plane pass
// through LDS, each loaded from memory once, by the lane of the same (xh, y),
// and supply the x and y neighbours of every lane; the z neighbours are the
// lane's own column (the spinors of the next two planes are held in
// registers: the nearer is the z-forward neighbour and then this lane's LDS
// entry, the farther is loaded two steps ahead, so that a chunk's last (halo)
// plane is read at about the time the next chunk's workgroup reads it as its
// own; the projected half of the previous plane is kept for the z-backward
// hop); the t neighbours and the links come from memory. Rows above and below the tile are staged by the
// first and last row of lanes unless the tile is the whole plane (WRAP).
template <typename T>
struct LdsWord;
template <>
struct LdsWord<double> {
  using W = double2;
  static constexpr int N = 12;
  __device__ static inline void put(W* L, int ns, int slot, const cx<double> s[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) L[k * ns + slot] = make_double2(s[k].r, s[k].i);
  }
  __device__ static inline void get(const W* L, int ns, int slot, cx<double> s[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double2 v = L[k * ns + slot];
      s[k] = {v.x, v.y};
    }
  }
};
template <>
struct LdsWord<float> {
  using W = float4;
  static constexpr int N = 6;
  __device__ static inline void put(W* L, int ns, int slot, const cx<float> s[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) L[k * ns + slot] = make_float4(s[2 * k].r, s[2 * k].i, s[2 * k + 1].r, s[2 * k + 1].i);
  }
  __device__ static inline void get(const W* L, int ns, int slot, cx<float> s[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const float4 v = L[k * ns + slot];
      s[2 * k] = {v.x, v.y};
      s[2 * k + 1] = {v.z, v.w};
    }
  }
};

// One hop with the neighbour's projected half h given.
template <int P, int MU, bool FWD>
__device__ inline void hop_half(const cx<typename IO<P>::T> h[6], const char* links, size_t lidx,
                                cx<typename IO<P>::T> acc[12]) {
  using T = typename IO<P>::T;
  cx<T> u[6], w[6];
  IO<P>::template load_link<true>(links, lidx, u);
  link_mul<FWD>(u, h, w);
  expand<MU, FWD>(acc, w);
}

template <int P, int EPI, bool CLOV, int RED, bool WRAP>
__global__ void __launch_bounds__(512) k_hopz(HopArgs a, int ty, int zc) {
  using T = typename IO<P>::T;
  using LW = LdsWord<T>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  typename LW::W* L = reinterpret_cast<typename LW::W*>(lds_raw);
  constexpr int NR = RED == RED_DOT ? 2 : (RED == RED_TS ? 3 : 0);
  if (a.skip && *a.skip) return;
  const Geom& g = a.g;
  const int lxh = g.lxh;
  const int ns = (WRAP ? ty : ty + 2) * lxh;  // sites of the LDS plane
  const int nzc = g.lz / zc, nyt = g.ly / ty;
  // z chunk fastest, then row tile, then t: each XCD (one contiguous range of
  // logical blocks) holds whole t slices, so the z and y halos and most t
  // neighbours are read by blocks of the same XCD
  const int lb = logical_block(a.remap);
  const int z0 = (lb % nzc) * zc;
  const int rest = lb / nzc;
  const int y0 = (rest % nyt) * ty;
  const int t = rest / nyt;
  const int xh = threadIdx.x % lxh, yr = threadIdx.x / lxh;
  const int y = y0 + yr;
  const int lr = WRAP ? yr : yr + 1;
  const int slot = lr * lxh + xh;
  const int lyf = WRAP ? (yr + 1 == ty ? 0 : yr + 1) : lr + 1;
  const int lyb = WRAP ? (yr == 0 ? ty - 1 : yr - 1) : lr - 1;
  const bool hlo = !WRAP && yr == 0, hhi = !WRAP && yr == ty - 1, halo = hlo || hhi;
  const int yh = hlo ? (y0 == 0 ? g.ly - 1 : y0 - 1) : (y0 + ty == g.ly ? 0 : y0 + ty);
  const int hslot = hlo ? xh : (ty + 1) * lxh + xh;
  const size_t yl = (size_t)lxh, zl = yl * g.ly, tl = zl * g.lz;
  const size_t tbase = tl * t;
  const size_t itf = (t + 1 == g.lt) ? 0 : tbase + tl;          // plane offsets of t + 1 and t - 1
  const size_t itb = (t == 0) ? tl * (g.lt - 1) : tbase - tl;
  const bool flipf = (g.t_bc < 0) && (t + 1 == g.lt);
  const bool flipb = (g.t_bc < 0) && (t == 0);
  const int ybk = y == 0 ? g.ly - 1 : y - 1;
  const char* gf = a.gauge + (size_t)(a.p * 4) * a.link_stride;        // U_mu(x), parity p
  const char* gb = a.gauge + (size_t)((1 - a.p) * 4) * a.link_stride;  // U_mu(x - mu), parity 1-p
  const size_t ls = a.link_stride;

  cx<T> nxt[12], nx2[12], hnx[12], zb[6];
  {
    const int zm = z0 == 0 ? g.lz - 1 : z0 - 1;
    cx<T> sp[12];
    IO<P>::load_spinor(a.in, xh + yl * y + zl * zm + tbase, sp);
    project<2, false>(sp, zb);
  }
  IO<P>::load_spinor(a.in, xh + yl * y + zl * z0 + tbase, nxt);
  {
    const int z1 = z0 + 1 == g.lz ? 0 : z0 + 1;
    IO<P>::load_spinor(a.in, xh + yl * y + zl * z1 + tbase, nx2);
  }
  if (halo) IO<P>::load_spinor(a.in, xh + yl * yh + zl * z0 + tbase, hnx);
  double red[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < zc; ++s) {
    const int z = z0 + s;
    const int zf = z + 1 == g.lz ? 0 : z + 1;
    const int zbk = z == 0 ? g.lz - 1 : z - 1;
    __syncthreads();  // every lane has read the previous plane
    LW::put(L, ns, slot, nxt);
    if (halo) LW::put(L, ns, hslot, hnx);
    __syncthreads();
    const size_t row = yl * y + zl * z + tbase;
    const size_t i = row + xh;
#pragma unroll
    for (int k = 0; k < 12; ++k) nxt[k] = nx2[k];  // plane z + 1: z-forward neighbour, next LDS entry
    if (s + 1 < zc) {
      const int zf2 = zf + 1 == g.lz ? 0 : zf + 1;
      IO<P>::load_spinor(a.in, xh + yl * y + zl * zf2 + tbase, nx2);  // plane z + 2, one step ahead
    }
    if (halo && s + 1 < zc) IO<P>::load_spinor(a.in, xh + yl * yh + zl * zf + tbase, hnx);
    const int x = 2 * xh + ((y + z + t + a.p) & 1);
    const int xf = (x + 1 == g.lx) ? 0 : x + 1;
    const int xb = (x == 0) ? g.lx - 1 : x - 1;
    cx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
    cx<T> sp[12], h[6];
    LW::get(L, ns, lr * lxh + (xf >> 1), sp);
    project<0, true>(sp, h);
    hop_half<P, 0, true>(h, gf + 0 * ls, i, acc);
    LW::get(L, ns, lr * lxh + (xb >> 1), sp);
    project<0, false>(sp, h);
    hop_half<P, 0, false>(h, gb + 0 * ls, row + (xb >> 1), acc);
    LW::get(L, ns, lyf * lxh + xh, sp);
    project<1, true>(sp, h);
    hop_half<P, 1, true>(h, gf + 1 * ls, i, acc);
    LW::get(L, ns, lyb * lxh + xh, sp);
    project<1, false>(sp, h);
    hop_half<P, 1, false>(h, gb + 1 * ls, xh + yl * ybk + zl * z + tbase, acc);
    project<2, true>(nxt, h);
    hop_half<P, 2, true>(h, gf + 2 * ls, i, acc);
    hop_half<P, 2, false>(zb, gb + 2 * ls, xh + yl * y + zl * zbk + tbase, acc);
    {
      cx<T> hf[6];
      const size_t jf = xh + yl * y + zl * z + itf, jb = xh + yl * y + zl * z + itb;
      IO<P>::load_half(a.in, jf, false, hf);
      const T twof = flipf ? T(-2) : T(2);
#pragma unroll
      for (int k = 0; k < 6; ++k) h[k] = twof * hf[k];
      hop_half<P, 3, true>(h, gf + 3 * ls, i, acc);
      IO<P>::load_half(a.in, jb, true, hf);
      const T twob = flipb ? T(-2) : T(2);
#pragma unroll
      for (int k = 0; k < 6; ++k) h[k] = twob * hf[k];
      hop_half<P, 3, false>(h, gb + 3 * ls, jb, acc);
    }
    // (1 + gamma_z) of this plane's own input: the z-backward neighbour of the next plane
    LW::get(L, ns, slot, sp);
    project<2, false>(sp, zb);
    cx<T> out[12];
    hop_epilogue<P, EPI, CLOV, RED>(a, i, acc, out, red);
    IO<P>::store_spinor(a.out, i, out);
  }
  if constexpr (NR > 0) {
    if (blockDim.x % 64 == 0) {
      block_reduce<NR>(red, a.partials + (size_t)blockIdx.x * NR);
    } else {  // partial wavefront (small lattices): through the LDS plane, summed in lane order
      double* R = reinterpret_cast<double*>(lds_raw);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NR; ++k) R[k * blockDim.x + threadIdx.x] = red[k];
      __syncthreads();
      if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          double acc = 0.0;
          for (unsigned j = 0; j < blockDim.x; ++j) acc += R[k * blockDim.x + j];
          a.partials[(size_t)blockIdx.x * NR + k] = acc;
        }
      }
    }
  }
}

// LDS bytes of one plane tile of the march kernel.
size_t march_lds_bytes(const Geom& g, int prec, int ty) {
  const int rows = ty == g.ly ? ty : ty + 2;
  return (size_t)rows * g.lxh * (prec == 0 ? 192 : 96);
}

template <int P>
__global__ void __launch_bounds__(256) k_site(const void* clov, const void* in, void* out, size_t vh) {
  using T = typename IO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vh) return;
  cx<T> s[12], o[12];
  IO<P>::load_spinor(in, i, s);
  if (clov) {
    clover_apply<P>(clov, i, s, o);
    IO<P>::store_spinor(out, i, o);
  } else {
    IO<P>::store_spinor(out, i, s);
  }
}

bool march_shape_ok(const Geom& g, int prec, int block, int zc) {
  if (block < 1 || block > 512 || block % g.lxh != 0) return false;
  const int ty = block / g.lxh;
  if (g.ly % ty != 0 || (ty < g.ly && ty < 2)) return false;
  if (zc < 1 || g.lz % zc != 0) return false;
  if (block * zc < 16) return false;  // at most V/32 blocks: the per-block partials buffers hold V/32 + 8
  return march_lds_bytes(g, prec, ty) <= 158 * 1024;  // with the reduction scratch, within gfx950's 160 KiB
}

int hop_blocks(lqcd_ctx* c, int prec) {
  if (c->hop_split[prec] == 0) {  // plane march: block = Lx/2 x rows lanes, hop_remap = z planes per block
    const int ty = c->hop_block[prec] / c->g.lxh;
    return (c->g.ly / ty) * (c->g.lz / c->hop_remap[prec]) * c->g.lt;
  }
  const int sites = c->hop_block[prec] / c->hop_split[prec];
  if (c->hop_remap[prec] == 2) {
    const int slab = c->g.vh / 8;  // sites of one XCD slab
    return 8 * ((slab + sites - 1) / sites);
  }
  return (c->g.vh + sites - 1) / sites;
}

template <int P, int EPI, bool CLOV, int RED>
static void launch_t(const HopArgs& a, int nb, int bs, hipStream_t s, bool nt, int split) {
  if (split == 0) {
    const int ty = bs / a.g.lxh;
    const size_t lds = march_lds_bytes(a.g, P, ty);
    HopArgs am = a;
    am.remap = 1;
    if (ty == a.g.ly) hipLaunchKernelGGL((k_hopz<P, EPI, CLOV, RED, true>), dim3(nb), dim3(bs), lds, s, am, ty, a.hz);
    else hipLaunchKernelGGL((k_hopz<P, EPI, CLOV, RED, false>), dim3(nb), dim3(bs), lds, s, am, ty, a.hz);
  } else if (split == 4) {
    if (nt) hipLaunchKernelGGL((k_hop4<P, EPI, CLOV, RED, true>), dim3(nb), dim3(bs), 0, s, a);
    else hipLaunchKernelGGL((k_hop4<P, EPI, CLOV, RED, false>), dim3(nb), dim3(bs), 0, s, a);
  } else if (split == 2) {
    if (nt) hipLaunchKernelGGL((k_hop2<P, EPI, CLOV, RED, true>), dim3(nb), dim3(bs), 0, s, a);
    else hipLaunchKernelGGL((k_hop2<P, EPI, CLOV, RED, false>), dim3(nb), dim3(bs), 0, s, a);
  } else {
    if (nt) hipLaunchKernelGGL((k_hop<P, EPI, CLOV, RED, true>), dim3(nb), dim3(bs), 0, s, a);
    else hipLaunchKernelGGL((k_hop<P, EPI, CLOV, RED, false>), dim3(nb), dim3(bs), 0, s, a);
  }
}

template <int P>
static int dispatch(lqcd_ctx* c, const HopCall& h, HopArgs& a, int nb, int bs) {
  const bool cl = h.clov != nullptr;
  const bool nt = c->hop_nt[h.prec] != 0;
  const int split = c->hop_split[h.prec];
  hipStream_t s = c->stream;
  if (h.epi == EPI_SCALE && h.red == RED_NONE) {
    launch_t<P, EPI_SCALE, false, RED_NONE>(a, nb, bs, s, nt, split);
  } else if (h.epi == EPI_SCALE && h.red == RED_DOT) {
    launch_t<P, EPI_SCALE, false, RED_DOT>(a, nb, bs, s, nt, split);
  } else if (h.epi == EPI_SCALE_CLOV && h.red == RED_NONE) {
    if (cl) launch_t<P, EPI_SCALE_CLOV, true, RED_NONE>(a, nb, bs, s, nt, split);
    else launch_t<P, EPI_SCALE, false, RED_NONE>(a, nb, bs, s, nt, split);
  } else if (h.epi == EPI_XPAY) {
    if (h.red == RED_NONE) {
      if (cl) launch_t<P, EPI_XPAY, true, RED_NONE>(a, nb, bs, s, nt, split);
      else launch_t<P, EPI_XPAY, false, RED_NONE>(a, nb, bs, s, nt, split);
    } else if (h.red == RED_DOT) {
      if (cl) launch_t<P, EPI_XPAY, true, RED_DOT>(a, nb, bs, s, nt, split);
      else launch_t<P, EPI_XPAY, false, RED_DOT>(a, nb, bs, s, nt, split);
    } else {
      if (cl) launch_t<P, EPI_XPAY, true, RED_TS>(a, nb, bs, s, nt, split);
      else launch_t<P, EPI_XPAY, false, RED_TS>(a, nb, bs, s, nt, split);
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
  const int split = c->hop_split[h.prec];
  if (split == 0) {
    if (!march_shape_ok(c->g, h.prec, bs, c->hop_remap[h.prec])) return set_error(LQCD_EINVAL, "bad plane-march shape");
  } else {
    if (bs % 64 != 0 || bs < 64 || bs > 256) return set_error(LQCD_EINVAL, "hop block size must be 64..256, multiple of 64");
    if (split != 1 && split != 2 && split != 4) return set_error(LQCD_EINVAL, "bad hop split");
  }
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
  a.hz = c->g.lz / 8;
  if (split == 0) {
    a.hz = c->hop_remap[h.prec];  // z planes per block of the plane march
  } else if (a.remap == 2 && (c->g.lz % 8 != 0)) {
    return set_error(LQCD_EINVAL, "XCD z-slabs need Lz divisible by 8");
  }
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
