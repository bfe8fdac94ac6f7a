// Domain-wall fermions, Moebius form (the operator kind the paper lists and
// benchmarks for Bridge++, Sec. 2-3; Shamir is b5 = 1, c5 = 0):
//   D = D_W (b5 + c5 S) + (1 - S),  D_W = (4 - M5) - 1/2 H on every slice,
//   (S psi)_s = P_- psi_{s+1} + P_+ psi_{s-1},  P_+- = (1 +- gamma5)/2,
//   psi_{Ls} -> -m_f psi_0, psi_{-1} -> -m_f psi_{Ls-1},
// H the Wilson hopping term of hopcore.h, and
//   D^dag = (b5 + c5 S^dag) D_W^dag + (1 - S^dag),  D_W^dag = gamma5 D_W gamma5,
// S^dag with the projectors exchanged. Solved by CG on the normal equations
// D^dag D x = D^dag b in FP64, or through the even-odd Schur complement by CG
// on its normal equations, in FP64 or as FP32 inner solves under FP64 defect
// correction.
//
// The fifth coordinate is an inner degree of freedom of the 4-d site (the
// paper, Sec. 2, reports this beating a construction from the 4-d Wilson
// operator): a 5-d field is two parity halves, each a site-blocked field over
// the 5-d index j = i Ls + s (i the 4-d checkerboard index), the even half
// first. One lane computes one 5-d site: the Ls lanes of a 4-d site load the
// same links (one cache line serves them all) and spinors at consecutive j, and
// the s-hops come from the neighbouring lanes through LDS. A launch covers
// both parities. The workgroups walk the lattice in an XCD-aware order
// (dwf_site, dwf_walk): each XCD takes a range of x columns, y rows or z
// planes in every slice and walks it so that the neighbours of the sites in
// flight were read shortly before by the same XCD and may still be in its L2.
//
// Kernels per application: D with c5 = 0 (b5 folded into the diagonal and the
// hop scale) and D^dag are one kernel each; D with c5 != 0 first forms
// phi = (b5 + c5 S) psi (k_dwf_phi), then the hop of phi in k_dwf.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "dwf.h"
#include "hopcore.h"
#include "internal.h"

namespace lq {
namespace {

constexpr int DWB = 256;  // largest workgroup; a workgroup holds whole 4-d sites (a multiple of Ls lanes)

struct DwfArgs {
  const char* gauge;
  size_t link_stride;
  Geom g;
  const char* in;
  const char* phi;  // Moebius D: (b5 + c5 S) in
  char* out;
  size_t hb;  // bytes of one parity half
  int Ls;
  int spb;   // 5-d sites per workgroup
  int walk;  // 0: linear order; 1: XCD z-slabs of hw planes (lz = 8 hw); 2: XCD y-ranges of hw rows (ly = 8 hw);
             // 3: XCD x-ranges of hw checkerboard columns (lx/2 = 8 hw)
  int hw;
  double d4;         // 4 - M5
  double b5, c5, mf;
  double* norm;      // k_dwf: partial sums of |out|^2, a (0, value) pair per workgroup, or null
  const char* upd;   // k_dwf_phi: in is first replaced in place by upd + upd_beta in (or null)
  double upd_beta;
};

// The 5-d site of this lane, or false past the end. XCD k (the workgroups
// are dealt to the 8 XCDs round-robin) takes
//   walk 1: the slab z in [k hw, (k+1) hw), walked x, y fastest, then z, then
//           t: the z and t neighbours were read one z plane or one slab slice
//           earlier;
//   walk 2: the rows y in [k hw, (k+1) hw), walked x fastest, then those rows,
//           then t, then z: the t neighbours were read one step earlier and the
//           z neighbours lt steps earlier, a working set of lt + 1 slices of
//           lx/2 x hw sites (the neighbours of the two edge rows come from the
//           other XCDs' ranges);
//   walk 3: the checkerboard columns xh in [k hw, (k+1) hw), walked those
//           columns fastest, then t, then z, then y: the t and z neighbours were
//           read hw and hw lt sites earlier and the y neighbours one y step
//           (hw lt lz sites) earlier, so the span between the first and the last
//           read of a spinor is two y steps (2 hw lt lz sites, about 5.5 MB of
//           FP64 traffic through the XCD's L2 at 64x32x16x8 x 8, against 11 MB
//           for the z neighbours of walk 2); only the x neighbours of the two
//           edge columns come from other XCDs (a quarter of a spinor per site
//           at hw = 4, against half of one for the y edges of walk 2).
// All Ls lanes of a 4-d site are in one workgroup in every walk.
__device__ inline bool dwf_site(const DwfArgs& a, size_t& j) {
  const Geom& g = a.g;
  if (threadIdx.x >= a.spb) return false;
  if (a.walk == 0) {
    j = (size_t)blockIdx.x * a.spb + threadIdx.x;
    return j < (size_t)g.vh * a.Ls;
  }
  const int k = blockIdx.x & 7;
  const size_t q = (size_t)(blockIdx.x >> 3) * a.spb + threadIdx.x;
  const size_t q4 = q / a.Ls, s = q - q4 * a.Ls;
  if (a.walk == 1) {
    const size_t xy = (size_t)g.lxh * g.ly;
    if (q4 >= xy * a.hw * g.lt) return false;
    const size_t xyi = q4 % xy, rest = q4 / xy;
    const size_t zin = rest % a.hw, t = rest / a.hw;
    j = (xyi + xy * ((size_t)k * a.hw + zin + (size_t)g.lz * t)) * a.Ls + s;
    return true;
  }
  if (a.walk == 3) {
    if (q4 >= (size_t)a.hw * g.lt * g.lz * g.ly) return false;
    const size_t xin = q4 % a.hw;
    size_t rest = q4 / a.hw;
    const size_t t = rest % g.lt;
    rest /= g.lt;
    const size_t z = rest % g.lz, y = rest / g.lz;
    j = ((size_t)k * a.hw + xin + (size_t)g.lxh * (y + (size_t)g.ly * (z + (size_t)g.lz * t))) * a.Ls + s;
    return true;
  }
  const size_t rows = (size_t)g.lxh * a.hw;
  if (q4 >= rows * g.lt * g.lz) return false;
  const size_t xr = q4 % rows, rest = q4 / rows;
  const size_t t = rest % g.lt, z = rest / g.lt;
  const size_t xin = xr % g.lxh, yin = xr / g.lxh;
  j = (xin + (size_t)g.lxh * ((size_t)k * a.hw + yin + (size_t)g.ly * (z + (size_t)g.lz * t))) * a.Ls + s;
  return true;
}

// The walk of a lattice: LQCD_DWF_WALK (0 linear, 1 z-slabs, 2 y-ranges,
// 3 x-ranges) where it fits the lattice, else x-ranges for FP64 fields where
// lx/2 is a multiple of 8, else y-ranges where ly is, else z-slabs where lz
// is, else linear; returns the grid's workgroup count for n 5-d sites of one
// parity. The x-ranges cut the FP64 spinor re-reads (each XCD keeps whole
// rows of its columns' neighbours); in FP32 a cache line of a link component
// spans 32 checkerboard sites of a row, so columns of lx/16 sites would fetch
// every link line on several XCDs, and the y-ranges are kept.
unsigned dwf_walk(const Geom& g, DwfArgs& a, size_t n, int prec) {
  const bool x_ok = g.lxh % 8 == 0, y_ok = g.ly % 8 == 0, z_ok = g.lz % 8 == 0;
  int w = (prec == 0 && x_ok) ? 3 : (y_ok ? 2 : (z_ok ? 1 : 0));
  if (const char* env = std::getenv("LQCD_DWF_WALK")) {
    const int f = std::atoi(env);
    if (f == 0 || (f == 1 && z_ok) || (f == 2 && y_ok) || (f == 3 && x_ok)) w = f;
  }
  a.walk = w;
  a.hw = w == 3 ? g.lxh / 8 : (w == 2 ? g.ly / 8 : (w == 1 ? g.lz / 8 : 0));
  return w ? 8u * (unsigned)((n / 8 + a.spb - 1) / a.spb) : (unsigned)((n + a.spb - 1) / a.spb);
}

// The s-neighbours of a lane: P_+ and P_- of every lane's field x go to LDS
// (as their upper spin pairs: P_+ x = (pp, -pp), P_- x = (pm, pm)); after the
// barrier the lane reads those of s + 1 and s - 1 (the walls wrap inside the
// 4-d site's Ls lanes) with the wall factors.
template <typename T>
struct SNeighbours {
  cx<T> (*lp)[DWB];
  cx<T> (*lm)[DWB];
  int up, dn;
  T wu, wd;
};

template <typename T>
__device__ inline void put_halves(cx<T> (*lp)[DWB], cx<T> (*lm)[DWB], const cx<T> x[12]) {
  const T half = T(0.5);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    lp[k][threadIdx.x] = half * (x[k] - x[6 + k]);
    lm[k][threadIdx.x] = half * (x[k] + x[6 + k]);
  }
}

template <typename T>
__device__ inline SNeighbours<T> neighbours(cx<T> (*lp)[DWB], cx<T> (*lm)[DWB], int s, int Ls, double mf) {
  SNeighbours<T> n;
  n.lp = lp;
  n.lm = lm;
  const int base = (int)threadIdx.x - s;
  n.up = base + (s + 1 < Ls ? s + 1 : 0);
  n.dn = base + (s > 0 ? s - 1 : Ls - 1);
  n.wu = s + 1 < Ls ? T(1) : T(-mf);
  n.wd = s > 0 ? T(1) : T(-mf);
  return n;
}

// o += f S x (DAG: S^dag x)
template <bool DAG, typename T>
__device__ inline void add_s(const SNeighbours<T>& n, T f, cx<T> o[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    // S x = P_- x_{s+1} + P_+ x_{s-1};  S^dag x = P_+ x_{s+1} + P_- x_{s-1}
    const cx<T> a = (f * n.wu) * (DAG ? n.lp[k][n.up] : n.lm[k][n.up]);
    const cx<T> b = (f * n.wd) * (DAG ? n.lm[k][n.dn] : n.lp[k][n.dn]);
    o[k] = o[k] + a + b;
    o[6 + k] = DAG ? o[6 + k] - a + b : o[6 + k] + a - b;
  }
}

// H (DAG: gamma5 H gamma5) of the other parity of f5 at this lane's 5-d site
template <int P, bool DAG>
__device__ inline void dwf_hop(const DwfArgs& a, const char* f5, int p, int i, int s, cx<typename IO<P>::T> acc[12]) {
  const Geom& g = a.g;
  const int Ls = a.Ls;
  const char* other = f5 + (size_t)(1 - p) * a.hb;
  const int xh = i % g.lxh;
  int r = i / g.lxh;
  const int y = r % g.ly;
  r /= g.ly;
  const int z = r % g.lz;
  const int t = r / g.lz;
  const int x = 2 * xh + ((y + z + t + p) & 1);
  const int row = i - xh;
  const int xf = (x + 1 == g.lx) ? 0 : x + 1;
  const int xb = (x == 0) ? g.lx - 1 : x - 1;
  const int yl = g.lxh, zl = g.lxh * g.ly, tl = g.lxh * g.ly * g.lz;
  const int ixf = row + (xf >> 1), ixb = row + (xb >> 1);
  const int iyf = i + ((y + 1 == g.ly) ? -(g.ly - 1) * yl : yl);
  const int iyb = i + ((y == 0) ? (g.ly - 1) * yl : -yl);
  const int izf = i + ((z + 1 == g.lz) ? -(g.lz - 1) * zl : zl);
  const int izb = i + ((z == 0) ? (g.lz - 1) * zl : -zl);
  const int itf = i + ((t + 1 == g.lt) ? -(g.lt - 1) * tl : tl);
  const int itb = i + ((t == 0) ? (g.lt - 1) * tl : -tl);
  const bool flipf = (g.t_bc < 0) && (t + 1 == g.lt);
  const bool flipb = (g.t_bc < 0) && (t == 0);
  const char* gf = a.gauge + (size_t)(p * 4) * a.link_stride;
  const char* gb = a.gauge + (size_t)((1 - p) * 4) * a.link_stride;
  const size_t ls = a.link_stride, vh = (size_t)g.vh;
  auto at = [&](int site) { return (size_t)site * Ls + s; };
  hop_dir<P, 0, true, false, DAG>(other, gf + 0 * ls, vh, at(ixf), (size_t)i, false, acc);
  hop_dir<P, 0, false, false, DAG>(other, gb + 0 * ls, vh, at(ixb), (size_t)ixb, false, acc);
  hop_dir<P, 1, true, false, DAG>(other, gf + 1 * ls, vh, at(iyf), (size_t)i, false, acc);
  hop_dir<P, 1, false, false, DAG>(other, gb + 1 * ls, vh, at(iyb), (size_t)iyb, false, acc);
  hop_dir<P, 2, true, false, DAG>(other, gf + 2 * ls, vh, at(izf), (size_t)i, false, acc);
  hop_dir<P, 2, false, false, DAG>(other, gb + 2 * ls, vh, at(izb), (size_t)izb, false, acc);
  hop_dir<P, 3, true, false, DAG>(other, gf + 3 * ls, vh, at(itf), (size_t)i, flipf, acc);
  hop_dir<P, 3, false, false, DAG>(other, gb + 3 * ls, vh, at(itb), (size_t)itb, flipb, acc);
  if (DAG) {  // gamma5 on the hop of gamma5 psi
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const cx<typename IO<P>::T> u = acc[k];
      acc[k] = typename IO<P>::T(-1) * acc[6 + k];
      acc[6 + k] = typename IO<P>::T(-1) * u;
    }
  }
}

// D (DAG false) or D^dag (DAG true) at every 5-d site. MOB (D only, c5 != 0):
// the hop acts on phi = (b5 + c5 S) psi, precomputed.
//   D, c5 = 0:  out = (b5 d4 + 1) psi - b5/2 H psi - S psi
//   D, MOB:     out = d4 phi - 1/2 H phi + psi - S psi
//   D^dag:      u = d4 psi - 1/2 gamma5 H gamma5 psi,
//               out = b5 u + psi + S^dag (c5 u - psi)
template <int P, bool DAG, bool MOB>
__global__ void __launch_bounds__(DWB) k_dwf(DwfArgs a) {
  using T = typename IO<P>::T;
  __shared__ cx<T> lp[6][DWB], lm[6][DWB];
  const int p = blockIdx.y, Ls = a.Ls;
  size_t j = 0;
  const bool live = dwf_site(a, j);
  const int i = live ? (int)(j / Ls) : 0;
  const int s = live ? (int)(j - (size_t)i * Ls) : 0;
  const char* own = a.in + (size_t)p * a.hb;

  cx<T> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
  if (live) dwf_hop<P, DAG>(a, MOB ? a.phi : a.in, p, i, s, acc);
  cx<T> v[12];
  if (live) {
    IO<P>::load_spinor(own, j, v);
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = {T(0), T(0)};
  }
  const T d4 = (T)a.d4, half = T(-0.5);
  if (DAG) {
    const T c5 = (T)a.c5;
    cx<T> w[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      acc[k] = d4 * v[k] + half * acc[k];  // u
      w[k] = c5 * acc[k] - v[k];
    }
    put_halves(lp, lm, w);
  } else {
    put_halves(lp, lm, v);
  }
  __syncthreads();
  cx<T> o[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) o[k] = {T(0), T(0)};
  if (live) {
    const SNeighbours<T> nb = neighbours(lp, lm, s, Ls, a.mf);
    if (DAG) {
      const T b5 = (T)a.b5;
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = b5 * acc[k] + v[k];
      add_s<true>(nb, T(1), o);
    } else if (MOB) {
      cx<T> f[12];
      IO<P>::load_spinor(a.phi + (size_t)p * a.hb, j, f);
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = d4 * f[k] + half * acc[k] + v[k];
      add_s<false>(nb, T(-1), o);
    } else {
      const T b5 = (T)a.b5, dg = b5 * d4 + T(1), sc = half * b5;
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = dg * v[k] + sc * acc[k];
      add_s<false>(nb, T(-1), o);
    }
    IO<P>::store_spinor(a.out + (size_t)p * a.hb, j, o);
  }
  if (a.norm) {  // uniform over the launch: the workgroup's partial |out|^2, slot 1 of its pair
    double nv[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 12; ++k) nv[1] += (double)o[k].r * (double)o[k].r + (double)o[k].i * (double)o[k].i;
    block_reduce<2>(nv, a.norm + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2);
  }
}

// out = (b5 + c5 S) in, every 5-d site; with a.upd, in is first replaced at
// this lane's site by upd + upd_beta in and stored back (a CG search-direction
// update fused into the operator, whose later kernel reads in at its own site)
template <int P>
__global__ void __launch_bounds__(DWB) k_dwf_phi(DwfArgs a) {
  using T = typename IO<P>::T;
  __shared__ cx<T> lp[6][DWB], lm[6][DWB];
  const int p = blockIdx.y;
  size_t j = 0;
  const bool live = dwf_site(a, j);
  const int s = live ? (int)(j % (size_t)a.Ls) : 0;
  cx<T> v[12];
  if (live) {
    IO<P>::load_spinor(a.in + (size_t)p * a.hb, j, v);
    if (a.upd) {
      cx<T> rv[12];
      IO<P>::load_spinor(a.upd + (size_t)p * a.hb, j, rv);
      const T bt = (T)a.upd_beta;
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = rv[k] + bt * v[k];
      IO<P>::store_spinor(const_cast<char*>(a.in) + (size_t)p * a.hb, j, v);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = {T(0), T(0)};
  }
  put_halves(lp, lm, v);
  __syncthreads();
  if (!live) return;
  const SNeighbours<T> nb = neighbours(lp, lm, s, a.Ls, a.mf);
  const T b5 = (T)a.b5;
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = b5 * v[k];
  add_s<false>(nb, (T)a.c5, v);
  IO<P>::store_spinor(a.out + (size_t)p * a.hb, j, v);
}

// ---------------------------------------------------------------- even-odd form
// D = M5op + Dhop with the site-local M5op = (4 - M5)(b5 + c5 S) + 1 - S and
// Dhop = -1/2 H (b5 + c5 S). Every site-local operator here has the form
// A_+ (x) P_+ + A_- (x) P_-, A_+- real Ls x Ls matrices over s (S: A_+ the
// lower shift with -m_f in the corner, A_- the upper shift with -m_f in the
// corner; adjoints are transposes).

// out_s = sum_s' (A_+ P_+ x + A_- P_- x)_s' [+ (C_+ P_+ y + C_- P_- y)_s'] on the
// parity-p half of 5-d fields; mats = {A_+, A_-, C_+, C_-}, each Ls x Ls row-major.
// With r5 (x part only), x is first replaced by r + beta x at this lane's site
// and stored back (a CG search-direction update fused into the operator).
template <int P>
__global__ void __launch_bounds__(DWB) k_dwf_sop(DwfArgs a, int p, const char* x5, const char* y5,
                                                 const double* mats, const char* r5, double beta) {
  using T = typename IO<P>::T;
  __shared__ cx<T> lp[6][DWB], lm[6][DWB];
  const int Ls = a.Ls;
  size_t j = 0;
  const bool live = dwf_site(a, j);
  const int s = live ? (int)(j % (size_t)Ls) : 0;
  const int base = (int)threadIdx.x - s;
  cx<T> o[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) o[k] = {T(0), T(0)};
  for (int pass = 0; pass < 2; ++pass) {
    const char* f = pass == 0 ? x5 : y5;
    if (!f) break;
    const double* Ap = mats + (size_t)(2 * pass) * Ls * Ls + (size_t)s * Ls;
    const double* Am = Ap + (size_t)Ls * Ls;
    cx<T> v[12];
    if (live) {
      IO<P>::load_spinor(f + (size_t)p * a.hb, j, v);
      if (pass == 0 && r5) {
        cx<T> rv[12];
        IO<P>::load_spinor(r5 + (size_t)p * a.hb, j, rv);
        const T bt = (T)beta;
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = rv[k] + bt * v[k];
        IO<P>::store_spinor(const_cast<char*>(f) + (size_t)p * a.hb, j, v);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = {T(0), T(0)};
    }
    if (pass == 1) __syncthreads();  // the x pass has read its halves
    put_halves(lp, lm, v);
    __syncthreads();
    if (live) {
      for (int t = 0; t < Ls; ++t) {
        const T cp = (T)Ap[t], cm = (T)Am[t];
        if (cp == T(0) && cm == T(0)) continue;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const cx<T> up = cp * lp[k][base + t], um = cm * lm[k][base + t];
          o[k] = o[k] + up + um;
          o[6 + k] = o[6 + k] - up + um;
        }
      }
    }
  }
  if (live) IO<P>::store_spinor(a.out + (size_t)p * a.hb, j, o);
}

// The one-parity hop followed by site-local operators in one pass: y = scale
// H in (DAG: scale gamma5 H gamma5 in) at this lane's 5-d site, then
// out_s = sum_s' (X_+ P_+ x + X_- P_- x)_s' + (Y_+ P_+ y + Y_- P_- y)_s' on
// the parity-p half, the x part only when mx is given (x read from memory at
// the own 4-d site), the y part from the lanes' registers through LDS, so the
// hop result never goes to memory. mx, my: pairs of Ls x Ls row-major real
// matrices (A_+, A_-) as k_dwf_sop takes them. With norm_partials, the
// workgroup's partial sum of |out|^2 goes to slot 1 of its pair (slot 0 = 0).
template <int P, bool DAG>
__global__ void __launch_bounds__(DWB) k_dwf_hopsop(DwfArgs a, int p, double scale, const char* x5,
                                                    const double* mx, const double* my, double* norm_partials) {
  using T = typename IO<P>::T;
  __shared__ cx<T> lp[6][DWB], lm[6][DWB];
  const int Ls = a.Ls;
  size_t j = 0;
  const bool live = dwf_site(a, j);
  const int i = live ? (int)(j / Ls) : 0;
  const int s = live ? (int)(j - (size_t)i * Ls) : 0;
  const int base = (int)threadIdx.x - s;
  cx<T> y[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) y[k] = {T(0), T(0)};
  if (live) {
    dwf_hop<P, DAG>(a, a.in, p, i, s, y);
    const T sc = (T)scale;
#pragma unroll
    for (int k = 0; k < 12; ++k) y[k] = sc * y[k];
  }
  cx<T> o[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) o[k] = {T(0), T(0)};
  for (int pass = 0; pass < 2; ++pass) {
    const double* M = pass == 0 ? mx : my;
    if (!M) continue;  // uniform over the launch
    cx<T> v[12];
    if (pass == 1) {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = y[k];
      if (mx) __syncthreads();  // the x pass has read its halves
    } else if (live) {
      IO<P>::load_spinor(x5 + (size_t)p * a.hb, j, v);
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = {T(0), T(0)};
    }
    put_halves(lp, lm, v);
    __syncthreads();
    if (live) {
      const double* Ap = M + (size_t)s * Ls;
      const double* Am = Ap + (size_t)Ls * Ls;
      for (int t = 0; t < Ls; ++t) {
        const T cp = (T)Ap[t], cm = (T)Am[t];
        if (cp == T(0) && cm == T(0)) continue;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const cx<T> up = cp * lp[k][base + t], um = cm * lm[k][base + t];
          o[k] = o[k] + up + um;
          o[6 + k] = o[6 + k] - up + um;
        }
      }
    }
  }
  if (live) IO<P>::store_spinor(a.out + (size_t)p * a.hb, j, o);
  if (norm_partials) {  // uniform over the launch
    double v[2] = {0.0, 0.0};
    if (live) {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[1] += (double)o[k].r * (double)o[k].r + (double)o[k].i * (double)o[k].i;
    }
    block_reduce<2>(v, norm_partials + (size_t)blockIdx.x * 2);
  }
}

// canonical [s][t][z][y][x][spin][colour] complex128 <-> native 5-d field
template <int P>
__global__ void __launch_bounds__(256) k_dwf_import(Geom g, int Ls, size_t hb, const double* canon, char* f5) {
  using T = typename IO<P>::T;
  const size_t vol = (size_t)g.vh * 2, q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= vol * Ls) return;
  const size_t s = q / vol, f = q - s * vol;
  const int x = (int)(f % g.lx);
  size_t r = f / g.lx;
  const int y = (int)(r % g.ly);
  r /= g.ly;
  const int z = (int)(r % g.lz), t = (int)(r / g.lz);
  const int p = (x + y + z + t) & 1;
  const double2* src = reinterpret_cast<const double2*>(canon) + 12 * q;
  cx<T> v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double2 e = src[k];
    v[k] = {(T)e.x, (T)e.y};
  }
  IO<P>::store_spinor(f5 + (size_t)p * hb, (f >> 1) * Ls + s, v);
}

template <int P>
__global__ void __launch_bounds__(256) k_dwf_export(Geom g, int Ls, size_t hb, const char* f5, double* canon) {
  using T = typename IO<P>::T;
  const size_t vol = (size_t)g.vh * 2, q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= vol * Ls) return;
  const size_t s = q / vol, f = q - s * vol;
  const int x = (int)(f % g.lx);
  size_t r = f / g.lx;
  const int y = (int)(r % g.ly);
  r /= g.ly;
  const int z = (int)(r % g.lz), t = (int)(r / g.lz);
  const int p = (x + y + z + t) & 1;
  cx<T> v[12];
  IO<P>::load_spinor(f5 + (size_t)p * hb, (f >> 1) * Ls + s, v);
  double2* dst = reinterpret_cast<double2*>(canon) + 12 * q;
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = make_double2((double)v[k].r, (double)v[k].i);
}

// Flat fields of precision P (the 5-d sites in storage order): out = a + cb b
template <int P>
__global__ void __launch_bounds__(256) k_flat_axpy(void* out, const void* a, const void* b, double cb, size_t n) {
  using T = typename IO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cx<T> x[12], y[12];
  IO<P>::load_spinor(a, i, x);
  IO<P>::load_spinor(b, i, y);
  const T c = (T)cb;
#pragma unroll
  for (int k = 0; k < 12; ++k) x[k] = x[k] + c * y[k];
  IO<P>::store_spinor(out, i, x);
}

// The CG update in one pass: x += alpha p, r -= alpha q, and the
// per-workgroup partial sums of |r|^2 in FP64 (slot 1 of each pair, as k_flat_dot)
template <int P>
__global__ void __launch_bounds__(256) k_flat_xr(void* x, const void* p, void* r, const void* q, double alpha,
                                                 double* partials, size_t n) {
  using T = typename IO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (i < n) {
    const T al = (T)alpha, mal = (T)(-alpha);
    cx<T> a[12], b[12];
    IO<P>::load_spinor(x, i, a);
    IO<P>::load_spinor(p, i, b);
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = a[k] + al * b[k];
    IO<P>::store_spinor(x, i, a);
    IO<P>::load_spinor(r, i, a);
    IO<P>::load_spinor(q, i, b);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      a[k] = a[k] + mal * b[k];
      v[1] += (double)a[k].r * (double)a[k].r + (double)a[k].i * (double)a[k].i;
    }
    IO<P>::store_spinor(r, i, a);
  }
  block_reduce<2>(v, partials + (size_t)blockIdx.x * 2);
}

// per-workgroup partial sums of Re <a, b> and <b, b> (FP64 sums)
template <int P>
__global__ void __launch_bounds__(256) k_flat_dot(const void* a, const void* b, double* partials, size_t n) {
  using T = typename IO<P>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (i < n) {
    cx<T> x[12], y[12];
    IO<P>::load_spinor(a, i, x);
    IO<P>::load_spinor(b, i, y);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      v[0] += (double)x[k].r * (double)y[k].r + (double)x[k].i * (double)y[k].i;
      v[1] += (double)y[k].r * (double)y[k].r + (double)y[k].i * (double)y[k].i;
    }
  }
  block_reduce<2>(v, partials + (size_t)blockIdx.x * 2);
}

// FP64 flat field rounded to FP32
__global__ void __launch_bounds__(256) k_flat_down(const void* in64, void* out32, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cx<double> a[12];
  cx<float> b[12];
  IO<0>::load_spinor(in64, i, a);
#pragma unroll
  for (int k = 0; k < 12; ++k) b[k] = {(float)a[k].r, (float)a[k].i};
  IO<1>::store_spinor(out32, i, b);
}

// x (FP64) += e (FP32)
__global__ void __launch_bounds__(256) k_flat_accum_up(void* x64, const void* e32, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cx<double> a[12];
  cx<float> b[12];
  IO<0>::load_spinor(x64, i, a);
  IO<1>::load_spinor(e32, i, b);
#pragma unroll
  for (int k = 0; k < 12; ++k) a[k] = a[k] + cx<double>{(double)b[k].r, (double)b[k].i};
  IO<0>::store_spinor(x64, i, a);
}

size_t half_bytes(int prec, size_t vh, int Ls) { return spinor_bytes(prec, vh * (size_t)Ls); }

}  // namespace

size_t dwf_field_bytes(int prec, size_t vh, int Ls) { return 2 * half_bytes(prec, vh, Ls); }

int dwf_import(lqcd_ctx* c, int prec, int Ls, const double* canon, void* f5) {
  const size_t hb = half_bytes(prec, c->g.vh, Ls), n = (size_t)c->g.vh * 2 * Ls;
  const dim3 grid((unsigned)((n + 255) / 256));
  char* f = reinterpret_cast<char*>(f5);
  if (prec == 0) hipLaunchKernelGGL(k_dwf_import<0>, grid, dim3(256), 0, c->stream, c->g, Ls, hb, canon, f);
  else if (prec == 1) hipLaunchKernelGGL(k_dwf_import<1>, grid, dim3(256), 0, c->stream, c->g, Ls, hb, canon, f);
  else return set_error(LQCD_EINVAL, "domain-wall fields: precision must be F64 or F32");
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int dwf_export(lqcd_ctx* c, int prec, int Ls, const void* f5, double* canon) {
  const size_t hb = half_bytes(prec, c->g.vh, Ls), n = (size_t)c->g.vh * 2 * Ls;
  const dim3 grid((unsigned)((n + 255) / 256));
  const char* f = reinterpret_cast<const char*>(f5);
  if (prec == 0) hipLaunchKernelGGL(k_dwf_export<0>, grid, dim3(256), 0, c->stream, c->g, Ls, hb, f, canon);
  else if (prec == 1) hipLaunchKernelGGL(k_dwf_export<1>, grid, dim3(256), 0, c->stream, c->g, Ls, hb, f, canon);
  else return set_error(LQCD_EINVAL, "domain-wall fields: precision must be F64 or F32");
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

// workgroups of one dwf_apply launch (both parities): the pairs its norm_partials receive
size_t dwf_apply_groups(const Geom& g, int prec, int Ls) {
  DwfArgs a{};
  a.spb = (DWB / Ls) * Ls;
  return 2 * (size_t)dwf_walk(g, a, (size_t)g.vh * Ls, prec);
}

// out = D in (dag = 0) or D^dag in (dag = 1) on native 5-d fields (in != out;
// tmp, a third field, holds phi for D with c5 != 0)
int dwf_apply(lqcd_ctx* c, int prec, const lqcd_dwf_params& d, int dag, const void* in, void* out, void* tmp,
              double* norm_partials, const void* upd, double upd_beta) {
  if (!c->gauge[prec]) return set_error(LQCD_ESTATE, "gauge field not set");
  if (d.Ls < 1 || d.Ls > DWB) return set_error(LQCD_EINVAL, "domain-wall operator: Ls must be in [1, 256]");
  if (prec != 0 && prec != 1) return set_error(LQCD_EINVAL, "domain-wall operator: precision must be F64 or F32");
  const bool mob = !dag && d.c5 != 0.0;
  if (mob && !tmp) return set_error(LQCD_EINVAL, "domain-wall operator: D with c5 != 0 needs a scratch field");
  if (upd && !mob) return set_error(LQCD_EINVAL, "domain-wall operator: a fused update needs D with c5 != 0");
  DwfArgs a{};
  a.gauge = reinterpret_cast<const char*>(c->gauge[prec]);
  a.link_stride = link_bytes(prec, c->g.vh);
  a.g = c->g;
  a.in = reinterpret_cast<const char*>(in);
  a.phi = reinterpret_cast<const char*>(tmp);
  a.out = reinterpret_cast<char*>(out);
  a.hb = half_bytes(prec, c->g.vh, d.Ls);
  a.Ls = d.Ls;
  a.spb = (DWB / d.Ls) * d.Ls;
  a.d4 = 4.0 - d.M5;
  a.b5 = d.b5;
  a.c5 = d.c5;
  a.mf = d.mf;
  const unsigned nb = dwf_walk(c->g, a, (size_t)c->g.vh * d.Ls, prec);
  const dim3 grid(nb, 2), block((a.spb + 63) / 64 * 64);
  a.norm = norm_partials;
  if (mob) {
    DwfArgs f = a;
    f.out = reinterpret_cast<char*>(tmp);
    f.norm = nullptr;
    f.upd = reinterpret_cast<const char*>(upd);
    f.upd_beta = upd_beta;
    if (prec == 0) hipLaunchKernelGGL(k_dwf_phi<0>, grid, block, 0, c->stream, f);
    else hipLaunchKernelGGL(k_dwf_phi<1>, grid, block, 0, c->stream, f);
  }
  if (prec == 0) {
    if (dag) hipLaunchKernelGGL((k_dwf<0, true, false>), grid, block, 0, c->stream, a);
    else if (mob) hipLaunchKernelGGL((k_dwf<0, false, true>), grid, block, 0, c->stream, a);
    else hipLaunchKernelGGL((k_dwf<0, false, false>), grid, block, 0, c->stream, a);
  } else {
    if (dag) hipLaunchKernelGGL((k_dwf<1, true, false>), grid, block, 0, c->stream, a);
    else if (mob) hipLaunchKernelGGL((k_dwf<1, false, true>), grid, block, 0, c->stream, a);
    else hipLaunchKernelGGL((k_dwf<1, false, false>), grid, block, 0, c->stream, a);
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

// The flat vector operations on n 5-d sites of precision prec (0 FP64, 1 FP32)
int axpy(lqcd_ctx* c, size_t n, void* out, const void* a, const void* b, double cb, int prec = 0) {
  const dim3 grid((unsigned)((n + 255) / 256));
  if (prec == 0) hipLaunchKernelGGL(k_flat_axpy<0>, grid, dim3(256), 0, c->stream, out, a, b, cb, n);
  else hipLaunchKernelGGL(k_flat_axpy<1>, grid, dim3(256), 0, c->stream, out, a, b, cb, n);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int sum_partials_host(lqcd_ctx* c, DWork& w, size_t n, double* ab, double* bb);

int dot(lqcd_ctx* c, DWork& w, size_t n, const void* a, const void* b, double* ab, double* bb, int prec = 0) {
  const int nb = (int)((n + 255) / 256);
  if (prec == 0) hipLaunchKernelGGL(k_flat_dot<0>, dim3(nb), dim3(256), 0, c->stream, a, b, w.partials, n);
  else hipLaunchKernelGGL(k_flat_dot<1>, dim3(nb), dim3(256), 0, c->stream, a, b, w.partials, n);
  LQ_HIP(hipGetLastError());
  return sum_partials_host(c, w, n, ab, bb);
}

// x += alpha p, r -= alpha q, *rr = |r|^2 (after the update)
int xr_update(lqcd_ctx* c, DWork& w, size_t n, void* x, const void* p, void* r, const void* q, double alpha,
              double* rr, int prec = 0) {
  const int nb = (int)((n + 255) / 256);
  if (prec == 0) hipLaunchKernelGGL(k_flat_xr<0>, dim3(nb), dim3(256), 0, c->stream, x, p, r, q, alpha, w.partials, n);
  else hipLaunchKernelGGL(k_flat_xr<1>, dim3(nb), dim3(256), 0, c->stream, x, p, r, q, alpha, w.partials, n);
  LQ_HIP(hipGetLastError());
  return sum_partials_host(c, w, n, nullptr, rr);
}

int flat_down(lqcd_ctx* c, size_t n, const void* in64, void* out32) {
  hipLaunchKernelGGL(k_flat_down, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, in64, out32, n);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int flat_accum_up(lqcd_ctx* c, size_t n, void* x64, const void* e32) {
  hipLaunchKernelGGL(k_flat_accum_up, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, x64, e32, n);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

// the sums of the (Re <a, b>, <b, b>) partials of the last reduction, on the host
int sum_partials_host(lqcd_ctx* c, DWork& w, size_t n, double* ab, double* bb) {
  const int nb = (int)((n + 255) / 256);
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
  const size_t bytes = dwf_field_bytes(0, c->g.vh, d.Ls), n = 2 * padded_sites((size_t)c->g.vh * d.Ls);
  void *bn, *r, *p, *q, *t, *ph;
  for (void** f : {&bn, &r, &p, &q, &t, &ph}) LQ_TRY(w.alloc(c, bytes, f));
  // pairs for the flat reductions (one per 256 sites) and for the norm of D p (one per operator workgroup)
  const size_t ngroups = dwf_apply_groups(c->g, 0, d.Ls);
  LQ_HIP(hipMalloc(&w.partials, std::max((size_t)(n + 255) / 256, ngroups) * 2 * sizeof(double)));
  double bb = 0.0;
  LQ_TRY(dot(c, w, n, b, b, nullptr, &bb));
  const double bnorm = std::sqrt(bb);
  st = lqcd_solve_stats{};
  const auto ts = clk::now();
  st.seconds_setup = std::chrono::duration<double>(ts - t0).count();
  LQ_HIP(hipMemsetAsync(x, 0, bytes, c->stream));  // x = 0 (padding included)
  if (bnorm == 0.0) return LQCD_OK;
  LQ_TRY(dwf_apply(c, 0, d, 1, b, bn, ph));  // D^dag b
  double bnn = 0.0;
  LQ_TRY(dot(c, w, n, bn, bn, nullptr, &bnn));
  int iters = 0, passes = 0, status = LQCD_OK;
  double true_rel = 1.0, rr = 0.0;
  double target = 0.1 * prm.tol * std::sqrt(bnn);
  for (;;) {
    // true residual of D x = b, and the normal-equation residual
    LQ_TRY(dwf_apply(c, 0, d, 0, x, q, ph));
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
    LQ_TRY(dwf_apply(c, 0, d, 1, t, r, ph));  // r = D^dag (b - D x)
    LQ_TRY(dot(c, w, n, r, r, nullptr, &rr));
    LQ_TRY(axpy(c, n, p, r, r, 0.0));             // p = r
    const double tgt = std::min(target, 0.5 * std::sqrt(rr));
    // Moebius D forms phi = (b5 + c5 S) p first, at each site from p there:
    // that pass also does the direction update p = r + beta p
    const bool fuse = d.c5 != 0.0;
    double beta = 0.0;
    bool first = true;
    while (iters < prm.max_iter) {
      // t = D p, with the partials of |D p|^2
      LQ_TRY(dwf_apply(c, 0, d, 0, p, t, ph, w.partials, fuse && !first ? r : nullptr, beta));
      LQ_TRY(dwf_apply(c, 0, d, 1, t, q, ph));              // q = D^dag D p
      double pq = 0.0;                                       // <p, D^dag D p> = |D p|^2
      LQ_TRY(sum_partials_host(c, w, ngroups * 256, nullptr, &pq));
      if (!(pq > 0.0)) break;
      const double alpha = rr / pq;
      double rn = 0.0;
      LQ_TRY(xr_update(c, w, n, x, p, r, q, alpha, &rn));
      ++iters;
      if (std::sqrt(rn) <= tgt) {
        rr = rn;
        break;
      }
      beta = rn / rr;
      first = false;
      if (!fuse) LQ_TRY(axpy(c, n, p, r, p, beta));
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

// ---------------------------------------------------------------- even-odd host side
namespace {

// pairs (A_+, A_-) of real Ls x Ls matrices, in this order in the device buffer
enum EoPair { EP_B, EP_BMINV, EP_M5, EP_MINUS_I, EP_BMINV_T, EP_M5_T, EP_MINUS_B_T, EP_MINV, EP_MINUS_MINV, EP_I,
              EP_MINUS_I2, EP_COUNT };

using Mat = std::vector<double>;

Mat matmul(const Mat& a, const Mat& b, int n) {
  Mat c((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j) c[(size_t)i * n + j] += a[(size_t)i * n + k] * b[(size_t)k * n + j];
  return c;
}

Mat transpose(const Mat& a, int n) {
  Mat t((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) t[(size_t)j * n + i] = a[(size_t)i * n + j];
  return t;
}

// Gauss-Jordan with partial pivoting; false if singular
bool invert(Mat a, int n, Mat& inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + col]) > std::fabs(a[(size_t)piv * n + col])) piv = r;
    const double pv = a[(size_t)piv * n + col];
    if (!(std::fabs(pv) > 1e-300)) return false;
    if (piv != col)
      for (int j = 0; j < n; ++j) {
        std::swap(a[(size_t)piv * n + j], a[(size_t)col * n + j]);
        std::swap(inv[(size_t)piv * n + j], inv[(size_t)col * n + j]);
      }
    const double ip = 1.0 / a[(size_t)col * n + col];
    for (int j = 0; j < n; ++j) {
      a[(size_t)col * n + j] *= ip;
      inv[(size_t)col * n + j] *= ip;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = a[(size_t)r * n + col];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[(size_t)r * n + j] -= f * a[(size_t)col * n + j];
        inv[(size_t)r * n + j] -= f * inv[(size_t)col * n + j];
      }
    }
  }
  return true;
}

// the pairs of the even-odd operators, for chirality + (h = 0) and - (h = 1)
int eo_matrices(const lqcd_dwf_params& d, std::vector<double>& out) {
  const int n = d.Ls;
  const size_t nn = (size_t)n * n;
  out.assign((size_t)EP_COUNT * 2 * nn, 0.0);
  for (int h = 0; h < 2; ++h) {
    Mat S(nn, 0.0), I(nn, 0.0);
    for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
    for (int i = 0; i < n; ++i) {
      if (h == 0) {  // P_+ psi_{s-1}, wall -m_f psi_{Ls-1} at s = 0
        if (i > 0) S[(size_t)i * n + i - 1] += 1.0;
        else S[(size_t)i * n + n - 1] += -d.mf;
      } else {       // P_- psi_{s+1}, wall -m_f psi_0 at s = Ls-1
        if (i + 1 < n) S[(size_t)i * n + i + 1] += 1.0;
        else S[(size_t)i * n] += -d.mf;
      }
    }
    Mat B(nn), M(nn), Minv;
    for (size_t k = 0; k < nn; ++k) {
      B[k] = d.b5 * I[k] + d.c5 * S[k];
      M[k] = (4.0 - d.M5) * B[k] + I[k] - S[k];
    }
    if (!invert(M, n, Minv)) return set_error(LQCD_ESINGULAR, "domain-wall even-odd: the site-local part is singular");
    const Mat BM = matmul(B, Minv, n);
    const Mat set[EP_COUNT] = {B, BM, M, I, transpose(BM, n), transpose(M, n), transpose(B, n), Minv, Minv, I, I};
    const double sign[EP_COUNT] = {1, 1, 1, -1, 1, 1, -1, 1, -1, 1, -1};
    for (int e = 0; e < EP_COUNT; ++e)
      for (size_t k = 0; k < nn; ++k) out[((size_t)e * 2 + h) * nn + k] = sign[e] * set[e][k];
  }
  return LQCD_OK;
}

struct EoCtx {
  lqcd_ctx* c;
  int prec;
  lqcd_dwf_params d;
  DwfArgs a;
  dim3 grid, block;
  const double* mats;
  const double* pair(int e) const { return mats + (size_t)e * 2 * d.Ls * d.Ls; }

  // r (optional): x is first replaced in place by r + beta x (x then written)
  int sop(int p, const void* x, const void* y, int e, void* out, const void* r = nullptr, double beta = 0.0) const {
    DwfArgs b = a;
    b.out = reinterpret_cast<char*>(out);
    const char* xs = reinterpret_cast<const char*>(x);
    const char* ys = reinterpret_cast<const char*>(y);
    const char* rs = reinterpret_cast<const char*>(r);
    if (prec == 0) hipLaunchKernelGGL(k_dwf_sop<0>, grid, block, 0, c->stream, b, p, xs, ys, pair(e), rs, beta);
    else hipLaunchKernelGGL(k_dwf_sop<1>, grid, block, 0, c->stream, b, p, xs, ys, pair(e), rs, beta);
    LQ_HIP(hipGetLastError());
    return LQCD_OK;
  }
  // out = scale H in, then the site-local operators of k_dwf_hopsop (x part
  // with pair ex when x is given, y part with pair ey)
  int hopsop(int p, const void* in, const void* x, int ex, int ey, void* out, bool dag,
             double* norm_partials = nullptr) const {
    DwfArgs b = a;
    b.in = reinterpret_cast<const char*>(in);
    b.out = reinterpret_cast<char*>(out);
    const char* xs = reinterpret_cast<const char*>(x);
    const double* mx = x ? pair(ex) : nullptr;
    const double* my = pair(ey);
    if (prec == 0) {
      if (dag) hipLaunchKernelGGL((k_dwf_hopsop<0, true>), grid, block, 0, c->stream, b, p, -0.5, xs, mx, my, norm_partials);
      else hipLaunchKernelGGL((k_dwf_hopsop<0, false>), grid, block, 0, c->stream, b, p, -0.5, xs, mx, my, norm_partials);
    } else {
      if (dag) hipLaunchKernelGGL((k_dwf_hopsop<1, true>), grid, block, 0, c->stream, b, p, -0.5, xs, mx, my, norm_partials);
      else hipLaunchKernelGGL((k_dwf_hopsop<1, false>), grid, block, 0, c->stream, b, p, -0.5, xs, mx, my, norm_partials);
    }
    LQ_HIP(hipGetLastError());
    return LQCD_OK;
  }
  // out_e = S_ee x_e (dag 0) or S_ee^dag x_e (dag 1); tA, tB: scratch 5-d fields.
  // Each hop is fused with the site-local operator after it (k_dwf_hopsop).
  // norm_partials (dag 0 only): the workgroups' partial sums of |out_e|^2, as
  // (0, value) pairs, one pair per workgroup of grid.
  // xr (dag 0 only): x_e is first replaced in place by xr_e + beta x_e, the CG
  // search-direction update, in the first launch.
  int schur(int dag, const void* x, void* out, void* tA, void* tB, double* norm_partials = nullptr,
            const void* xr = nullptr, double beta = 0.0) const {
    if (!dag) {
      LQ_TRY(sop(0, x, nullptr, EP_B, tA, xr, beta));                        // B x
      LQ_TRY(hopsop(1, tA, nullptr, 0, EP_BMINV, tB, false));                // B M5^-1 Dhop_oe x
      return hopsop(0, tB, x, EP_M5, EP_MINUS_I, out, false, norm_partials);  // M5 x - Dhop_eo (that)
    }
    LQ_TRY(hopsop(1, x, nullptr, 0, EP_BMINV_T, tA, true));       // M5^-dag B^dag (-1/2 H^dag_oe x)
    return hopsop(0, tA, x, EP_M5_T, EP_MINUS_B_T, out, true);   // M5^dag x - B^dag (-1/2 H^dag_eo that)
  }
};

int eo_setup(lqcd_ctx* c, int prec, const lqcd_dwf_params& d, const double* mats, EoCtx& e) {
  if (!c->gauge[prec]) return set_error(LQCD_ESTATE, "gauge field not set");
  if (d.Ls < 1 || d.Ls > DWB) return set_error(LQCD_EINVAL, "domain-wall operator: Ls must be in [1, 256]");
  if (prec != 0 && prec != 1) return set_error(LQCD_EINVAL, "domain-wall operator: precision must be F64 or F32");
  e.c = c;
  e.prec = prec;
  e.d = d;
  e.mats = mats;
  DwfArgs& a = e.a;
  a = DwfArgs{};
  a.gauge = reinterpret_cast<const char*>(c->gauge[prec]);
  a.link_stride = link_bytes(prec, c->g.vh);
  a.g = c->g;
  a.hb = half_bytes(prec, c->g.vh, d.Ls);
  a.Ls = d.Ls;
  a.spb = (DWB / d.Ls) * d.Ls;
  a.d4 = 4.0 - d.M5;
  a.b5 = d.b5;
  a.c5 = d.c5;
  a.mf = d.mf;
  e.grid = dim3(dwf_walk(c->g, a, (size_t)c->g.vh * d.Ls, prec));
  e.block = dim3((a.spb + 63) / 64 * 64);
  return LQCD_OK;
}

struct DevMats {
  double* p = nullptr;
  ~DevMats() { (void)hipFree(p); }
  int upload(lqcd_ctx* c, const lqcd_dwf_params& d) {
    std::vector<double> h;
    LQ_TRY(eo_matrices(d, h));
    if (hipMalloc(reinterpret_cast<void**>(&p), h.size() * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(LQCD_ENOMEM, "domain-wall even-odd matrices");
    }
    LQ_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    LQ_HIP(hipStreamSynchronize(c->stream));
    return LQCD_OK;
  }
};

}  // namespace

int dwf_schur_apply(lqcd_ctx* c, int prec, const lqcd_dwf_params& d, int dag, const void* in, void* out, void* tA,
                    void* tB) {
  DevMats m;
  LQ_TRY(m.upload(c, d));
  EoCtx e;
  LQ_TRY(eo_setup(c, prec, d, m.p, e));
  LQ_TRY(e.schur(dag, in, out, tA, tB));
  LQ_HIP(hipStreamSynchronize(c->stream));  // m is freed on return
  return LQCD_OK;
}

int dwf_solve_eo(lqcd_ctx* c, const lqcd_dwf_params& d, const lqcd_solve_params& prm, const void* b, void* x,
                 lqcd_solve_stats& st) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  DevMats m;
  LQ_TRY(m.upload(c, d));
  EoCtx e;
  LQ_TRY(eo_setup(c, 0, d, m.p, e));
  DWork w;
  const size_t bytes = dwf_field_bytes(0, c->g.vh, d.Ls);
  const size_t nh = padded_sites((size_t)c->g.vh * d.Ls), nf = 2 * nh;
  void *bp, *r, *pv, *q, *sx, *tA, *tB, *res;
  for (void** f : {&bp, &r, &pv, &q, &sx, &tA, &tB, &res}) LQ_TRY(w.alloc(c, bytes, f));
  // mixed precision: the inner CG in FP32 on its own operator context and fields
  const bool mixed = prm.inner_prec == LQCD_F32;
  const double delta = prm.inner_tol > 0.0 && prm.inner_tol < 1.0 ? prm.inner_tol : 1e-6;
  EoCtx e32{};
  void *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *sx32 = nullptr, *tA32 = nullptr, *tB32 = nullptr,
       *e32f = nullptr;
  if (mixed) {
    LQ_TRY(eo_setup(c, 1, d, m.p, e32));
    const size_t bytes32 = dwf_field_bytes(1, c->g.vh, d.Ls);
    for (void** f : {&r32, &p32, &q32, &sx32, &tA32, &tB32, &e32f}) LQ_TRY(w.alloc(c, bytes32, f));
  }
  // pairs for the flat reductions (one per 256 sites) and for the norm of S p (one per operator workgroup)
  const size_t npairs = std::max({(size_t)(nf + 255) / 256, (size_t)e.grid.x, mixed ? (size_t)e32.grid.x : 0});
  LQ_HIP(hipMalloc(&w.partials, npairs * 2 * sizeof(double)));
  auto ev = [](void* f) { return f; };  // even half = start of the field
  double bb = 0.0;
  LQ_TRY(dot(c, w, nf, b, b, nullptr, &bb));
  const double bnorm = std::sqrt(bb);
  st = lqcd_solve_stats{};
  const auto ts = clk::now();
  st.seconds_setup = std::chrono::duration<double>(ts - t0).count();
  LQ_HIP(hipMemsetAsync(x, 0, bytes, c->stream));
  if (bnorm == 0.0) return LQCD_OK;
  // b' = b_e - Dhop_eo M5^-1 b_o
  LQ_TRY(e.sop(1, b, nullptr, EP_BMINV, tA));
  LQ_TRY(e.hopsop(0, tA, b, EP_I, EP_MINUS_I2, bp, false));
  LQ_TRY(e.schur(1, bp, sx, tA, tB));  // S^dag b'
  double sbb = 0.0;
  LQ_TRY(dot(c, w, nh, ev(sx), ev(sx), nullptr, &sbb));
  int iters = 0, passes = 0, status = LQCD_OK;
  double true_rel = 1.0, target = 0.1 * prm.tol * std::sqrt(sbb);
  // out_e = S^dag S in_e and *sn = |S in_e|^2 (= <in_e, out_e>, summed by the
  // workgroups of the operator's last launch: no separate dot product pass)
  // With rp, in is first updated in place to rp + beta in (the CG direction
  // update, fused into the operator's first launch).
  auto normal = [&](void* in, void* out, double* sn, const void* rp, double beta) -> int {
    LQ_TRY(e.schur(0, in, sx, tA, tB, w.partials, rp, beta));
    LQ_TRY(e.schur(1, sx, out, tA, tB));
    return sum_partials_host(c, w, (size_t)e.grid.x * 256, nullptr, sn);
  };
  auto normal32 = [&](void* in, void* out, double* sn, const void* rp, double beta) -> int {  // the same in FP32
    LQ_TRY(e32.schur(0, in, sx32, tA32, tB32, w.partials, rp, beta));
    LQ_TRY(e32.schur(1, sx32, out, tA32, tB32));
    return sum_partials_host(c, w, (size_t)e32.grid.x * 256, nullptr, sn);
  };
  for (;;) {
    // x_o from x_e, then the true residual with the full operator
    LQ_TRY(e.sop(0, x, nullptr, EP_B, tA));
    LQ_TRY(e.hopsop(1, tA, b, EP_MINV, EP_MINUS_MINV, x, false));
    LQ_TRY(dwf_apply(c, 0, d, 0, x, q, tA));
    LQ_TRY(axpy(c, nf, res, b, q, -1.0));
    double tt = 0.0;
    LQ_TRY(dot(c, w, nf, res, res, nullptr, &tt));
    true_rel = std::sqrt(tt) / bnorm;
    if (log_level() >= 1)
      std::fprintf(stderr, "[lqcd] domain-wall even-odd CG pass %d: %d iterations, |b - D x|/|b| %.3e\n", passes, iters,
                   true_rel);
    if (true_rel <= prm.tol) break;
    if (!(true_rel == true_rel)) {
      status = set_error(LQCD_EBREAKDOWN, "domain-wall even-odd CG produced NaN");
      break;
    }
    if (iters >= prm.max_iter || passes >= prm.max_outer) {
      status = set_error(LQCD_ENOCONV, "domain-wall even-odd CG did not reach the tolerance");
      break;
    }
    ++passes;
    // r = S^dag (b' - S x_e) on the even half
    LQ_TRY(e.schur(0, x, q, tA, tB));
    LQ_TRY(axpy(c, nh, ev(res), ev(bp), ev(q), -1.0));
    LQ_TRY(e.schur(1, res, r, tA, tB));
    double rr = 0.0;
    LQ_TRY(dot(c, w, nh, ev(r), ev(r), nullptr, &rr));
    if (mixed) {
      // defect correction: S^dag S e = r by CG in FP32 from e = 0 until the
      // iterated residual has dropped by delta (or reached the normal
      // target), then x_e += e in FP64 and the next pass starts from the
      // true residual
      LQ_TRY(flat_down(c, nh, ev(r), ev(r32)));
      LQ_HIP(hipMemsetAsync(e32f, 0, half_bytes(1, c->g.vh, d.Ls), c->stream));
      LQ_TRY(axpy(c, nh, ev(p32), ev(r32), ev(r32), 0.0, 1));
      double rr32 = 0.0;
      LQ_TRY(dot(c, w, nh, ev(r32), ev(r32), nullptr, &rr32, 1));
      const double tgt32 = std::max(delta * std::sqrt(rr32), target);
      double beta = 0.0;
      bool first = true;
      while (iters < prm.max_iter) {
        double pq = 0.0;
        LQ_TRY(normal32(p32, q32, &pq, first ? nullptr : r32, beta));  // p = r + beta p first, after the first
        if (!(pq > 0.0)) break;
        const double alpha = rr32 / pq;
        double rn = 0.0;
        LQ_TRY(xr_update(c, w, nh, ev(e32f), ev(p32), ev(r32), ev(q32), alpha, &rn, 1));
        ++iters;
        if (std::sqrt(rn) <= tgt32) break;
        beta = rn / rr32;
        first = false;
        rr32 = rn;
      }
      LQ_TRY(flat_accum_up(c, nh, ev(x), ev(e32f)));
      target *= 0.5;
      continue;
    }
    LQ_TRY(axpy(c, nh, ev(pv), ev(r), ev(r), 0.0));
    const double tgt = std::min(target, 0.5 * std::sqrt(rr));
    double beta = 0.0;
    bool first = true;
    while (iters < prm.max_iter) {
      double pq = 0.0;
      LQ_TRY(normal(pv, q, &pq, first ? nullptr : r, beta));  // p = r + beta p first, after the first
      if (!(pq > 0.0)) break;
      const double alpha = rr / pq;
      double rn = 0.0;
      LQ_TRY(xr_update(c, w, nh, ev(x), ev(pv), ev(r), ev(q), alpha, &rn));
      ++iters;
      if (std::sqrt(rn) <= tgt) break;
      beta = rn / rr;
      first = false;
      rr = rn;
    }
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
