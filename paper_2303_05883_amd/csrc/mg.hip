// Two-level aggregation multigrid (the paper's headline solver, Sec. 3, in
// the DD-alpha-AMG style): test vectors split by chirality on aggregates span
// the coarse space, D_c = P^dag D P is a nearest-neighbour stencil of
// (2n) x (2n) blocks on the lattice of aggregates, and the preconditioner is a
// coarse-grid correction (FP32 BiCGStab on D_c) followed by SAP smoothing,
// inside the FP64 flexible BiCGStab of sap.hip.
//
// Chirality: the Dirac-Pauli gamma5 mixes the upper (u, spins 0-1) and lower
// (l, spins 2-3) pairs; the chiral components are c_+ = (u - l)/sqrt2 and
// c_- = (u + l)/sqrt2. The basis is stored as n FP32 fields in the spinor
// layout with c_+ in the place of u and c_- in the place of l, so each
// chirality is one half of the spinor's words. Coarse vectors are FP32
// complex, index (a * 2 + chi) * n + k, a = ax + nax (ay + nay (az + naz at)).
//
// D_c is built with 16 aggregate classes (the parities of the aggregate
// coordinates) x 2n columns: for class c and column (chi, k), w = P e with e
// one at (a, chi, k) for every aggregate a of class c, y = D w in FP32, and
// every aggregate projects y: one of class c gives the column of its own
// block, one whose class differs from c in the bit of direction mu gives the
// columns of its +mu and -mu blocks from the sites on its +mu and -mu faces
// (only hops from the neighbour in that direction reach them; aggregate
// extents >= 2 keep the faces apart).
#include <chrono>
#include <cmath>
#include <cstdio>
#include <type_traits>
#include <vector>

#include "blas.h"
#include "fieldio.h"
#include "internal.h"
#include "mg.h"
#include "ops.h"
#include "sap.h"

namespace lq {
namespace {

constexpr int NMAX = 24;  // largest number of test vectors
constexpr float RS2 = 0.70710678118654752f;

struct MgGeom {
  Geom g;
  int a[4];   // aggregate extents
  int na[4];  // aggregates per direction
  int nagg;
  int asz;  // sites per aggregate
  int n;    // test vectors
  size_t hb;  // bytes of one FP32 half field
};

__device__ inline void coords_of(const Geom& g, int p, int i, int& x, int& y, int& z, int& t) {
  const int xh = i % g.lxh;
  int r = i / g.lxh;
  y = r % g.ly;
  r /= g.ly;
  z = r % g.lz;
  t = r / g.lz;
  x = 2 * xh + ((y + z + t + p) & 1);
}

__device__ inline int agg_of(const MgGeom& m, int x, int y, int z, int t) {
  return x / m.a[0] + m.na[0] * (y / m.a[1] + m.na[1] * (z / m.a[2] + m.na[2] * (t / m.a[3])));
}

__device__ inline int class_of(const MgGeom& m, int agg) {
  const int ax = agg % m.na[0];
  int r = agg / m.na[0];
  const int ay = r % m.na[1];
  r /= m.na[1];
  const int az = r % m.na[2], at = r / m.na[2];
  return (ax & 1) | ((ay & 1) << 1) | ((az & 1) << 2) | ((at & 1) << 3);
}

// local site l of aggregate agg -> global coordinates, parity and half index
__device__ inline void agg_site(const MgGeom& m, int agg, int l, int c[4], int& p, int& i) {
  int ac[4];
  int r = agg;
  for (int d = 0; d < 3; ++d) {
    ac[d] = r % m.na[d];
    r /= m.na[d];
  }
  ac[3] = r;
  int q = l;
  for (int d = 0; d < 4; ++d) {
    const int lc = d < 3 ? q % m.a[d] : q;
    if (d < 3) q /= m.a[d];
    c[d] = ac[d] * m.a[d] + lc;
  }
  p = (c[0] + c[1] + c[2] + c[3]) & 1;
  const size_t full = (size_t)c[0] + (size_t)m.g.lx * ((size_t)c[1] + (size_t)m.g.ly * ((size_t)c[2] + (size_t)m.g.lz * c[3]));
  i = (int)(full >> 1);
}

// The aggregate of this workgroup: workgroups are dealt to the 8 XCDs
// round-robin, so with nagg a multiple of 8 XCD k takes the contiguous range
// [k nagg/8, (k+1) nagg/8) in order, and aggregates next to each other in x
// (which share the cache lines of the site-blocked fields) meet in one L2.
__device__ inline int agg_of_block(const MgGeom& m) {
  if (m.nagg % 8 != 0) return blockIdx.x;
  return (blockIdx.x & 7) * (m.nagg >> 3) + (blockIdx.x >> 3);
}

__device__ inline const char* half_of(const void* f2, int p, size_t hb) {
  return reinterpret_cast<const char*>(f2) + (size_t)p * hb;
}
__device__ inline char* half_of(void* f2, int p, size_t hb) { return reinterpret_cast<char*>(f2) + (size_t)p * hb; }

__device__ inline void store_half(void* f, size_t i, bool upper, const cx<float> s[6]) {
  float4* b = reinterpret_cast<float4*>(f);
  const int o = upper ? 0 : 3;
#pragma unroll
  for (int k = 0; k < 3; ++k) b[widx(i, o + k, 6)] = make_float4(s[2 * k].r, s[2 * k].i, s[2 * k + 1].r, s[2 * k + 1].i);
}

// (u, l) -> (c_+, c_-), and back
__device__ inline void to_chiral(const cx<float> v[12], cx<float> c[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    c[k] = RS2 * (v[k] - v[6 + k]);
    c[6 + k] = RS2 * (v[k] + v[6 + k]);
  }
}
__device__ inline void from_chiral(const cx<float> c[12], cx<float> v[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    v[k] = RS2 * (c[k] + c[6 + k]);
    v[6 + k] = RS2 * (c[6 + k] - c[k]);
  }
}

// all-reduce of two doubles over the workgroup (every lane gets the sums)
__device__ inline void wg_sum2(double& a, double& b) {
  __shared__ double red[16][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  __syncthreads();  // red is free (the previous reduction's reads are done)
  if (lane == 0) {
    red[wave][0] = a;
    red[wave][1] = b;
  }
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  a = 0.0;
  b = 0.0;
  for (int w = 0; w < nw; ++w) {
    a += red[w][0];
    b += red[w][1];
  }
}

// ------------------------------------------------------------------ setup
// Gram-Schmidt of the chiral part chi of the n vectors V (DP, FP32, n fields of
// two halves) on one aggregate, in the order k = 0 .. n-1, into the basis B
// (chiral storage). One workgroup per (aggregate, chi), one lane per site.
__global__ void __launch_bounds__(256) k_mg_orth(MgGeom m, const char* V, char* B) {
  const int agg = agg_of_block(m), chi = blockIdx.y;
  const bool live = (int)threadIdx.x < m.asz;
  int c[4], p = 0, i = 0;
  if (live) agg_site(m, agg, threadIdx.x, c, p, i);
  const size_t fb = 2 * m.hb;
  for (int k = 0; k < m.n; ++k) {
    cx<float> w[6];
    if (live) {
      cx<float> v[12], ch[12];
      IO<1>::load_spinor(half_of(V + k * fb, p, m.hb), i, v);
      to_chiral(v, ch);
#pragma unroll
      for (int q = 0; q < 6; ++q) w[q] = chi == 0 ? ch[q] : ch[6 + q];
    } else {
#pragma unroll
      for (int q = 0; q < 6; ++q) w[q] = {0.f, 0.f};
    }
    for (int j = 0; j < k; ++j) {
      cx<float> bj[6];
      double dr = 0.0, di = 0.0;
      if (live) {
        IO<1>::load_half(half_of(B + j * fb, p, m.hb), i, chi == 0, bj);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const cx<float> d = cmulc(bj[q], w[q]);
          dr += d.r;
          di += d.i;
        }
      }
      wg_sum2(dr, di);
      if (live) {
        const cx<float> d = {(float)dr, (float)di};
#pragma unroll
        for (int q = 0; q < 6; ++q) w[q] = w[q] - d * bj[q];
      }
    }
    double nn = 0.0, zero = 0.0;
    if (live)
#pragma unroll
      for (int q = 0; q < 6; ++q) nn += (double)w[q].r * w[q].r + (double)w[q].i * w[q].i;
    wg_sum2(nn, zero);
    const float inv = nn > 0.0 ? (float)(1.0 / std::sqrt(nn)) : 0.f;
    if (live) {
#pragma unroll
      for (int q = 0; q < 6; ++q) w[q] = inv * w[q];
      store_half(half_of(B + k * fb, p, m.hb), i, chi == 0, w);
    }
    __syncthreads();  // B_k complete before the next k reads it
  }
}

// V_k = the DP form of the basis vector B_k (every aggregate and chirality)
__global__ void __launch_bounds__(256) k_mg_to_dp(MgGeom m, const char* B, char* V) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)m.g.vh) return;
  const int p = blockIdx.y, k = blockIdx.z;
  const size_t off = (size_t)k * 2 * m.hb + (size_t)p * m.hb;
  cx<float> ch[12], v[12];
  IO<1>::load_spinor(B + off, i, ch);
  from_chiral(ch, v);
  IO<1>::store_spinor(V + off, i, v);
}

// w = P e with e one at (chi, k) of every aggregate of class cls
__global__ void __launch_bounds__(256) k_mg_unit(MgGeom m, const char* B, int cls, int col, char* w) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)m.g.vh) return;
  const int p = blockIdx.y;
  int x, y, z, t;
  coords_of(m.g, p, (int)i, x, y, z, t);
  const int chi = col / m.n, k = col % m.n;
  cx<float> ch[12], v[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) ch[q] = {0.f, 0.f};
  if (class_of(m, agg_of(m, x, y, z, t)) == cls) {
    cx<float> h[6];
    IO<1>::load_half(B + (size_t)k * 2 * m.hb + (size_t)p * m.hb, i, chi == 0, h);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      if (chi == 0) ch[q] = h[q];
      else ch[6 + q] = h[q];
    }
  }
  from_chiral(ch, v);
  IO<1>::store_spinor(w + (size_t)p * m.hb, i, v);
}

// ------------------------------------------------------------------ restriction
// Per-lane sums of <B_k^chi, chiral_chi(r)> over the lane's site (if it is
// selected), then the workgroup sum, written by lane 0 to out[0 .. 2n).
template <int NC>
__device__ inline void restrict_agg(const MgGeom& m, const char* B, const void* r2, int agg, int face_dir,
                                    int face_side, float2* out, size_t stride) {
  __shared__ float red[4][2 * NMAX * 2];
  cx<float> acc[2][NC];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[h][k] = {0.f, 0.f};
  const int l = threadIdx.x;
  if (l < m.asz) {
    int c[4], p, i;
    agg_site(m, agg, l, c, p, i);
    bool on = true;
    if (face_dir >= 0) {
      const int lc = c[face_dir] % m.a[face_dir];
      on = face_side > 0 ? lc == m.a[face_dir] - 1 : lc == 0;
    }
    if (on) {
      cx<float> v[12], ch[12];
      IO<1>::load_spinor(half_of(r2, p, m.hb), i, v);
      to_chiral(v, ch);
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        if (k < m.n) {
          cx<float> b[12];
          IO<1>::load_spinor(B + (size_t)k * 2 * m.hb + (size_t)p * m.hb, i, b);
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            acc[0][k] = acc[0][k] + cmulc(b[q], ch[q]);
            acc[1][k] = acc[1][k] + cmulc(b[6 + q], ch[6 + q]);
          }
        }
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      float re = acc[h][k].r, im = acc[h][k].i;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o, 64);
        im += __shfl_xor(im, o, 64);
      }
      if (lane == 0) {
        red[wave][(h * NC + k) * 2] = re;
        red[wave][(h * NC + k) * 2 + 1] = im;
      }
    }
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  if ((int)threadIdx.x < 2 * m.n) {
    const int h = threadIdx.x / m.n, k = threadIdx.x % m.n;
    float re = 0.f, im = 0.f;
    for (int w = 0; w < nw; ++w) {
      re += red[w][(h * NC + k) * 2];
      im += red[w][(h * NC + k) * 2 + 1];
    }
    out[(size_t)threadIdx.x * stride] = make_float2(re, im);
  }
  __syncthreads();  // red reused by the next call in this workgroup
}

// rc = P^dag r (r: FP32 DP, two halves)
template <int NC>
__global__ void __launch_bounds__(256) k_mg_restrict(MgGeom m, const char* B, const void* r2, float2* rc) {
  const int agg = agg_of_block(m);
  restrict_agg<NC>(m, B, r2, agg, -1, 0, rc + (size_t)agg * 2 * m.n, 1);
}

// columns col of the coarse blocks from y = D (P e_{class, col}); M holds,
// for each (agg, dir), the 2n x 2n block by pairs of columns: entry (row, col)
// at ((agg * 9 + dir) * n + col / 2) * 4n + 2 row + col % 2 (dir 0 = self,
// 1 + 2 mu = +mu, 2 + 2 mu = -mu), so that the lanes of consecutive rows read
// consecutive 16-byte pairs in the coarse apply
template <int NC>
__global__ void __launch_bounds__(256) k_mg_collect(MgGeom m, const char* B, const void* y2, int cls, int col,
                                                    float2* M) {
  const int agg = agg_of_block(m);
  const int d = class_of(m, agg) ^ cls;
  const int n2 = 2 * m.n;
  float2* base = M + (size_t)agg * 9 * n2 * n2 + (size_t)(col >> 1) * 2 * n2 + (col & 1);
  if (d == 0) {
    restrict_agg<NC>(m, B, y2, agg, -1, 0, base, 2);
    return;
  }
  if (d & (d - 1)) return;  // two or more bits: no neighbour of class cls
  const int mu = d == 1 ? 0 : d == 2 ? 1 : d == 4 ? 2 : 3;
  restrict_agg<NC>(m, B, y2, agg, mu, +1, base + (size_t)(1 + 2 * mu) * n2 * n2, 2);
  restrict_agg<NC>(m, B, y2, agg, mu, -1, base + (size_t)(2 + 2 * mu) * n2 * n2, 2);
}

// ------------------------------------------------------------------ prolongation
// x = P e (FP32 DP, two halves)
template <int NC>
__global__ void __launch_bounds__(256) k_mg_prolong(MgGeom m, const char* B, const float2* e, char* x2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)m.g.vh) return;
  const int p = blockIdx.y;
  int x, y, z, t;
  coords_of(m.g, p, (int)i, x, y, z, t);
  const float2* ea = e + (size_t)agg_of(m, x, y, z, t) * 2 * m.n;
  cx<float> ch[12], v[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) ch[q] = {0.f, 0.f};
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (k < m.n) {
      const float2 cp = ea[k], cm = ea[m.n + k];
      const cx<float> a = {cp.x, cp.y}, b = {cm.x, cm.y};
      cx<float> bv[12];
      IO<1>::load_spinor(B + (size_t)k * 2 * m.hb + (size_t)p * m.hb, i, bv);
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        ch[q] = ch[q] + a * bv[q];
        ch[6 + q] = ch[6 + q] + b * bv[6 + q];
      }
    }
  }
  from_chiral(ch, v);
  IO<1>::store_spinor(x2 + (size_t)p * m.hb, i, v);
}

// ------------------------------------------------------------------ coarse operator
// y = D_c x: four lanes per (aggregate, row), lane j of the four taking the
// stencil blocks j, j + 4 and j + 8, their sums added by lane exchanges (the
// coarse lattice is small: this quadruples the waves in flight)
__global__ void __launch_bounds__(256) k_mg_capply(MgGeom m, const float2* M, const float2* x, float2* y) {
  const int n2 = 2 * m.n;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t q = t >> 2;
  const int sub = (int)(t & 3);
  const bool live = q < (size_t)m.nagg * n2;
  float re = 0.f, im = 0.f;
  if (live) {
    const int agg = (int)(q / n2), row = (int)(q % n2);
    int ac[4];
    int r = agg;
    for (int d = 0; d < 3; ++d) {
      ac[d] = r % m.na[d];
      r /= m.na[d];
    }
    ac[3] = r;
    for (int dir = sub; dir < 9; dir += 4) {
      int nb = agg;
      if (dir > 0) {
        const int mu = (dir - 1) >> 1, sg = (dir & 1) ? 1 : -1;
        int cc[4] = {ac[0], ac[1], ac[2], ac[3]};
        cc[mu] = (cc[mu] + sg + m.na[mu]) % m.na[mu];
        nb = cc[0] + m.na[0] * (cc[1] + m.na[1] * (cc[2] + m.na[2] * cc[3]));
      }
      // a pair of columns per load; the rows of a block sit side by side for
      // each pair, so consecutive lanes read consecutive 16 bytes
      const float4* Mr = reinterpret_cast<const float4*>(M + ((size_t)agg * 9 + dir) * n2 * n2) + row;
      const float4* xv = reinterpret_cast<const float4*>(x + (size_t)nb * n2);
      for (int c = 0; c < n2 / 2; ++c) {
        const float4 a = Mr[(size_t)c * n2], b = xv[c];
        re += a.x * b.x - a.y * b.y + a.z * b.z - a.w * b.w;
        im += a.x * b.y + a.y * b.x + a.z * b.w + a.w * b.z;
      }
    }
  }
  re += __shfl_xor(re, 1, 64);
  im += __shfl_xor(im, 1, 64);
  re += __shfl_xor(re, 2, 64);
  im += __shfl_xor(im, 2, 64);
  if (live && sub == 0) y[q] = make_float2(re, im);
}

// coarse vectors: out = ca a + cb b + cc c (b, c may be null)
__global__ void __launch_bounds__(256) k_c_lin3(float2* out, const float2* a, float2 ca, const float2* b, float2 cb,
                                                const float2* c, float2 cc, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  auto mul = [](float2 s, float2 v) { return make_float2(s.x * v.x - s.y * v.y, s.x * v.y + s.y * v.x); };
  float2 w = mul(ca, a[i]);
  if (b) {
    const float2 t = mul(cb, b[i]);
    w.x += t.x;
    w.y += t.y;
  }
  if (c) {
    const float2 t = mul(cc, c[i]);
    w.x += t.x;
    w.y += t.y;
  }
  out[i] = w;
}

// per-workgroup partial sums of <a, b> and <b, b> (FP64)
__global__ void __launch_bounds__(256) k_c_dot(const float2* a, const float2* b, double* partials, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (i < n) {
    const float2 x = a[i], y = b[i];
    v[0] = (double)x.x * y.x + (double)x.y * y.y;
    v[1] = (double)x.x * y.y - (double)x.y * y.x;
    v[2] = (double)y.x * y.x + (double)y.y * y.y;
  }
  block_reduce<3>(v, partials + (size_t)blockIdx.x * 3);
}

// FP32 full fields (two halves): out = a + s b
__global__ void __launch_bounds__(256) k_f32_axpy(char* out, const char* a, float s, const char* b, MgGeom m) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)m.g.vh) return;
  const size_t off = (size_t)blockIdx.y * m.hb;
  cx<float> x[12], y[12];
  IO<1>::load_spinor(a + off, i, x);
  IO<1>::load_spinor(b + off, i, y);
#pragma unroll
  for (int k = 0; k < 12; ++k) x[k] = x[k] + s * y[k];
  IO<1>::store_spinor(out + off, i, x);
}

struct MgState {
  MgGeom m{};
  lqcd_mg_params prm{};
  char* B = nullptr;    // n chiral basis fields (FP32, two halves each)
  float2* M = nullptr;  // [nagg][9][n column pairs][2n rows][2]
  float2* cv[8] = {};   // coarse work vectors
  char* f32[4] = {};    // FP32 full fields (two halves)
  double* partials = nullptr;
  std::vector<double> host;
  ~MgState() {
    (void)hipFree(B);
    (void)hipFree(M);
    for (auto* p : cv) (void)hipFree(p);
    for (auto* p : f32) (void)hipFree(p);
    (void)hipFree(partials);
  }
  size_t nc() const { return (size_t)m.nagg * 2 * m.n; }
};

void free_state(void* p) { delete reinterpret_cast<MgState*>(p); }

MgState* state_of(lqcd_ctx* c) { return reinterpret_cast<MgState*>(c->mg); }

int grid1(size_t n) { return (int)((n + 255) / 256); }

template <typename F>
int dispatch_nc(int n, F&& f) {
  if (n <= 8) return f(std::integral_constant<int, 8>{});
  if (n <= 16) return f(std::integral_constant<int, 16>{});
  return f(std::integral_constant<int, NMAX>{});
}

int alloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(LQCD_ENOMEM, "multigrid workspace allocation failed");
  }
  return LQCD_OK;
}

int agg_block(const MgGeom& m) { return (m.asz + 63) / 64 * 64; }

int restrict_to(lqcd_ctx* c, MgState& s, const void* r2, float2* rc) {
  const MgGeom& m = s.m;
  LQ_TRY(dispatch_nc(m.n, [&](auto nc) {
    hipLaunchKernelGGL(k_mg_restrict<decltype(nc)::value>, dim3(m.nagg), dim3(agg_block(m)), 0, c->stream, m, s.B,
                       r2, rc);
    return LQCD_OK;
  }));
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int prolong_to(lqcd_ctx* c, MgState& s, const float2* e, void* x2) {
  const MgGeom& m = s.m;
  LQ_TRY(dispatch_nc(m.n, [&](auto nc) {
    hipLaunchKernelGGL(k_mg_prolong<decltype(nc)::value>, dim3(grid1(m.g.vh), 2), dim3(256), 0, c->stream, m, s.B, e,
                       reinterpret_cast<char*>(x2));
    return LQCD_OK;
  }));
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int capply(lqcd_ctx* c, MgState& s, const float2* x, float2* y) {
  hipLaunchKernelGGL(k_mg_capply, dim3(grid1(4 * s.nc())), dim3(256), 0, c->stream, s.m, s.M, x, y);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int clin(lqcd_ctx* c, MgState& s, float2* out, float2 ca, const float2* a, float2 cb = {0, 0},
         const float2* b = nullptr, float2 cc = {0, 0}, const float2* cf = nullptr) {
  hipLaunchKernelGGL(k_c_lin3, dim3(grid1(s.nc())), dim3(256), 0, c->stream, out, a, ca, b, cb, cf, cc, s.nc());
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int cdot(lqcd_ctx* c, MgState& s, const float2* a, const float2* b, cx<double>* ab, double* bb) {
  const int nb = grid1(s.nc());
  hipLaunchKernelGGL(k_c_dot, dim3(nb), dim3(256), 0, c->stream, a, b, s.partials, s.nc());
  LQ_HIP(hipGetLastError());
  s.host.resize((size_t)nb * 3);
  LQ_HIP(hipMemcpyAsync(s.host.data(), s.partials, s.host.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  double v[3] = {0.0, 0.0, 0.0};
  for (size_t k = 0; k < s.host.size(); k += 3)
    for (int j = 0; j < 3; ++j) v[j] += s.host[k + j];
  if (ab) *ab = {v[0], v[1]};
  if (bb) *bb = v[2];
  return LQCD_OK;
}

inline float2 f2(cx<double> z) { return make_float2((float)z.r, (float)z.i); }
inline cx<double> cdiv(cx<double> a, cx<double> b) {
  const double d = b.r * b.r + b.i * b.i;
  return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

// e = D_c^-1 rc approximately: BiCGStab from zero to |rc - D_c e| <= tol |rc|
// (iterated residual) or max_iter iterations. cv[0] = rc; result in cv[1].
int coarse_solve(lqcd_ctx* c, MgState& s, int& iters) {
  float2 *b = s.cv[0], *x = s.cv[1], *r = s.cv[2], *rh = s.cv[3], *p = s.cv[4], *v = s.cv[5], *t = s.cv[6],
         *q = s.cv[7];
  LQ_HIP(hipMemsetAsync(x, 0, s.nc() * sizeof(float2), c->stream));
  double bb = 0.0;
  LQ_TRY(cdot(c, s, b, b, nullptr, &bb));
  iters = 0;
  if (bb == 0.0) return LQCD_OK;
  const double target = s.prm.coarse_tol * std::sqrt(bb);
  LQ_TRY(clin(c, s, r, {1, 0}, b));
  LQ_TRY(clin(c, s, rh, {1, 0}, b));
  LQ_HIP(hipMemsetAsync(p, 0, s.nc() * sizeof(float2), c->stream));
  LQ_HIP(hipMemsetAsync(v, 0, s.nc() * sizeof(float2), c->stream));
  cx<double> rho_old{1, 0}, alpha{1, 0}, omega{1, 0};
  // rho = <rhat, r>; later iterations take it from the residual-norm pass
  cx<double> rho;
  LQ_TRY(cdot(c, s, rh, r, &rho, nullptr));
  while (iters < s.prm.coarse_max_iter) {
    if (rho.r == 0.0 && rho.i == 0.0) break;
    const cx<double> beta = cdiv(rho, rho_old) * cdiv(alpha, omega);
    LQ_TRY(clin(c, s, p, {1, 0}, r, f2(beta), p, f2({-(beta * omega).r, -(beta * omega).i}), v));
    LQ_TRY(capply(c, s, p, v));
    cx<double> rv;
    LQ_TRY(cdot(c, s, rh, v, &rv, nullptr));
    if (rv.r == 0.0 && rv.i == 0.0) break;
    alpha = cdiv(rho, rv);
    LQ_TRY(clin(c, s, q, {1, 0}, r, f2({-alpha.r, -alpha.i}), v));  // s
    LQ_TRY(capply(c, s, q, t));
    // one pass: <s, t> (its conjugate is <t, s>) and <t, t>
    cx<double> st;
    double tt = 0.0;
    LQ_TRY(cdot(c, s, q, t, &st, &tt));
    omega = tt != 0.0 ? cx<double>{st.r / tt, -st.i / tt} : cx<double>{0, 0};
    LQ_TRY(clin(c, s, x, {1, 0}, x, f2(alpha), p, f2(omega), q));
    LQ_TRY(clin(c, s, r, {1, 0}, q, f2({-omega.r, -omega.i}), t));
    rho_old = rho;
    ++iters;
    // one pass: the next rho = <rhat, r> and |r|^2
    double rr = 0.0;
    LQ_TRY(cdot(c, s, rh, r, &rho, &rr));
    if (std::sqrt(rr) <= target || (omega.r == 0.0 && omega.i == 0.0)) break;
  }
  return LQCD_OK;
}

__global__ void __launch_bounds__(256) k_c_convert(const void* src, int src_f64, void* dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (src_f64) {
    const double2 v = reinterpret_cast<const double2*>(src)[i];
    reinterpret_cast<float2*>(dst)[i] = make_float2((float)v.x, (float)v.y);
  } else {
    const float2 v = reinterpret_cast<const float2*>(src)[i];
    reinterpret_cast<double2*>(dst)[i] = make_double2((double)v.x, (double)v.y);
  }
}

}  // namespace

int mg_coarse_convert(lqcd_ctx* c, const void* src, bool src_f64, void* dst, size_t n) {
  hipLaunchKernelGGL(k_c_convert, dim3(grid1(n)), dim3(256), 0, c->stream, src, src_f64 ? 1 : 0, dst, n);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

bool mg_shape_ok(const Geom& g, const int a[4]) {
  const int L[4] = {g.lx, g.ly, g.lz, g.lt};
  int asz = 1;
  for (int d = 0; d < 4; ++d) {
    if (a[d] < 2 || L[d] % a[d] != 0 || (L[d] / a[d]) % 2 != 0) return false;
    asz *= a[d];
  }
  return asz <= 256;
}

int mg_setup(lqcd_ctx* c, const lqcd_mg_params& prm, const double* start) {
  if (c->mg && c->mg_free) {
    c->mg_free(c->mg);
    c->mg = nullptr;
  }
  auto* s = new MgState();
  c->mg = s;
  c->mg_free = free_state;
  s->prm = prm;
  MgGeom& m = s->m;
  m.g = c->g;
  const int L[4] = {c->g.lx, c->g.ly, c->g.lz, c->g.lt};
  m.nagg = 1;
  m.asz = 1;
  for (int d = 0; d < 4; ++d) {
    m.a[d] = prm.agg[d];
    m.na[d] = L[d] / prm.agg[d];
    m.nagg *= m.na[d];
    m.asz *= m.a[d];
  }
  m.n = prm.nvec;
  m.hb = spinor_bytes(1, c->g.vh);
  const size_t fb = 2 * m.hb, n2 = 2 * (size_t)m.n;
  LQ_TRY(alloc((void**)&s->B, fb * m.n));
  LQ_TRY(alloc((void**)&s->M, (size_t)m.nagg * 9 * n2 * n2 * sizeof(float2)));
  for (auto& p : s->cv) LQ_TRY(alloc((void**)&p, s->nc() * sizeof(float2)));
  for (auto& p : s->f32) LQ_TRY(alloc((void**)&p, fb));
  LQ_TRY(alloc((void**)&s->partials, (size_t)grid1(s->nc()) * 3 * sizeof(double)));
  // padding sites of every FP32 field read as zero
  LQ_HIP(hipMemsetAsync(s->B, 0, fb * m.n, c->stream));
  for (auto& p : s->f32) LQ_HIP(hipMemsetAsync(p, 0, fb, c->stream));

  // test vectors V (DP, FP32) from the canonical start vectors
  char* V = nullptr;
  LQ_TRY(alloc((void**)&V, fb * m.n));
  struct Free {
    char* p;
    ~Free() { (void)hipFree(p); }
  } fv{V};
  LQ_HIP(hipMemsetAsync(V, 0, fb * m.n, c->stream));
  const size_t vol = (size_t)c->g.vh * 2;
  for (int k = 0; k < m.n; ++k)
    for (int p = 0; p < 2; ++p)
      LQ_TRY(launch_import_spinor(c, 1, p, start + (size_t)k * vol * 24, V + (size_t)k * fb + (size_t)p * m.hb));
  const dim3 og(m.nagg, 2), ob(agg_block(m));
  if (prm.setup_iters == 0) hipLaunchKernelGGL(k_mg_orth, og, ob, 0, c->stream, m, V, s->B);
  const dim3 g2(grid1(c->g.vh), 2);
  for (int it = 0; it < prm.setup_iters; ++it) {
    // one SAP-smoothing step of D v = 0 per vector: v <- v - M_SAP D v
    char *t = s->f32[0], *u = s->f32[1];
    for (int k = 0; k < m.n; ++k) {
      char* vk = V + (size_t)k * fb;
      LQ_TRY(op_full(c, 1, vk, vk + m.hb, t, t + m.hb));
      LQ_TRY(sap_apply(c, prm.sap.block, prm.sap.ncycles, prm.sap.nmr, t, t + m.hb, u, u + m.hb));
      hipLaunchKernelGGL(k_f32_axpy, g2, dim3(256), 0, c->stream, vk, vk, -1.f, u, m);
    }
    hipLaunchKernelGGL(k_mg_orth, og, ob, 0, c->stream, m, V, s->B);
    hipLaunchKernelGGL(k_mg_to_dp, dim3(grid1(c->g.vh), 2, m.n), dim3(256), 0, c->stream, m, s->B, V);
  }
  LQ_HIP(hipGetLastError());

  // coarse operator, 16 classes x 2n columns
  char *w = s->f32[0], *y = s->f32[1];
  for (int cls = 0; cls < 16; ++cls)
    for (int col = 0; col < (int)n2; ++col) {
      hipLaunchKernelGGL(k_mg_unit, dim3(grid1(c->g.vh), 2), dim3(256), 0, c->stream, m, s->B, cls, col, w);
      LQ_TRY(op_full(c, 1, w, w + m.hb, y, y + m.hb));
      LQ_TRY(dispatch_nc(m.n, [&](auto nc) {
        hipLaunchKernelGGL(k_mg_collect<decltype(nc)::value>, dim3(m.nagg), ob, 0, c->stream, m, s->B, y, cls, col,
                           s->M);
        return LQCD_OK;
      }));
    }
  LQ_HIP(hipGetLastError());
  LQ_HIP(hipStreamSynchronize(c->stream));
  return LQCD_OK;
}

size_t mg_coarse_size(lqcd_ctx* c) { return c->mg ? state_of(c)->nc() : 0; }

int mg_restrict(lqcd_ctx* c, const void* r_e, const void* r_o, void* rc) {
  MgState& s = *state_of(c);
  char* r2 = s.f32[2];
  LQ_HIP(hipMemcpyAsync(r2, r_e, s.m.hb, hipMemcpyDeviceToDevice, c->stream));
  LQ_HIP(hipMemcpyAsync(r2 + s.m.hb, r_o, s.m.hb, hipMemcpyDeviceToDevice, c->stream));
  return restrict_to(c, s, r2, reinterpret_cast<float2*>(rc));
}

int mg_prolong(lqcd_ctx* c, const void* ec, void* x_e, void* x_o) {
  MgState& s = *state_of(c);
  char* x2 = s.f32[2];
  LQ_TRY(prolong_to(c, s, reinterpret_cast<const float2*>(ec), x2));
  LQ_HIP(hipMemcpyAsync(x_e, x2, s.m.hb, hipMemcpyDeviceToDevice, c->stream));
  LQ_HIP(hipMemcpyAsync(x_o, x2 + s.m.hb, s.m.hb, hipMemcpyDeviceToDevice, c->stream));
  return LQCD_OK;
}

int mg_coarse_apply(lqcd_ctx* c, const void* in, void* out) {
  MgState& s = *state_of(c);
  return capply(c, s, reinterpret_cast<const float2*>(in), reinterpret_cast<float2*>(out));
}

// x = coarse correction + SAP post-smoothing of r (FP32 halves in and out)
int mg_precond(lqcd_ctx* c, const void* r_e, const void* r_o, void* x_e, void* x_o, int* coarse_iters) {
  MgState& s = *state_of(c);
  const size_t hb = s.m.hb;
  char *r2 = s.f32[2], *x2 = s.f32[0], *t2 = s.f32[1], *u2 = s.f32[3];
  LQ_HIP(hipMemcpyAsync(r2, r_e, hb, hipMemcpyDeviceToDevice, c->stream));
  LQ_HIP(hipMemcpyAsync(r2 + hb, r_o, hb, hipMemcpyDeviceToDevice, c->stream));
  LQ_TRY(restrict_to(c, s, r2, s.cv[0]));
  int it = 0;
  LQ_TRY(coarse_solve(c, s, it));
  if (coarse_iters) *coarse_iters = it;
  LQ_TRY(prolong_to(c, s, s.cv[1], x2));
  LQ_TRY(op_full(c, 1, x2, x2 + hb, t2, t2 + hb));
  const dim3 g2(grid1(c->g.vh), 2);
  hipLaunchKernelGGL(k_f32_axpy, g2, dim3(256), 0, c->stream, t2, r2, -1.f, t2, s.m);  // r - D x
  LQ_TRY(sap_apply(c, s.prm.sap.block, s.prm.sap.ncycles, s.prm.sap.nmr, t2, t2 + hb, u2, u2 + hb));
  hipLaunchKernelGGL(k_f32_axpy, g2, dim3(256), 0, c->stream, x2, x2, 1.f, u2, s.m);
  LQ_HIP(hipGetLastError());
  LQ_HIP(hipMemcpyAsync(x_e, x2, hb, hipMemcpyDeviceToDevice, c->stream));
  LQ_HIP(hipMemcpyAsync(x_o, x2 + hb, hb, hipMemcpyDeviceToDevice, c->stream));
  return LQCD_OK;
}

int solve_mg(lqcd_ctx* c, const lqcd_solve_params& prm, const void* b_e, const void* b_o, void* x_e, void* x_o,
             bool zero_x, lqcd_solve_stats& st, long* coarse_iters_total) {
  MgState& s = *state_of(c);
  const size_t b32 = s.m.hb;
  void *e32[2] = {}, *q32[2] = {};
  struct Free {
    void** p;
    ~Free() {
      for (int k = 0; k < 2; ++k) (void)hipFree(p[k]);
    }
  } fe{e32}, fq{q32};
  for (int h = 0; h < 2; ++h) {
    LQ_TRY(alloc(&e32[h], b32));
    LQ_TRY(alloc(&q32[h], b32));
  }
  long total = 0;
  FlexPrecond pre = [&](const void* ie, const void* io, void* oe, void* oo) -> int {
    LQ_TRY(launch_convert_field(c, 0, ie, 1, e32[0]));
    LQ_TRY(launch_convert_field(c, 0, io, 1, e32[1]));
    int it = 0;
    LQ_TRY(mg_precond(c, e32[0], e32[1], q32[0], q32[1], &it));
    total += it;
    LQ_TRY(launch_convert_field(c, 1, q32[0], 0, oe));
    LQ_TRY(launch_convert_field(c, 1, q32[1], 0, oo));
    return LQCD_OK;
  };
  const int status = solve_flexible(c, prm, pre, "MG", b_e, b_o, x_e, x_o, zero_x, st);
  if (coarse_iters_total) *coarse_iters_total = total;
  return status;
}

}  // namespace lq
