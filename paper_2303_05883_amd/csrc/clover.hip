// Clover site matrices on the GPU (set-up, FP64).
//
// A(x) = 1 + kappa c_SW sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x), with
// F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dag)/(8i) and Q_{mu nu} the sum of the four
// plaquettes of the (mu, nu) plane that start and end at x (the clover
// operator the paper benchmarks, Sec. 2/3; its even-odd use needs A and A^-1,
// Eq. (1)). sigma_{mu nu} = [gamma_mu, gamma_nu]/(2i) commutes with gamma5, so
// in the chiral basis chi_+- = (psi_{0,1} -+ psi_{2,3})/sqrt(2) A is
// diag(B_+, B_-) with 6x6 Hermitian blocks. With the Dirac-Pauli gammas:
//   sigma_{jk} = eps_{jkl} diag(s_l, s_l) -> s_l in both blocks,
//   sigma_{jt} = [[0, s_j], [s_j, 0]]       -> -s_j in B_+, +s_j in B_-,
// so B_+- = 1 + kappa c_SW [ s_x (F_yz -+ F_xt) + s_y (-F_xz -+ F_yt) + s_z (F_xy -+ F_zt) ].
// The inverse is taken block by block (Gauss-Jordan, partial pivoting).
#include "fieldio.h"
#include "internal.h"

namespace lq {

namespace {

struct M3 {
  cx<double> a[9];
};

__device__ inline M3 mul(const M3& x, const M3& y) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> s = x.a[3 * i] * y.a[j];
      s = s + x.a[3 * i + 1] * y.a[3 + j];
      s = s + x.a[3 * i + 2] * y.a[6 + j];
      r.a[3 * i + j] = s;
    }
  return r;
}

__device__ inline M3 dag(const M3& x) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[3 * i + j] = conj(x.a[3 * j + i]);
  return r;
}

struct Site {
  int c[4];
};

__device__ inline Site moved(const Geom& g, Site s, int mu, int d) {
  const int L[4] = {g.lx, g.ly, g.lz, g.lt};
  int v = s.c[mu] + d;
  if (v < 0) v += L[mu];
  if (v >= L[mu]) v -= L[mu];
  s.c[mu] = v;
  return s;
}

// U_mu at site s, rebuilt from the two stored FP64 rows.
__device__ inline M3 link(const Geom& g, const char* g64, Site s, int mu) {
  const int p = (s.c[0] + s.c[1] + s.c[2] + s.c[3]) & 1;
  const size_t i = (size_t)(s.c[0] >> 1) + (size_t)g.lxh * (s.c[1] + (size_t)g.ly * (s.c[2] + (size_t)g.lz * s.c[3]));
  const void* blk = g64 + (size_t)(p * 4 + mu) * link_bytes(0, g.vh);
  cx<double> u[6], r2[3];
  IO<0>::load_link(blk, i, u);
  reconstruct(u, r2);
  M3 m;
#pragma unroll
  for (int k = 0; k < 6; ++k) m.a[k] = u[k];
  m.a[6] = r2[0];
  m.a[7] = r2[1];
  m.a[8] = r2[2];
  return m;
}

// F_{mu nu}(s) from the four leaves.
__device__ M3 field_strength(const Geom& g, const char* g64, Site s, int mu, int nu) {
  const Site xm = moved(g, s, mu, -1), xn = moved(g, s, nu, -1);
  const Site xpm = moved(g, s, mu, 1), xpn = moved(g, s, nu, 1);
  const Site xmpn = moved(g, xm, nu, 1), xmmn = moved(g, xm, nu, -1), xpmmn = moved(g, xn, mu, 1);
  const M3 umx = link(g, g64, s, mu), unx = link(g, g64, s, nu);
  M3 q = mul(mul(umx, link(g, g64, xpm, nu)), mul(dag(link(g, g64, xpn, mu)), dag(unx)));
  const M3 umxm = link(g, g64, xm, mu);
  const M3 l2 = mul(mul(unx, dag(link(g, g64, xmpn, mu))), mul(dag(link(g, g64, xm, nu)), umxm));
  const M3 l3 = mul(mul(dag(umxm), dag(link(g, g64, xmmn, nu))), mul(link(g, g64, xmmn, mu), link(g, g64, xn, nu)));
  const M3 unxn = link(g, g64, xn, nu);
  const M3 l4 = mul(mul(dag(unxn), link(g, g64, xn, mu)), mul(link(g, g64, xpmmn, nu), dag(umx)));
#pragma unroll
  for (int k = 0; k < 9; ++k) q.a[k] = q.a[k] + l2.a[k] + l3.a[k] + l4.a[k];
  // F = (Q - Q^dag) / (8i) = -i (Q - Q^dag) / 8
  M3 f;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const cx<double> d = q.a[3 * i + j] - conj(q.a[3 * j + i]);
      f.a[3 * i + j] = 0.125 * mul_mi(d);
    }
  return f;
}

// 6x6 complex matrix, row-major, index 3*s + colour.
struct M6 {
  cx<double> a[36];
};

// m += coef * (pauli (x) f), pauli given as 2x2 complex
__device__ inline void add_kron(M6& m, const cx<double> pauli[4], const M3& f, double coef) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const cx<double> ps = pauli[2 * s + t];
      if (ps.r == 0.0 && ps.i == 0.0) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const cx<double> v = ps * f.a[3 * a + b];
          m.a[6 * (3 * s + a) + 3 * t + b] = m.a[6 * (3 * s + a) + 3 * t + b] + coef * v;
        }
    }
}

// Gauss-Jordan inverse with partial pivoting; returns false if a pivot vanishes.
__device__ bool invert6(const M6& in, M6& out) {
  cx<double> a[6][12];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      a[i][j] = in.a[6 * i + j];
      a[i][6 + j] = {i == j ? 1.0 : 0.0, 0.0};
    }
  double scale = 0.0;
  for (int k = 0; k < 36; ++k) scale = fmax(scale, fabs(in.a[k].r) + fabs(in.a[k].i));
  for (int col = 0; col < 6; ++col) {
    int piv = col;
    double best = -1.0;
    for (int r = col; r < 6; ++r) {
      const double m = a[r][col].r * a[r][col].r + a[r][col].i * a[r][col].i;
      if (m > best) {
        best = m;
        piv = r;
      }
    }
    if (!(sqrt(best) > 1e-13 * scale)) return false;
    if (piv != col)
      for (int j = 0; j < 12; ++j) {
        const cx<double> tmp = a[col][j];
        a[col][j] = a[piv][j];
        a[piv][j] = tmp;
      }
    const cx<double> p = a[col][col];
    const double den = p.r * p.r + p.i * p.i;
    const cx<double> inv = {p.r / den, -p.i / den};
    for (int j = 0; j < 12; ++j) a[col][j] = a[col][j] * inv;
    for (int r = 0; r < 6; ++r) {
      if (r == col) continue;
      const cx<double> f = a[r][col];
      if (f.r == 0.0 && f.i == 0.0) continue;
      for (int j = 0; j < 12; ++j) a[r][j] = a[r][j] - f * a[col][j];
    }
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) out.a[6 * i + j] = a[i][6 + j];
  return true;
}

// Store a Hermitian 6x6 block (times `half`) into 18 slots of the FP64 layout.
__device__ inline void store_block(void* dst, size_t i, int blk, const M6& m, double half) {
  double2* b = reinterpret_cast<double2*>(dst);
  const int o = blk * 18;
  // diagonal (real part; the imaginary part of a Hermitian diagonal is zero)
  b[widx(i, o + 0, 36)] = make_double2(half * m.a[0].r, half * m.a[7].r);
  b[widx(i, o + 1, 36)] = make_double2(half * m.a[14].r, half * m.a[21].r);
  b[widx(i, o + 2, 36)] = make_double2(half * m.a[28].r, half * m.a[35].r);
  int k = 3;
  for (int r = 0; r < 6; ++r)
    for (int c = r + 1; c < 6; ++c) {
      // average with the conjugate of the mirrored entry: exact for Hermitian input,
      // removes the rounding asymmetry of the inverse
      const cx<double> u = m.a[6 * r + c], l = conj(m.a[6 * c + r]);
      b[widx(i, o + k, 36)] = make_double2(half * 0.5 * (u.r + l.r), half * 0.5 * (u.i + l.i));
      ++k;
    }
}

__global__ void __launch_bounds__(128) k_build_clover(Geom g, int p, const char* g64, double kc, void* a_out,
                                                      void* ainv_out, unsigned long long* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.vh) return;
  Site s;
  {
    const int xh = i % g.lxh;
    int r = i / g.lxh;
    s.c[1] = r % g.ly;
    r /= g.ly;
    s.c[2] = r % g.lz;
    s.c[3] = r / g.lz;
    s.c[0] = 2 * xh + ((s.c[1] + s.c[2] + s.c[3] + p) & 1);
  }
  // F in the order xy, xz, xt, yz, yt, zt
  const M3 fxy = field_strength(g, g64, s, 0, 1);
  const M3 fxz = field_strength(g, g64, s, 0, 2);
  const M3 fxt = field_strength(g, g64, s, 0, 3);
  const M3 fyz = field_strength(g, g64, s, 1, 2);
  const M3 fyt = field_strength(g, g64, s, 1, 3);
  const M3 fzt = field_strength(g, g64, s, 2, 3);
  const cx<double> sx[4] = {{0, 0}, {1, 0}, {1, 0}, {0, 0}};
  const cx<double> sy[4] = {{0, 0}, {0, -1}, {0, 1}, {0, 0}};
  const cx<double> sz[4] = {{1, 0}, {0, 0}, {0, 0}, {-1, 0}};
  bool ok = true;
  for (int blk = 0; blk < 2; ++blk) {
    const double sg = blk == 0 ? -1.0 : 1.0;  // sign of the sigma_{jt} terms in this block
    M6 m;
    for (int k = 0; k < 36; ++k) m.a[k] = {(k % 7 == 0) ? 1.0 : 0.0, 0.0};
    add_kron(m, sx, fyz, kc);
    add_kron(m, sx, fxt, sg * kc);
    add_kron(m, sy, fxz, -kc);
    add_kron(m, sy, fyt, sg * kc);
    add_kron(m, sz, fxy, kc);
    add_kron(m, sz, fzt, sg * kc);
    store_block(a_out, i, blk, m, 0.5);
    M6 inv;
    if (!invert6(m, inv)) {
      ok = false;
      for (int k = 0; k < 36; ++k) inv.a[k] = {0.0, 0.0};
    }
    store_block(ainv_out, i, blk, inv, 0.5);
  }
  if (!ok) atomicOr(flag, 1ull);
}

// FP64 clover slot -> FP32 / FP16 slot (elementwise over the 72 reals per site).
__global__ void __launch_bounds__(256) k_clover_down(const double2* src, size_t vh, float4* d32, half8* d16) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vh) return;
  for (int k = 0; k < 9; ++k) {
    double2 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = src[widx(i, 4 * k + j, 36)];
    d32[widx(i, 2 * k, 18)] = make_float4((float)v[0].x, (float)v[0].y, (float)v[1].x, (float)v[1].y);
    d32[widx(i, 2 * k + 1, 18)] = make_float4((float)v[2].x, (float)v[2].y, (float)v[3].x, (float)v[3].y);
    half8 h;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      h[2 * j] = (_Float16)v[j].x;
      h[2 * j + 1] = (_Float16)v[j].y;
    }
    d16[widx(i, k, 9)] = h;
  }
}

}  // namespace

int build_clover(lqcd_ctx* c, double kappa, double csw) {
  const size_t vh = c->g.vh;
  unsigned long long* flag = reinterpret_cast<unsigned long long*>(c->dscal);
  LQ_HIP(hipMemsetAsync(flag, 0, sizeof(unsigned long long), c->stream));
  const int bs = 128;
  const int nb = (int)((vh + bs - 1) / bs);
  for (int p = 0; p < 2; ++p)
    hipLaunchKernelGGL(k_build_clover, dim3(nb), dim3(bs), 0, c->stream, c->g, p,
                       reinterpret_cast<const char*>(c->gauge[0]), kappa * csw, c->clov[0][p], c->clov[0][2 + p],
                       flag);
  LQ_HIP(hipGetLastError());
  const int nb2 = (int)((vh + 255) / 256);
  for (int slot = 0; slot < 4; ++slot)
    hipLaunchKernelGGL(k_clover_down, dim3(nb2), dim3(256), 0, c->stream,
                       reinterpret_cast<const double2*>(c->clov[0][slot]), vh,
                       reinterpret_cast<float4*>(c->clov[1][slot]), reinterpret_cast<half8*>(c->clov[2][slot]));
  LQ_HIP(hipGetLastError());
  unsigned long long h = 0;
  LQ_HIP(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  if (h) return set_error(LQCD_ESINGULAR, "a clover block is singular");
  return LQCD_OK;
}

}  // namespace lq
