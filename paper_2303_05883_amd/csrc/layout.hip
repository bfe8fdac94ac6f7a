// Conversions at the boundary: canonical complex128 fields <-> native
// checkerboarded structure-of-arrays fields, link compression to two rows with
// an SU(3) check, and precision conversion of native fields (the paper,
// Sec. 2: the machine-specific layout and basis differ from the application's,
// so data are converted before and after the machine-specific code).
#include "fieldio.h"
#include "internal.h"

namespace lq {

namespace {

__device__ inline void site_coords(const Geom& g, int p, int i, int& x, int& y, int& z, int& t) {
  const int xh = i % g.lxh;
  int r = i / g.lxh;
  y = r % g.ly;
  r /= g.ly;
  z = r % g.lz;
  t = r / g.lz;
  x = 2 * xh + ((y + z + t + p) & 1);
}

__device__ inline size_t full_index(const Geom& g, int x, int y, int z, int t) {
  return (size_t)x + (size_t)g.lx * ((size_t)y + (size_t)g.ly * ((size_t)z + (size_t)g.lz * (size_t)t));
}

template <int P>
__global__ void __launch_bounds__(256) k_import_spinor(Geom g, int p, const double* canon, void* half) {
  using T = typename IO<P>::T;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.vh) return;
  int x, y, z, t;
  site_coords(g, p, i, x, y, z, t);
  const double2* src = reinterpret_cast<const double2*>(canon) + 12 * full_index(g, x, y, z, t);
  cx<T> s[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double2 v = src[k];
    s[k] = {(T)v.x, (T)v.y};
  }
  IO<P>::store_spinor(half, i, s);
}

template <int P>
__global__ void __launch_bounds__(256) k_export_spinor(Geom g, int p, const void* half, double* canon) {
  using T = typename IO<P>::T;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.vh) return;
  int x, y, z, t;
  site_coords(g, p, i, x, y, z, t);
  double2* dst = reinterpret_cast<double2*>(canon) + 12 * full_index(g, x, y, z, t);
  cx<T> s[12];
  IO<P>::load_spinor(half, i, s);
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = make_double2((double)s[k].r, (double)s[k].i);
}

__global__ void __launch_bounds__(256) k_zero_parity(Geom g, int p, double* canon) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.vh) return;
  int x, y, z, t;
  site_coords(g, p, i, x, y, z, t);
  double2* dst = reinterpret_cast<double2*>(canon) + 12 * full_index(g, x, y, z, t);
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = make_double2(0.0, 0.0);
}

// Atomic max of a non-negative double kept as its bit pattern (monotone for
// non-negative IEEE values); a non-finite value raises the flag instead.
__device__ inline void record_error(unsigned long long* chk, double e) {
  if (!(e <= 1e300)) {
    atomicOr(chk + 1, 1ull);
    return;
  }
  atomicMax(chk, (unsigned long long)__double_as_longlong(e));
}

// One thread per (site of parity p): checks each of its 4 links and writes
// rows 0, 1 in FP64, FP32 and FP16 layouts.
__global__ void __launch_bounds__(256) k_import_gauge(Geom g, int p, const double* canon, void* g64, void* g32,
                                                      void* g16, unsigned long long* chk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.vh) return;
  int x, y, z, t;
  site_coords(g, p, i, x, y, z, t);
  const size_t vh = g.vh;
  const double2* src = reinterpret_cast<const double2*>(canon) + 36 * full_index(g, x, y, z, t);
  double err = 0.0;
  for (int mu = 0; mu < 4; ++mu) {
    cx<double> u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double2 v = src[9 * mu + k];
      u[k] = {v.x, v.y};
    }
    // max |U U^dag - 1|
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        cx<double> s = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 3; ++k) s = s + u[3 * a + k] * conj(u[3 * b + k]);
        if (a == b) s.r -= 1.0;
        err = fmax(err, sqrt(s.r * s.r + s.i * s.i));
        if (!(s.r == s.r) || !(s.i == s.i)) err = __longlong_as_double(0x7ff8000000000000ll);
      }
    // |det U - 1|
    const cx<double> det = u[0] * (u[4] * u[8] - u[5] * u[7]) - u[1] * (u[3] * u[8] - u[5] * u[6]) +
                           u[2] * (u[3] * u[7] - u[4] * u[6]);
    const double dr = det.r - 1.0, di = det.i;
    const double de = sqrt(dr * dr + di * di);
    err = (de == de) ? fmax(err, de) : de;
    if (!(err == err)) break;

    const size_t blkidx = (size_t)(p * 4 + mu);
    double2* d64 = reinterpret_cast<double2*>(reinterpret_cast<char*>(g64) + blkidx * link_bytes(0, vh));
    float4* d32 = reinterpret_cast<float4*>(reinterpret_cast<char*>(g32) + blkidx * link_bytes(1, vh));
    half4* d16 = reinterpret_cast<half4*>(reinterpret_cast<char*>(g16) + blkidx * link_bytes(2, vh));
#pragma unroll
    for (int k = 0; k < 6; ++k) d64[widx(i, k, 6)] = make_double2(u[k].r, u[k].i);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      d32[widx(i, k, 3)] = make_float4((float)u[2 * k].r, (float)u[2 * k].i, (float)u[2 * k + 1].r,
                                    (float)u[2 * k + 1].i);
      half4 h;
      h[0] = (_Float16)u[2 * k].r;
      h[1] = (_Float16)u[2 * k].i;
      h[2] = (_Float16)u[2 * k + 1].r;
      h[3] = (_Float16)u[2 * k + 1].i;
      d16[widx(i, k, 3)] = h;
    }
  }
  record_error(chk, err);
}

template <int PS, int PD>
__global__ void __launch_bounds__(256) k_convert(const void* src, void* dst, size_t vh) {
  using TS = typename IO<PS>::T;
  using TD = typename IO<PD>::T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vh) return;
  cx<TS> s[12];
  cx<TD> d[12];
  IO<PS>::load_spinor(src, i, s);
#pragma unroll
  for (int k = 0; k < 12; ++k) d[k] = {(TD)s[k].r, (TD)s[k].i};
  IO<PD>::store_spinor(dst, i, d);
}

__global__ void __launch_bounds__(256) k_check_finite(const double* p, size_t n, unsigned long long* flag) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (; i < n; i += stride) {
    const double v = p[i];
    bad |= !(fabs(v) <= 1.7976931348623157e308);
  }
  if (bad) atomicOr(flag, 1ull);
}

inline int grid_for(size_t n, int bs) { return (int)((n + bs - 1) / bs); }

}  // namespace

int launch_import_spinor(lqcd_ctx* c, int prec, int parity, const double* canon, void* half) {
  const int nb = grid_for(c->g.vh, 256);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_import_spinor<0>, dim3(nb), dim3(256), 0, c->stream, c->g, parity, canon, half); break;
    case 1: hipLaunchKernelGGL(k_import_spinor<1>, dim3(nb), dim3(256), 0, c->stream, c->g, parity, canon, half); break;
    case 2: hipLaunchKernelGGL(k_import_spinor<2>, dim3(nb), dim3(256), 0, c->stream, c->g, parity, canon, half); break;
    default: return set_error(LQCD_EINVAL, "bad precision");
  }
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int launch_export_spinor(lqcd_ctx* c, int prec, int parity, const void* half, double* canon) {
  const int nb = grid_for(c->g.vh, 256);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_export_spinor<0>, dim3(nb), dim3(256), 0, c->stream, c->g, parity, half, canon); break;
    case 1: hipLaunchKernelGGL(k_export_spinor<1>, dim3(nb), dim3(256), 0, c->stream, c->g, parity, half, canon); break;
    case 2: hipLaunchKernelGGL(k_export_spinor<2>, dim3(nb), dim3(256), 0, c->stream, c->g, parity, half, canon); break;
    default: return set_error(LQCD_EINVAL, "bad precision");
  }
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int launch_zero_parity(lqcd_ctx* c, int parity, double* canon) {
  hipLaunchKernelGGL(k_zero_parity, dim3(grid_for(c->g.vh, 256)), dim3(256), 0, c->stream, c->g, parity, canon);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int launch_import_gauge(lqcd_ctx* c, const double* canon, double* check) {
  unsigned long long* chk = reinterpret_cast<unsigned long long*>(check);
  for (int p = 0; p < 2; ++p)
    hipLaunchKernelGGL(k_import_gauge, dim3(grid_for(c->g.vh, 256)), dim3(256), 0, c->stream, c->g, p, canon,
                       c->gauge[0], c->gauge[1], c->gauge[2], chk);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int launch_convert_field(lqcd_ctx* c, int sp, const void* src, int dp, void* dst) {
  const size_t vh = c->g.vh;
  const int nb = grid_for(vh, 256);
  hipStream_t s = c->stream;
#define LQ_CONV(A, B) \
  if (sp == A && dp == B) hipLaunchKernelGGL((k_convert<A, B>), dim3(nb), dim3(256), 0, s, src, dst, vh)
  LQ_CONV(0, 1); else LQ_CONV(1, 0); else LQ_CONV(0, 2); else LQ_CONV(2, 0); else LQ_CONV(1, 2);
  else LQ_CONV(2, 1); else LQ_CONV(0, 0); else LQ_CONV(1, 1); else LQ_CONV(2, 2);
  else return set_error(LQCD_EINVAL, "bad precision pair");
#undef LQ_CONV
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

int launch_check_finite(lqcd_ctx* c, const double* p, size_t n, double* flag) {
  int nb = grid_for(n, 256);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_check_finite, dim3(nb), dim3(256), 0, c->stream, p, n,
                     reinterpret_cast<unsigned long long*>(flag));
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

}  // namespace lq
