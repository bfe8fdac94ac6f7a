// Device-side loads and stores of the native field layouts (see internal.h),
// one specialisation per storage precision: 0 = FP64, 1 = FP32, 2 = FP16.
// FP64 fields compute in double, FP32 and FP16 fields in float.
#pragma once

#include "internal.h"

namespace lq {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

// 16- and 8-byte loads; NT = non-temporal (streamed once, kept out of the caches'
// reuse set so that neighbour spinors stay resident).
template <bool NT>
__device__ inline double2 ld16(const double2* p) {
  if (NT) {
    const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p));
    return make_double2(v.x, v.y);
  }
  return *p;
}
template <bool NT>
__device__ inline float4 ld16(const float4* p) {
  if (NT) {
    const fvec4 v = __builtin_nontemporal_load(reinterpret_cast<const fvec4*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
  }
  return *p;
}
template <bool NT>
__device__ inline half4 ld8(const half4* p) {
  if (NT) return __builtin_nontemporal_load(p);
  return *p;
}

// Site-blocked layout: a field is a sequence of blocks of SB consecutive
// sites; inside a block, word k of every site is stored together (SB words of
// 16 bytes, 8 for FP16 links), so one wavefront reads each word of its 64
// sites from one contiguous 1 KiB run and every block of a field is one
// contiguous region. Word index of word k (of nw) of site i:
__device__ inline size_t widx(size_t i, int k, int nw) {
  return ((i / SB) * (size_t)nw + (size_t)k) * SB + (i % SB);
}

template <int P>
struct IO;

// ------------------------------------------------------------------ FP64
// spinor: 12 words (spin-major complex), link: 6 words (rows 0, 1), clover:
// 36 words (18 per chiral block)
template <>
struct IO<0> {
  using T = double;
  __device__ static inline void load_spinor(const void* f, size_t i, cx<T> s[12]) {
    const double2* b = reinterpret_cast<const double2*>(f);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      double2 v = b[widx(i, k, 12)];
      s[k] = {v.x, v.y};
    }
  }
  // sel 0: the whole spinor; sel 1: spins 0,1 into both halves; sel 2: spins
  // 2,3 into both halves (one instruction stream whatever the lane's sel)
  __device__ static inline void load_spinor_sel(const void* f, size_t i, int sel, cx<T> s[12]) {
    const double2* b = reinterpret_cast<const double2*>(f);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const int h = sel == 0 ? k / 6 : sel - 1;
      double2 v = b[widx(i, k % 6 + 6 * h, 12)];
      s[k] = {v.x, v.y};
    }
  }
  // spins 0,1 (upper = true) or spins 2,3 into s[0..5]
  __device__ static inline void load_half(const void* f, size_t i, bool upper, cx<T> s[6]) {
    const double2* b = reinterpret_cast<const double2*>(f);
    const int o = upper ? 0 : 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double2 v = b[widx(i, o + k, 12)];
      s[k] = {v.x, v.y};
    }
  }
  // the spinor as stored and its scale (1 here; FP16 fields store codes and a scale)
  __device__ static inline void load_spinor_codes(const void* f, size_t i, cx<T> s[12], T& scale) {
    load_spinor(f, i, s);
    scale = T(1);
  }
  __device__ static inline void load_half_codes(const void* f, size_t i, bool upper, cx<T> s[6], T& scale) {
    load_half(f, i, upper, s);
    scale = T(1);
  }
  __device__ static inline void store_spinor(void* f, size_t i, const cx<T> s[12]) {
    double2* b = reinterpret_cast<double2*>(f);
#pragma unroll
    for (int k = 0; k < 12; ++k) b[widx(i, k, 12)] = make_double2(s[k].r, s[k].i);
  }
  // words k with k % nl == lane (the lanes of one site share the stores)
  __device__ static inline void store_part(void* f, size_t i, const cx<T> s[12], int lane, int nl) {
    double2* b = reinterpret_cast<double2*>(f);
#pragma unroll
    for (int k = 0; k < 12; ++k)
      if (k % nl == lane) b[widx(i, k, 12)] = make_double2(s[k].r, s[k].i);
  }
  template <bool NT = false>
  __device__ static inline void load_link(const void* g, size_t i, cx<T> u[6]) {
    const double2* b = reinterpret_cast<const double2*>(g);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double2 v = ld16<NT>(b + widx(i, k, 6));
      u[k] = {v.x, v.y};
    }
  }
  // 18 complex slots of one chiral block (blk = 0: +, 1: -)
  template <bool NT = false>
  __device__ static inline void load_clover_block(const void* c, size_t i, int blk, cx<T> m[18]) {
    const double2* b = reinterpret_cast<const double2*>(c);
#pragma unroll
    for (int k = 0; k < 18; ++k) {
      double2 v = ld16<NT>(b + widx(i, blk * 18 + k, 36));
      m[k] = {v.x, v.y};
    }
  }
};

// ------------------------------------------------------------------ FP32
// spinor: 6 words of 2 complex, link: 3 words, clover: 18 words (9 per block)
template <>
struct IO<1> {
  using T = float;
  __device__ static inline void load_spinor(const void* f, size_t i, cx<T> s[12]) {
    const float4* b = reinterpret_cast<const float4*>(f);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float4 v = b[widx(i, k, 6)];
      s[2 * k] = {v.x, v.y};
      s[2 * k + 1] = {v.z, v.w};
    }
  }
  __device__ static inline void load_spinor_sel(const void* f, size_t i, int sel, cx<T> s[12]) {
    const float4* b = reinterpret_cast<const float4*>(f);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int h = sel == 0 ? k / 3 : sel - 1;
      float4 v = b[widx(i, k % 3 + 3 * h, 6)];
      s[2 * k] = {v.x, v.y};
      s[2 * k + 1] = {v.z, v.w};
    }
  }
  __device__ static inline void load_half(const void* f, size_t i, bool upper, cx<T> s[6]) {
    const float4* b = reinterpret_cast<const float4*>(f);
    const int o = upper ? 0 : 3;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float4 v = b[widx(i, o + k, 6)];
      s[2 * k] = {v.x, v.y};
      s[2 * k + 1] = {v.z, v.w};
    }
  }
  __device__ static inline void load_spinor_codes(const void* f, size_t i, cx<T> s[12], T& scale) {
    load_spinor(f, i, s);
    scale = T(1);
  }
  __device__ static inline void load_half_codes(const void* f, size_t i, bool upper, cx<T> s[6], T& scale) {
    load_half(f, i, upper, s);
    scale = T(1);
  }
  __device__ static inline void store_spinor(void* f, size_t i, const cx<T> s[12]) {
    float4* b = reinterpret_cast<float4*>(f);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      b[widx(i, k, 6)] = make_float4(s[2 * k].r, s[2 * k].i, s[2 * k + 1].r, s[2 * k + 1].i);
  }
  __device__ static inline void store_part(void* f, size_t i, const cx<T> s[12], int lane, int nl) {
    float4* b = reinterpret_cast<float4*>(f);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (k % nl == lane) b[widx(i, k, 6)] = make_float4(s[2 * k].r, s[2 * k].i, s[2 * k + 1].r, s[2 * k + 1].i);
  }
  template <bool NT = false>
  __device__ static inline void load_link(const void* g, size_t i, cx<T> u[6]) {
    const float4* b = reinterpret_cast<const float4*>(g);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float4 v = ld16<NT>(b + widx(i, k, 3));
      u[2 * k] = {v.x, v.y};
      u[2 * k + 1] = {v.z, v.w};
    }
  }
  template <bool NT = false>
  __device__ static inline void load_clover_block(const void* c, size_t i, int blk, cx<T> m[18]) {
    const float4* b = reinterpret_cast<const float4*>(c);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float4 v = ld16<NT>(b + widx(i, blk * 9 + k, 18));
      m[2 * k] = {v.x, v.y};
      m[2 * k + 1] = {v.z, v.w};
    }
  }
};

// ------------------------------------------------------------------ FP16
// spinor block: 3 words of 4 complex (half8, in units of the site's scale)
// for each of the SB sites, then the SB float scales (max |component|);
// link: 3 words of 8 bytes (half4); clover: 9 half8 words (36 complex)
template <>
struct IO<2> {
  using T = float;
  static constexpr size_t BLOCK_BYTES = SB * (3 * 16 + 4);
  __device__ static inline const half8* words(const void* f, size_t i) {
    return reinterpret_cast<const half8*>(reinterpret_cast<const char*>(f) + (i / SB) * BLOCK_BYTES) + (i % SB);
  }
  __device__ static inline half8* words(void* f, size_t i) {
    return reinterpret_cast<half8*>(reinterpret_cast<char*>(f) + (i / SB) * BLOCK_BYTES) + (i % SB);
  }
  __device__ static inline float* scale(const void* f, size_t i) {
    return reinterpret_cast<float*>(const_cast<char*>(reinterpret_cast<const char*>(f)) + (i / SB) * BLOCK_BYTES +
                                    3 * 16 * SB) + (i % SB);
  }
  __device__ static inline void load_spinor(const void* f, size_t i, cx<T> s[12]) {
    const half8* b = words(f, i);
    const float n = *scale(f, i);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      half8 v = b[k * SB];
#pragma unroll
      for (int j = 0; j < 4; ++j) s[4 * k + j] = {n * (float)v[2 * j], n * (float)v[2 * j + 1]};
    }
  }
  // the codes (the spinor in units of its scale) and the scale
  __device__ static inline void load_spinor_codes(const void* f, size_t i, cx<T> s[12], T& sc) {
    const half8* b = words(f, i);
    sc = *scale(f, i);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      half8 v = b[k * SB];
#pragma unroll
      for (int j = 0; j < 4; ++j) s[4 * k + j] = {(float)v[2 * j], (float)v[2 * j + 1]};
    }
  }
  // spins 0,1 (complex 0..5: word 0, first half of word 1) or spins 2,3
  // (second half of word 1, word 2), converting only those
  __device__ static inline void load_half_codes(const void* f, size_t i, bool upper, cx<T> s[6], T& sc) {
    const half8* b = words(f, i);
    sc = *scale(f, i);
    const half8 w1 = b[SB];
    const half8 w02 = b[upper ? 0 : 2 * SB];
    const int o = upper ? 0 : 2;
#pragma unroll
    for (int j = 0; j < 4; ++j) s[o + j] = {(float)w02[2 * j], (float)w02[2 * j + 1]};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int jj = upper ? j : j + 2;
      s[(upper ? 4 : 0) + j] = {(float)w1[2 * jj], (float)w1[2 * jj + 1]};
    }
  }
  // the FP16 words mix spins 1 and 2, so every selection loads the whole spinor
  __device__ static inline void load_spinor_sel(const void* f, size_t i, int, cx<T> s[12]) {
    load_spinor(f, i, s);
  }
  __device__ static inline void load_half(const void* f, size_t i, bool upper, cx<T> s[6]) {
    cx<T> all[12];
    load_spinor(f, i, all);
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] = all[(upper ? 0 : 6) + k];
  }
  // words 0..2 and the scale (as word 3), those with k % nl == lane
  __device__ static inline void store_part(void* f, size_t i, const cx<T> s[12], int lane, int nl) {
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(s[k].r), fabsf(s[k].i)));
    const float inv = m > 0.f ? 1.0f / m : 0.f;
    half8* b = words(f, i);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k % nl != lane) continue;
      half8 v;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[2 * j] = (_Float16)(s[4 * k + j].r * inv);
        v[2 * j + 1] = (_Float16)(s[4 * k + j].i * inv);
      }
      b[k * SB] = v;
    }
    if (3 % nl == lane) *scale(f, i) = m;
  }
  __device__ static inline void store_spinor(void* f, size_t i, const cx<T> s[12]) { store_part(f, i, s, 0, 1); }
  template <bool NT = false>
  __device__ static inline void load_link(const void* g, size_t i, cx<T> u[6]) {
    const half4* b = reinterpret_cast<const half4*>(g);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      half4 v = ld8<NT>(b + widx(i, k, 3));
      u[2 * k] = {(float)v[0], (float)v[1]};
      u[2 * k + 1] = {(float)v[2], (float)v[3]};
    }
  }
  // block + is complex 0..17 (words 0..4), block - is complex 18..35 (words 4..8)
  template <bool NT = false>
  __device__ static inline void load_clover_block(const void* c, size_t i, int blk, cx<T> m[18]) {
    const half8* b = reinterpret_cast<const half8*>(c);
    cx<T> part[20];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const half8* q = b + widx(i, blk * 4 + k, 9);
      half8 v = NT ? __builtin_nontemporal_load(q) : *q;
#pragma unroll
      for (int j = 0; j < 4; ++j) part[4 * k + j] = {(float)v[2 * j], (float)v[2 * j + 1]};
    }
    const int off = blk * 2;  // complex 18 is element 2 of word 4
#pragma unroll
    for (int k = 0; k < 18; ++k) m[k] = part[k + off];
  }
};

// Rebuild row 2 of an SU(3) matrix from rows 0, 1: row2 = conj(row0 x row1).
template <typename T>
__device__ inline void reconstruct(const cx<T> u[6], cx<T> r2[3]) {
  r2[0] = conj(u[1] * u[5] - u[2] * u[4]);
  r2[1] = conj(u[2] * u[3] - u[0] * u[5]);
  r2[2] = conj(u[0] * u[4] - u[1] * u[3]);
}

// y = M x for a Hermitian 6x6 block in the 18-slot packed form.
template <typename T>
__device__ inline void herm6_mul(const cx<T> m[18], const cx<T> x[6], cx<T> y[6]) {
  const T d[6] = {m[0].r, m[0].i, m[1].r, m[1].i, m[2].r, m[2].i};
#pragma unroll
  for (int a = 0; a < 6; ++a) y[a] = d[a] * x[a];
  int k = 3;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
#pragma unroll
    for (int b = a + 1; b < 6; ++b) {
      const cx<T> c = m[k++];
      y[a] = y[a] + c * x[b];
      y[b] = y[b] + cmulc(c, x[a]);
    }
  }
}

// out = A psi with A given by its two chiral blocks (1/2 of the basis change folded in).
template <int P>
__device__ inline void clover_apply(const void* clov, size_t i, const cx<typename IO<P>::T> in[12],
                                    cx<typename IO<P>::T> out[12]) {
  using T = typename IO<P>::T;
  cx<T> chp[6], chm[6], yp[6], ym[6], m[18];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    chp[k] = in[k] - in[k + 6];
    chm[k] = in[k] + in[k + 6];
  }
  IO<P>::template load_clover_block<false>(clov, i, 0, m);
  herm6_mul(m, chp, yp);
  IO<P>::template load_clover_block<false>(clov, i, 1, m);
  herm6_mul(m, chm, ym);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    out[k] = yp[k] + ym[k];
    out[k + 6] = ym[k] - yp[k];
  }
}

// Exchange with the neighbouring lane of a quad: CTRL = 0xB1 swaps lanes
// (0,1)(2,3), CTRL = 0x4E swaps (0,2)(1,3) (DPP quad permutations).
template <int CTRL>
__device__ inline float quad_swap(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double quad_swap(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}
// v(lane) + v(lane xor 32): the two halves of the wavefront swap values
// (v_permlane32_swap exchanges lanes 32..63 of its first operand with lanes
// 0..31 of its second, so the two results hold own + partner in every lane).
__device__ inline float half_sum(float v) {
  const int b = __builtin_bit_cast(int, v);
  const auto r = __builtin_amdgcn_permlane32_swap(b, b, false, false);
  return __builtin_bit_cast(float, (int)r[0]) + __builtin_bit_cast(float, (int)r[1]);
}
__device__ inline double half_sum(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = (int)(unsigned)(b & 0xffffffffull), hi = (int)(unsigned)(b >> 32);
  const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double a0 = __builtin_bit_cast(double, ((unsigned long long)(unsigned)rh[0] << 32) | (unsigned)rl[0]);
  const double a1 = __builtin_bit_cast(double, ((unsigned long long)(unsigned)rh[1] << 32) | (unsigned)rl[1]);
  return a0 + a1;
}
// Sum over the four lanes of a quad; every lane receives the total.
template <typename T>
__device__ inline T quad_sum(T v) {
  v += quad_swap<0xB1>(v);
  v += quad_swap<0x4E>(v);
  return v;
}

// blockIdx -> logical block: with remap on, each of the 8 XCDs (which receive
// blocks round-robin) gets one contiguous range of logical blocks, so that
// neighbouring sites share that XCD's L2.
__device__ inline int logical_block(int remap) {
  const int b = blockIdx.x;
  if (!remap) return b;
  const int nb = gridDim.x;
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd * q + (xcd < r ? xcd : r) + idx;
}

// Deterministic block reduction of N doubles: wavefront butterfly, then the
// waves' partials summed in wave order by thread 0. Result written to out[0..N).
template <int N>
__device__ inline void block_reduce(double v[N], double* out) {
  __shared__ double red[16][N > 0 ? N : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    v[k] = x;
  }
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) red[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[w][k];
      out[k] = s;
    }
  }
}

}  // namespace lq
