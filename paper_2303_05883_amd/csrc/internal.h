// Internal declarations of the gfx950 Wilson/clover library: lattice geometry,
// complex arithmetic, the native field layouts and the context.
//
// Native layouts (all fields are checkerboarded: one array per parity, site
// index i = x/2 + (Lx/2) * (y + Ly * (z + Lz * t)) among the sites of that
// parity). A site's data is a list of "words" of 16 bytes (8 for FP16 links).
// Fields are site-blocked: blocks of SB = 64 consecutive sites, and inside a
// block word k of all 64 sites stored together (word-major), so a wavefront
// reads each word of its 64 sites as one contiguous 1 KiB run and a block of
// a field is one contiguous region of memory (few DRAM pages and TLB entries
// per wavefront, where separate full-length planes would touch one page per
// word). The site count per parity is rounded up to a multiple of SB; the
// padding sites are never read or written.
//
//   spinor, 12 complex (index 3*spin + colour):
//     F64: 12 words of double2 (one complex each)
//     F32:  6 words of float4  (two complex each)
//     F16:  3 words of 8 x fp16 (four complex each) per site, then the block's
//           64 per-site scales s = max |re|, |im| over the 24 reals (float;
//           s = 0 for an all-zero site, whose codes are then all zero)
//   link, rows 0 and 1 of the SU(3) matrix (6 complex, index 3*row + col);
//     row 2 = conj(row0 x row1) is rebuilt in registers:
//     F64: 6 words of double2, F32: 3 words of float4, F16: 3 words of 4 x fp16
//     gauge[p][mu] holds U_mu(x) for the sites x of parity p.
//   clover, one parity: the site matrix A (or A^-1) in the chiral basis
//     chi_+ = psi_{0,1} - psi_{2,3}, chi_- = psi_{0,1} + psi_{2,3}, where it is
//     two Hermitian 6x6 blocks; the stored blocks carry the factor 1/2 of the
//     basis change. Per block 18 complex slots: slots 0..2 hold the real
//     diagonal as (d0,d1), (d2,d3), (d4,d5); slots 3..17 hold the upper
//     off-diagonal entries (i<j) in row-major order. Block + then block -.
//     F64: 36 words of double2, F32: 18 words of float4, F16: 9 words of 8 x fp16.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/lqcd.h"

namespace lq {

// ---------------------------------------------------------------- geometry
struct Geom {
  int lx, ly, lz, lt;
  int lxh;      // lx / 2
  int vh;       // sites per parity
  int t_bc;     // -1 antiperiodic, +1 periodic
};

// ---------------------------------------------------------------- complex
template <typename T>
struct cx {
  T r, i;
};

template <typename T>
__host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__host__ __device__ inline cx<T> operator-(cx<T> a) { return {-a.r, -a.i}; }
template <typename T>
__host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T>
__host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
// conj(a) * b
template <typename T>
__host__ __device__ inline cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
template <typename T>
__host__ __device__ inline cx<T> conj(cx<T> a) { return {a.r, -a.i}; }
// i * a and -i * a
template <typename T>
__host__ __device__ inline cx<T> mul_i(cx<T> a) { return {-a.i, a.r}; }
template <typename T>
__host__ __device__ inline cx<T> mul_mi(cx<T> a) { return {a.i, -a.r}; }

// ---------------------------------------------------------------- precisions
constexpr int SB = 64;  // sites per block of the site-blocked layout
// Sites per parity rounded up to whole blocks.
__host__ __device__ inline size_t padded_sites(size_t vh) { return (vh + SB - 1) / SB * SB; }
// Number of 16-byte words per site of each kind, per precision.
constexpr int spinor_words(int prec) { return prec == 0 ? 12 : (prec == 1 ? 6 : 3); }
constexpr int clover_words(int prec) { return prec == 0 ? 36 : (prec == 1 ? 18 : 9); }

// Bytes of one native half field (one parity) of the given precision.
__host__ __device__ inline size_t spinor_bytes(int prec, size_t vh) {
  return ((size_t)spinor_words(prec) * 16 + (prec == 2 ? 4 : 0)) * padded_sites(vh);
}
// Bytes of the links of one (parity, mu).
__host__ __device__ inline size_t link_bytes(int prec, size_t vh) {
  return (size_t)(prec == 2 ? 24 : (prec == 1 ? 48 : 96)) * padded_sites(vh);
}
__host__ __device__ inline size_t clover_bytes(int prec, size_t vh) {
  return (size_t)clover_words(prec) * 16 * padded_sites(vh);
}

// ---------------------------------------------------------------- context
struct Workspace;    // solver vectors, allocated on first use (solver.hip)

}  // namespace lq

struct lqcd_ctx {
  lq::Geom g;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  bool own_stream = false;
  int device = 0;
  void* noalloc_scratch = nullptr;  // this device's copy of the no-allocation scratch array

  // gauge[prec]: 2 parities x 4 directions x link_bytes
  void* gauge[3] = {nullptr, nullptr, nullptr};
  // clover per precision, slots 0: A on even, 1: A on odd, 2: A^-1 on even, 3: A^-1 on odd
  void* clov[3][4] = {};
  bool have_gauge = false;
  bool have_clover = false;
  bool is_wilson = true;   // c_SW == 0: A = 1, no clover storage used
  double kappa = 0.0;
  double csw = 0.0;

  // staging for canonical conversions
  void* canon_a = nullptr;   // 12 complex x V (full-lattice spinor)
  void* canon_b = nullptr;
  void* half_a[3] = {};      // native half fields per precision (scratch for apply)
  void* half_b[3] = {};
  void* half_c[3] = {};
  void* half_d[3] = {};
  double* dscal = nullptr;     // device scalars for small results
  double* hscal = nullptr;     // pinned host mirror

  // launch shape of the hop per precision (autotuned)
  int hop_block[3] = {256, 256, 256};
  int hop_remap[3] = {1, 1, 1};
  int hop_nt[3] = {0, 0, 0};     // non-temporal link loads
  int hop_split[3] = {1, 1, 1};  // lanes per output site: 1, 2 (forward / backward) or 4 (one direction each);
                                 // 0: plane march (hop_block = Lx/2 x rows lanes, hop_remap = z planes per block)

  lq::Workspace* ws = nullptr;
  // workspace of the last batched solve led by this context (reused when the
  // next batch has the same shape)
  void* batch = nullptr;
  void (*batch_free)(void*) = nullptr;
  // multigrid setup (test vectors, coarse operator); dropped when the gauge
  // field or the clover term changes
  void* mg = nullptr;
  void (*mg_free)(void*) = nullptr;
  // SAP: block residuals and last block updates (FP32 full fields, even half
  // then odd half), allocated on first use
  void* sap_res = nullptr;
  void* sap_delta = nullptr;
};

namespace lq {

// ---------------------------------------------------------------- errors
int set_error(int status, const std::string& msg);
#define LQ_HIP(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::lq::set_error(LQCD_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define LQ_TRY(call)            \
  do {                          \
    int s_ = (call);            \
    if (s_ != LQCD_OK) return s_; \
  } while (0)

// api.hip: the two canonical full-lattice staging vectors of a context
int ensure_canon(lqcd_ctx* c);

// ---------------------------------------------------------------- kernels (host launchers)
// layout.hip
int launch_import_spinor(lqcd_ctx* c, int prec, int parity, const double* canon, void* half);
int launch_export_spinor(lqcd_ctx* c, int prec, int parity, const void* half, double* canon);
int launch_zero_parity(lqcd_ctx* c, int parity, double* canon);
int launch_import_gauge(lqcd_ctx* c, const double* canon, double* check /* device, 3 doubles */);
int launch_convert_field(lqcd_ctx* c, int src_prec, const void* src, int dst_prec, void* dst);
int launch_check_finite(lqcd_ctx* c, const double* p, size_t n, double* flag);

// clover.hip
int build_clover(lqcd_ctx* c, double kappa, double csw);

// hop.hip
enum Epi { EPI_SCALE = 0, EPI_SCALE_CLOV = 1, EPI_XPAY = 2 };
enum Red { RED_NONE = 0, RED_DOT = 1, RED_TS = 2 };
struct HopCall {
  int prec;
  int out_parity;
  const void* in;       // half field, parity 1 - out_parity
  void* out;            // half field, parity out_parity
  int epi;
  double scale;         // multiplies H psi
  const void* clov;     // clover slot at the output parity (EPI_SCALE_CLOV, EPI_XPAY), or null = 1
  const void* xown;     // EPI_XPAY: own-parity input
  int red;
  const void* w;        // RED_DOT: <w, out>
  double* partials;     // RED_*: per-block partial sums
  const int* skip;      // optional device flag: when nonzero the launch does nothing
};
int launch_hop(lqcd_ctx* c, const HopCall& h, int* nblocks_out);
// Progress lines on stderr when LQCD_LOG is set (each outer pass, and every
// inner convergence check when LQCD_LOG=2).
inline int log_level() {
  const char* e = std::getenv("LQCD_LOG");
  return e ? std::atoi(e) : 0;
}

int hop_blocks(lqcd_ctx* c, int prec);
// Whether (block lanes, zc planes) is a valid plane-march shape on this lattice.
bool march_shape_ok(const Geom& g, int prec, int block, int zc);
// most blocks any hop launch shape uses (partials buffers are sized for it)
inline size_t max_hop_blocks(size_t vh) { return (vh + 15) / 16 + 8; }
// out = C x (C = clover slot, or identity -> copy)
int launch_site(lqcd_ctx* c, int prec, const void* clov, const void* in, void* out);

// blas.hip (declared in blas.h)

}  // namespace lq
