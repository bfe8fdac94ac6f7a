// Batched solves: several lattices of different sizes, each with several
// right-hand sides (e.g. the 12 spin-colour point sources of a propagator),
// solved together. Each right-hand side ("segment") runs its own BiCGStab (own
// rho, alpha, omega; not block Krylov), but every operator step of every
// unconverged segment of every lattice is ONE persistent kernel launch:
//
//  * the hop walks a tile list of (lattice, site block, group of right-hand
//    sides); a thread computes its site for every right-hand side of its
//    group, loading each link and clover block once for all of them, and the
//    groups of one site block are consecutive tiles in one of 8 contiguous
//    chunks, one per XCD (blocks reach the XCDs round-robin), so links are
//    reused from that XCD's L2 across groups too (the paper's motivation:
//    many equations on one gauge field, Sec. 3);
//  * vector updates and the fused reductions are batched the same way, with
//    per-segment partial sums and per-segment finalize blocks;
//  * converged segments are masked: their tiles return at once;
//  * check_every iterations of the whole batch are replayed from one captured
//    hipGraph.
// The FP64 defect-correction outer loop, the even-odd source preparation and
// the reconstruction run per segment with the single-field kernels.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "blascore.h"
#include "hopcore.h"
#include "internal.h"
#include "ops.h"
#include "solver.h"

namespace lq {

namespace {

enum Fld { F_R = 0, F_RHAT, F_P, F_V, F_S, F_T, F_Y, F_X, F_COUNT };

struct BLat {
  Geom g;
  const char* gauge;  // links of the inner precision
  size_t link_stride;
  const void* clov_e;     // A_ee (slot 0) or null
  const void* clov_oinv;  // A_oo^-1 (slot 3) or null
  double kappa;
  int tile0;   // first hop tile of this lattice
  int ntile;   // hop tiles: nsb * ceil(nrhs / NB)
  int nsb;     // hop site blocks
  int btile0;  // first blas tile
  int nbb;     // blas blocks
  int nrhs;
  int seg0;
};

struct BSeg {
  void* f[F_COUNT];
  Scal* sc;
  double* partials;
  int lat;
};

constexpr int MAXLAT = 16;
constexpr int BS = 256;
// right-hand sides per thread in the batched hop (links shared between them)
template <int P>
struct RhsBlock {
  static constexpr int NB = P == 0 ? 2 : 4;
};

struct BHopArgs {
  const BLat* lat;
  const BSeg* seg;
  int nlat;
  int in_sel, out_sel, own_sel, w_sel;
  int out_parity;
  int clov_slot;      // 0: A_ee, 3: A_oo^-1
  int scale_mode;     // 0: 1, 1: -kappa^2
  int bound[9];       // XCD chunk boundaries of the hop tile list
};

__device__ inline int find_lat(const BLat* lat, int nlat, int tile, bool blas) {
  int l = 0;
  for (int k = 1; k < nlat; ++k)
    if (tile >= (blas ? lat[k].btile0 : lat[k].tile0)) l = k;
  return l;
}

// Tiles are (lattice, site block, group of NB right-hand sides), groups
// fastest; each thread computes one site for the NB right-hand sides of its
// group (link and clover loads shared).
template <int P, int EPI, bool CLOV, int RED, bool NT, int NB>
__global__ void __launch_bounds__(BS) k_bhop(BHopArgs b) {
  constexpr int NR = RED == RED_DOT ? 2 : (RED == RED_TS ? 3 : 0);
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, nslot = gridDim.x >> 3;
  for (int t = b.bound[xcd] + slot; t < b.bound[xcd + 1]; t += nslot) {
    const int l = find_lat(b.lat, b.nlat, t, false);
    const BLat& L = b.lat[l];
    const int ngroup = (L.nrhs + NB - 1) / NB;
    const int local = t - L.tile0;
    const int sb = local / ngroup, grp = local % ngroup;
    MultiPtrs<NB> m;
    m.act = 0u;
    int segs[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int r = grp * NB + q;
      segs[q] = -1;
      m.in[q] = nullptr;
      m.out[q] = nullptr;
      m.own[q] = nullptr;
      m.w[q] = nullptr;
      if (r < L.nrhs) {
        const BSeg& S = b.seg[L.seg0 + r];
        segs[q] = L.seg0 + r;
        if (!S.sc->done) m.act |= 1u << q;  // uniform over the block
        m.in[q] = S.f[b.in_sel];
        m.out[q] = S.f[b.out_sel];
        m.own[q] = b.own_sel >= 0 ? S.f[b.own_sel] : nullptr;
        m.w[q] = b.w_sel >= 0 ? S.f[b.w_sel] : nullptr;
      }
    }
    if (m.act == 0u) continue;
    HopArgs a;
    a.in = nullptr;
    a.out = nullptr;
    a.gauge = L.gauge;
    a.link_stride = L.link_stride;
    a.clov = b.clov_slot == 0 ? L.clov_e : L.clov_oinv;
    a.xown = nullptr;
    a.w = nullptr;
    a.partials = nullptr;
    a.skip = nullptr;
    a.scale = b.scale_mode == 0 ? 1.0 : -L.kappa * L.kappa;
    a.g = L.g;
    a.p = b.out_parity;
    a.remap = 0;
    a.hz = 0;
    const size_t i = (size_t)sb * BS + threadIdx.x;
    double red[NB][3];
#pragma unroll
    for (int q = 0; q < NB; ++q) red[q][0] = red[q][1] = red[q][2] = 0.0;
    if (i < (size_t)L.g.vh) hop_site_multi<P, EPI, CLOV, RED, NT, NB>(a, m, i, red);
    if constexpr (NR > 0) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (!((m.act >> q) & 1u)) continue;
        block_reduce<NR>(red[q], b.seg[segs[q]].partials + (size_t)sb * NR);
        __syncthreads();
      }
    }
  }
}

enum BOp { B_P_UPDATE = 0, B_S_UPDATE, B_XR_UPDATE, B_START };

struct BBlasArgs {
  const BLat* lat;
  const BSeg* seg;
  int nlat;
  int ntile;
};

// Vector updates over every segment; tile = (segment, block of BS sites).
template <int P, int PX, int OP>
__global__ void __launch_bounds__(BS) k_bblas(BBlasArgs b) {
  for (int t = blockIdx.x; t < b.ntile; t += gridDim.x) {
    const int l = find_lat(b.lat, b.nlat, t, true);
    const BLat& L = b.lat[l];
    const int local = t - L.btile0;
    const int r = local / L.nbb, blk = local % L.nbb;
    const BSeg& S = b.seg[L.seg0 + r];
    if (OP != B_START && S.sc->done) continue;
    const size_t vh = (size_t)L.g.vh;
    const size_t i = (size_t)blk * BS + threadIdx.x;
    const bool act = i < vh;
    if (OP == B_P_UPDATE) {
      if (act) p_update_site<P>(S.f[F_R], S.f[F_P], S.f[F_V], S.sc, i);
    } else if (OP == B_S_UPDATE) {
      if (act) s_update_site<P>(S.f[F_R], S.f[F_V], S.f[F_S], S.sc, i);
    } else {
      double red[3] = {0.0, 0.0, 0.0};
      if (OP == B_XR_UPDATE) {
        if (act)
          xr_update_site<P, PX>(S.f[F_X], S.f[F_P], S.f[F_S], S.f[F_T], S.f[F_R], S.f[F_RHAT], S.sc, i, red);
      } else {  // start: rhat = p = r, <rhat, r>, <r, r>
        if (act) {
          copy_site<P>(S.f[F_R], S.f[F_RHAT], i);
          copy_site<P>(S.f[F_R], S.f[F_P], i);
          dot_norm_site<P>(S.f[F_R], S.f[F_R], i, red);
        }
      }
      block_reduce<3>(red, S.partials + (size_t)blk * 3);
      __syncthreads();
    }
  }
}

enum BFin { BF_ALPHA = 0, BF_OMEGA, BF_RHO, BF_INIT };

// One block per segment: finalize its reduction and update its scalars.
template <int OP>
__global__ void __launch_bounds__(1024) k_bfin(const BLat* lat, const BSeg* seg, const double* target2,
                                              int max_iters) {
  const BSeg& S = seg[blockIdx.x];
  const BLat& L = lat[S.lat];
  if (OP != BF_INIT && S.sc->done) return;
  if (OP == BF_ALPHA) {
    double v[2];
    sum_partials<2>(S.partials, L.nsb, v);
    if (threadIdx.x == 0) scal_alpha(S.sc, v);
  } else if (OP == BF_OMEGA) {
    double v[3];
    sum_partials<3>(S.partials, L.nsb, v);
    if (threadIdx.x == 0) scal_omega(S.sc, v);
  } else if (OP == BF_RHO) {
    double v[3];
    sum_partials<3>(S.partials, L.nbb, v);
    if (threadIdx.x == 0) scal_rho(S.sc, v);
  } else {
    double v[3];
    sum_partials<3>(S.partials, L.nbb, v);
    if (threadIdx.x == 0) scal_init(S.sc, v, target2[blockIdx.x], max_iters);
  }
}

// ------------------------------------------------------------------ host side

struct Batch {
  std::vector<lqcd_ctx*> ctx;
  std::vector<BLat> hlat;
  std::vector<BSeg> hseg;
  std::vector<int> seg_lat;
  BLat* dlat = nullptr;
  BSeg* dseg = nullptr;
  std::vector<void*> owned;  // device buffers
  // per segment FP64 fields: b_e, b_o, bhat, x_e, x_o, r64
  std::vector<std::array<void*, 6>> f64;
  double* snorm = nullptr;   // device: 16 doubles per segment
  double* htmp = nullptr;    // pinned host mirror
  double* dtarget = nullptr; // device: per-segment target2 of the inner solve
  Scal* hscal = nullptr;     // pinned host copies of the segments' Scal
  int prec = 1, xprec = 1;
  int hop_tiles = 0, blas_tiles = 0;
  int bound[9] = {};
  bool clover = false;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_k = 0;
  // shape key: (sites per parity, nrhs) per lattice, inner precision, clover
  std::vector<std::pair<int, int>> key;
  Scal* dscal_all = nullptr;
  bool ready = false;  // every buffer allocated

  ~Batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void* p : owned) (void)hipFree(p);
    if (htmp) (void)hipHostFree(htmp);
    if (hscal) (void)hipHostFree(hscal);
  }
  int dev_alloc(void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();
      return set_error(LQCD_ENOMEM, "batch workspace allocation of " + std::to_string(bytes) + " bytes failed");
    }
    owned.push_back(*p);
    return LQCD_OK;
  }
};

int batch_hop(Batch& B, hipStream_t s, int in_sel, int out_sel, int own_sel, int w_sel, int parity, int epi,
              int red, int clov_slot, int scale_mode) {
  BHopArgs a;
  a.lat = B.dlat;
  a.seg = B.dseg;
  a.nlat = (int)B.hlat.size();
  a.in_sel = in_sel;
  a.out_sel = out_sel;
  a.own_sel = own_sel;
  a.w_sel = w_sel;
  a.out_parity = parity;
  a.clov_slot = clov_slot;
  a.scale_mode = scale_mode;
  for (int k = 0; k < 9; ++k) a.bound[k] = B.bound[k];
  const int grid = 8 * 256;  // persistent: 256 blocks per XCD
  const bool cl = B.clover;
#define LQ_BHOP(P)                                                                                       \
  if (epi == EPI_SCALE_CLOV) {                                                                           \
    if (cl) hipLaunchKernelGGL((k_bhop<P, EPI_SCALE_CLOV, true, RED_NONE, true, RhsBlock<P>::NB>), dim3(grid), dim3(BS), 0, s, a); \
    else hipLaunchKernelGGL((k_bhop<P, EPI_SCALE, false, RED_NONE, true, RhsBlock<P>::NB>), dim3(grid), dim3(BS), 0, s, a);      \
  } else if (red == RED_DOT) {                                                                           \
    if (cl) hipLaunchKernelGGL((k_bhop<P, EPI_XPAY, true, RED_DOT, true, RhsBlock<P>::NB>), dim3(grid), dim3(BS), 0, s, a);        \
    else hipLaunchKernelGGL((k_bhop<P, EPI_XPAY, false, RED_DOT, true, RhsBlock<P>::NB>), dim3(grid), dim3(BS), 0, s, a);          \
  } else {                                                                                               \
    if (cl) hipLaunchKernelGGL((k_bhop<P, EPI_XPAY, true, RED_TS, true, RhsBlock<P>::NB>), dim3(grid), dim3(BS), 0, s, a);         \
    else hipLaunchKernelGGL((k_bhop<P, EPI_XPAY, false, RED_TS, true, RhsBlock<P>::NB>), dim3(grid), dim3(BS), 0, s, a);           \
  }
  if (B.prec == 1) {
    LQ_BHOP(1)
  } else if (B.prec == 2) {
    LQ_BHOP(2)
  } else {
    LQ_BHOP(0)
  }
#undef LQ_BHOP
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

template <int OP>
int batch_blas_t(Batch& B, hipStream_t s) {
  BBlasArgs a{B.dlat, B.dseg, (int)B.hlat.size(), B.blas_tiles};
  const int grid = std::min(B.blas_tiles, 8 * 512);
  if (B.prec == 1) hipLaunchKernelGGL((k_bblas<1, 1, OP>), dim3(grid), dim3(BS), 0, s, a);
  else if (B.prec == 2) hipLaunchKernelGGL((k_bblas<2, 1, OP>), dim3(grid), dim3(BS), 0, s, a);
  else hipLaunchKernelGGL((k_bblas<0, 0, OP>), dim3(grid), dim3(BS), 0, s, a);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

template <int OP>
int batch_fin(Batch& B, hipStream_t s, int max_iters) {
  hipLaunchKernelGGL((k_bfin<OP>), dim3((unsigned)B.hseg.size()), dim3(1024), 0, s, B.dlat, B.dseg, B.dtarget,
                     max_iters);
  LQ_HIP(hipGetLastError());
  return LQCD_OK;
}

// One BiCGStab iteration of every segment (after p is known).
int batch_iteration(Batch& B, hipStream_t s) {
  LQ_TRY(batch_hop(B, s, F_P, F_Y, -1, -1, 1, EPI_SCALE_CLOV, RED_NONE, 3, 0));
  LQ_TRY(batch_hop(B, s, F_Y, F_V, F_P, F_RHAT, 0, EPI_XPAY, RED_DOT, 0, 1));
  LQ_TRY(batch_fin<BF_ALPHA>(B, s, 0));
  LQ_TRY(batch_blas_t<B_S_UPDATE>(B, s));
  LQ_TRY(batch_hop(B, s, F_S, F_Y, -1, -1, 1, EPI_SCALE_CLOV, RED_NONE, 3, 0));
  LQ_TRY(batch_hop(B, s, F_Y, F_T, F_S, -1, 0, EPI_XPAY, RED_TS, 0, 1));
  LQ_TRY(batch_fin<BF_OMEGA>(B, s, 0));
  LQ_TRY(batch_blas_t<B_XR_UPDATE>(B, s));
  LQ_TRY(batch_fin<BF_RHO>(B, s, 0));
  return batch_blas_t<B_P_UPDATE>(B, s);
}

int batch_chunk(Batch& B, lqcd_ctx* c0, int k, bool use_graph) {
  if (!use_graph) {
    for (int j = 0; j < k; ++j) LQ_TRY(batch_iteration(B, B.stream));
    return LQCD_OK;
  }
  if (!B.exec || B.graph_k != k) {
    if (B.exec) (void)hipGraphExecDestroy(B.exec);
    if (B.graph) (void)hipGraphDestroy(B.graph);
    B.exec = nullptr;
    B.graph = nullptr;
    if (!c0->cap_stream) LQ_HIP(hipStreamCreateWithFlags(&c0->cap_stream, hipStreamNonBlocking));
    LQ_HIP(hipStreamBeginCapture(c0->cap_stream, hipStreamCaptureModeThreadLocal));
    int st = LQCD_OK;
    for (int j = 0; j < k && st == LQCD_OK; ++j) st = batch_iteration(B, c0->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c0->cap_stream, &g);
    if (st != LQCD_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return set_error(LQCD_EHIP, std::string("batch graph capture: ") + hipGetErrorString(e));
    B.graph = g;
    LQ_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
    B.graph_k = k;
  }
  LQ_HIP(hipGraphLaunch(B.exec, B.stream));
  return LQCD_OK;
}

// r64 = b' - S x_e (FP64) for one segment; |r64|^2, 1/|r64|, |r64| into dst[0..2]
int seg_residual(lqcd_ctx* c, const std::array<void*, 6>& f, double* dst) {
  Workspace* w = c->ws;
  double* part = w->inner[0].r ? w->inner[0].partials : w->inner[1].r ? w->inner[1].partials : w->inner[2].partials;
  LQ_TRY(op_schur(c, 0, f[3], w->v64, w->y64, RED_NONE, nullptr, nullptr, nullptr, nullptr));
  LQ_TRY(blas_sub_norm(c, f[2], w->v64, f[5], part));
  return fin_norm(c, dst, part, blas_blocks(c->g.vh), 1, 0);
}

int seg_norm(lqcd_ctx* c, const void* a, double* dst) {
  Workspace* w = c->ws;
  double* part = w->inner[0].r ? w->inner[0].partials : w->inner[1].r ? w->inner[1].partials : w->inner[2].partials;
  LQ_TRY(blas_dot_norm(c, 0, a, a, part));
  return fin_norm(c, dst, part, blas_blocks(c->g.vh), 3, 2);
}

void free_batch(void* p) { delete reinterpret_cast<Batch*>(p); }

}  // namespace

}  // namespace lq

using namespace lq;

extern "C" int lqcd_solve_batch(lqcd_ctx* const* ctxs, const int* nrhs, const double* const* b, double* const* x,
                                int nlattices, const lqcd_solve_params* prm_in, lqcd_solve_stats* stats) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  if (!ctxs || !nrhs || !b || !x || nlattices < 1 || nlattices > MAXLAT)
    return set_error(LQCD_EINVAL, "bad batch arguments (1 to 16 lattices)");
  lqcd_solve_params prm;
  if (prm_in) prm = *prm_in;
  else lqcd_default_params(&prm);
  if (!(prm.tol > 0) || prm.inner_prec < 0 || prm.inner_prec > 2 || prm.max_iter < 1 || prm.max_outer < 1)
    return set_error(LQCD_EINVAL, "bad solver parameters");
  if (prm.x0) return set_error(LQCD_EINVAL, "batched solves start from x = 0");
  if (prm.even_odd != 1) return set_error(LQCD_EINVAL, "batched solves are even-odd preconditioned");
  hipStream_t stream = ctxs[0] ? ctxs[0]->stream : nullptr;
  bool clover = false;
  for (int l = 0; l < nlattices; ++l) {
    lqcd_ctx* c = ctxs[l];
    if (!c || !b[l] || !x[l] || nrhs[l] < 1) return set_error(LQCD_EINVAL, "null context, vector or nrhs < 1");
    if (!c->have_gauge || !c->have_clover) return set_error(LQCD_ESTATE, "set_gauge and set_clover must come first");
    if (c->stream != stream) return set_error(LQCD_EINVAL, "all contexts of a batch must share one stream");
    if (l == 0) clover = !c->is_wilson;
    else if (clover != !c->is_wilson) return set_error(LQCD_EINVAL, "a batch is all clover or all Wilson");
    for (int m = 0; m < l; ++m)
      if (ctxs[m] == c) return set_error(LQCD_EINVAL, "a context appears twice in the batch");
  }
  const int IP = prm.inner_prec;
  std::vector<std::pair<int, int>> key;
  for (int l = 0; l < nlattices; ++l) key.push_back({ctxs[l]->g.vh, nrhs[l]});
  key.push_back({IP, clover ? 1 : 0});
  lqcd_ctx* lead = ctxs[0];
  Batch* cached = reinterpret_cast<Batch*>(lead->batch);
  const bool reuse = cached && cached->ready && cached->key == key;
  if (!reuse && cached) {
    (void)hipStreamSynchronize(stream);
    lead->batch_free(cached);
    lead->batch = nullptr;
    lead->batch_free = nullptr;
  }
  if (!reuse) {
    lead->batch = new Batch();
    lead->batch_free = free_batch;
  }
  Batch& B = *reinterpret_cast<Batch*>(lead->batch);
  B.stream = stream;
  B.prec = IP;
  B.xprec = IP == 2 ? 1 : IP;
  B.clover = clover;
  const int check = prm.check_every > 0 ? prm.check_every : 8;
  const double delta = prm.inner_tol > 0 ? prm.inner_tol : (IP == 1 ? 1e-6 : (IP == 2 ? 1e-2 : 1e-10));

  // descriptors (rebuilt every call from the current contexts) and buffers
  // (allocated when the batch shape is new)
  int total_seg = 0;
  for (int l = 0; l < nlattices; ++l) total_seg += nrhs[l];
  if (!reuse) {
    B.key = key;
    LQ_TRY(B.dev_alloc(reinterpret_cast<void**>(&B.dscal_all), (size_t)total_seg * sizeof(Scal)));
  }
  Scal* dscal_all = B.dscal_all;
  B.hlat.clear();
  B.ctx.clear();
  int tile = 0, btile = 0, seg = 0;
  for (int l = 0; l < nlattices; ++l) {
    lqcd_ctx* c = ctxs[l];
    LQ_TRY(ensure_workspace(c, 0));
    BLat L{};
    L.g = c->g;
    L.gauge = reinterpret_cast<const char*>(c->gauge[IP]);
    L.link_stride = link_bytes(IP, c->g.vh);
    L.clov_e = clover ? c->clov[IP][0] : nullptr;
    L.clov_oinv = clover ? c->clov[IP][3] : nullptr;
    L.kappa = c->kappa;
    L.nsb = (c->g.vh + BS - 1) / BS;
    L.nbb = L.nsb;
    L.nrhs = nrhs[l];
    L.tile0 = tile;
    {
      const int nbk = IP == 0 ? RhsBlock<0>::NB : RhsBlock<1>::NB;
      L.ntile = L.nsb * ((L.nrhs + nbk - 1) / nbk);
    }
    L.btile0 = btile;
    L.seg0 = seg;
    tile += L.ntile;
    btile += L.nbb * L.nrhs;
    B.hlat.push_back(L);
    B.ctx.push_back(c);
    for (int r = 0; r < nrhs[l]; ++r, ++seg) {
      if (reuse) continue;
      BSeg S{};
      const size_t vh = c->g.vh;
      for (int f = 0; f < F_COUNT; ++f)
        LQ_TRY(B.dev_alloc(&S.f[f], spinor_bytes(f == F_X ? B.xprec : IP, vh)));
      S.sc = dscal_all + seg;
      LQ_TRY(B.dev_alloc(reinterpret_cast<void**>(&S.partials), (size_t)L.nsb * 3 * sizeof(double)));
      S.lat = l;
      B.hseg.push_back(S);
      B.seg_lat.push_back(l);
      std::array<void*, 6> f64{};
      for (auto& p : f64) LQ_TRY(B.dev_alloc(&p, spinor_bytes(0, vh)));
      B.f64.push_back(f64);
    }
  }
  const int nseg = seg;
  B.hop_tiles = tile;
  B.blas_tiles = btile;
  for (int k = 0; k <= 8; ++k) B.bound[k] = (int)((long long)tile * k / 8);
  if (!reuse) {
    LQ_TRY(B.dev_alloc(reinterpret_cast<void**>(&B.dlat), B.hlat.size() * sizeof(BLat)));
    LQ_TRY(B.dev_alloc(reinterpret_cast<void**>(&B.dseg), B.hseg.size() * sizeof(BSeg)));
    LQ_TRY(B.dev_alloc(reinterpret_cast<void**>(&B.snorm), (size_t)nseg * 16 * sizeof(double)));
    LQ_TRY(B.dev_alloc(reinterpret_cast<void**>(&B.dtarget), (size_t)nseg * sizeof(double)));
    if (hipHostMalloc(reinterpret_cast<void**>(&B.htmp), (size_t)nseg * 16 * sizeof(double)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&B.hscal), (size_t)nseg * sizeof(Scal)) != hipSuccess)
      return set_error(LQCD_ENOMEM, "pinned host allocation failed");
    B.ready = true;
  }
  LQ_HIP(hipMemcpyAsync(B.dlat, B.hlat.data(), B.hlat.size() * sizeof(BLat), hipMemcpyHostToDevice, stream));
  LQ_HIP(hipMemcpyAsync(B.dseg, B.hseg.data(), B.hseg.size() * sizeof(BSeg), hipMemcpyHostToDevice, stream));

  // import and prepare every segment: b', |b|^2, x = 0, r = b'
  for (int s = 0; s < nseg; ++s) {
    lqcd_ctx* c = B.ctx[B.seg_lat[s]];
    const auto& f = B.f64[s];
    const int l = B.seg_lat[s];
    const int r = s - B.hlat[l].seg0;
    const size_t n = (size_t)c->g.vh * 2 * 24;
    const double* bs = b[l] + (size_t)r * n;
    const double* db = bs;
    if (!prm.on_device) {
      LQ_TRY(ensure_canon(c));
      LQ_HIP(hipMemcpyAsync(c->canon_a, bs, n * sizeof(double), hipMemcpyHostToDevice, stream));
      db = reinterpret_cast<const double*>(c->canon_a);
    }
    LQ_TRY(launch_import_spinor(c, 0, 0, db, f[0]));
    LQ_TRY(launch_import_spinor(c, 0, 1, db, f[1]));
    double* nrm = B.snorm + 16 * s;
    LQ_TRY(seg_norm(c, f[0], nrm + 0));
    LQ_TRY(seg_norm(c, f[1], nrm + 3));
    const void* ainv_o = clover_slot(c, 0, 3);
    Workspace* w = c->ws;
    const void* src_o = f[1];
    if (ainv_o) {
      LQ_TRY(launch_site(c, 0, ainv_o, f[1], w->y64));
      src_o = w->y64;
    }
    LQ_TRY(op_hop_xpay(c, 0, 0, src_o, f[0], nullptr, f[2], c->kappa));
    LQ_TRY(blas_zero(c, 0, f[3]));
    LQ_TRY(seg_residual(c, f, nrm + 6));
  }
  LQ_HIP(hipMemcpyAsync(B.htmp, B.snorm, (size_t)nseg * 16 * sizeof(double), hipMemcpyDeviceToHost, stream));
  LQ_HIP(hipStreamSynchronize(stream));
  std::vector<double> bnorm2(nseg), target(nseg), rnorm(nseg);
  std::vector<int> inner_it(nseg, 0), outer_it(nseg, 0), restarts(nseg, 0), fails(nseg, 0);
  for (int s = 0; s < nseg; ++s) {
    bnorm2[s] = B.htmp[16 * s] + B.htmp[16 * s + 3];
    target[s] = prm.tol * std::sqrt(bnorm2[s]);
    rnorm[s] = B.htmp[16 * s + 8];
  }
  const double t_setup0 = std::chrono::duration<double>(clk::now() - t0).count();

  int status = LQCD_OK;
  int total_inner = 0;
  for (;;) {
    std::vector<int> active;
    for (int s = 0; s < nseg; ++s)
      if (bnorm2[s] > 0 && rnorm[s] > target[s] && fails[s] <= 5) active.push_back(s);
    if (active.empty()) break;
    int max_outer = 0;
    for (int s : active) max_outer = std::max(max_outer, outer_it[s]);
    if (max_outer >= prm.max_outer || total_inner >= prm.max_iter) {
      status = set_error(LQCD_ENOCONV, "batched solve did not reach the tolerance");
      break;
    }
    // inner right-hand sides r / |r| (zero for the segments that are done) and targets
    std::vector<double> t2(nseg, 1e300);
    for (int s = 0; s < nseg; ++s) {
      lqcd_ctx* c = B.ctx[B.seg_lat[s]];
      const BSeg& S = B.hseg[s];
      const bool act = std::find(active.begin(), active.end(), s) != active.end();
      if (act) {
        LQ_TRY(blas_scale_down(c, IP, B.f64[s][5], S.f[F_R], B.snorm + 16 * s + 7, 0.0));
        double d = delta;
        const double need = target[s] / rnorm[s];
        if (need > d) d = need * 0.5;
        t2[s] = d * d;
      } else {
        LQ_TRY(blas_zero(c, IP, S.f[F_R]));
      }
      LQ_TRY(blas_zero(c, B.xprec, S.f[F_X]));
    }
    LQ_HIP(hipMemcpyAsync(B.dtarget, t2.data(), nseg * sizeof(double), hipMemcpyHostToDevice, stream));
    LQ_TRY(batch_blas_t<B_START>(B, stream));
    LQ_TRY(batch_fin<BF_INIT>(B, stream, prm.max_iter - total_inner));
    // iterate until every segment's inner solve is done
    for (;;) {
      LQ_HIP(hipMemcpyAsync(B.hscal, dscal_all, (size_t)nseg * sizeof(Scal), hipMemcpyDeviceToHost, stream));
      LQ_HIP(hipStreamSynchronize(stream));
      bool all = true;
      for (int s = 0; s < nseg; ++s) all = all && B.hscal[s].done;
      if (all) break;
      LQ_TRY(batch_chunk(B, ctxs[0], check, prm.use_graph != 0));
    }
    int most = 0;
    for (int s : active) {
      inner_it[s] += B.hscal[s].iters;
      most = std::max(most, B.hscal[s].iters);
      outer_it[s] += 1;
      if (B.hscal[s].breakdown) ++restarts[s];
    }
    total_inner += most;
    // x += |r| e; new FP64 residual
    for (int s : active) {
      lqcd_ctx* c = B.ctx[B.seg_lat[s]];
      LQ_TRY(blas_accum_up(c, B.xprec, B.f64[s][3], B.hseg[s].f[F_X], B.snorm + 16 * s + 8));
      LQ_TRY(seg_residual(c, B.f64[s], B.snorm + 16 * s + 6));
    }
    LQ_HIP(hipMemcpyAsync(B.htmp, B.snorm, (size_t)nseg * 16 * sizeof(double), hipMemcpyDeviceToHost, stream));
    LQ_HIP(hipStreamSynchronize(stream));
    for (int s : active) {
      const double prev = rnorm[s];
      rnorm[s] = B.htmp[16 * s + 8];
      if (!(rnorm[s] < prev)) ++fails[s];
    }
    if (std::getenv("LQCD_LOG")) {
      double worst = 0.0;
      for (int s = 0; s < nseg; ++s)
        if (bnorm2[s] > 0) worst = std::max(worst, rnorm[s] / std::sqrt(bnorm2[s]));
      std::fprintf(stderr, "[lqcd] batch outer pass: %zu active, %d inner iterations so far, worst |r|/|b| %.3e\n",
                   active.size(), total_inner, worst);
    }
  }
  for (int s = 0; s < nseg; ++s)
    if (fails[s] > 5 && status == LQCD_OK) status = set_error(LQCD_EBREAKDOWN, "a batched right-hand side stagnated");

  // reconstruction, true residuals, export
  const auto t_rec = clk::now();
  for (int s = 0; s < nseg; ++s) {
    lqcd_ctx* c = B.ctx[B.seg_lat[s]];
    const auto& f = B.f64[s];
    Workspace* w = c->ws;
    const int l = B.seg_lat[s];
    const int r = s - B.hlat[l].seg0;
    const size_t n = (size_t)c->g.vh * 2 * 24;
    const void* ainv_o = clover_slot(c, 0, 3);
    if (bnorm2[s] == 0.0) {
      LQ_TRY(blas_zero(c, 0, f[3]));
      LQ_TRY(blas_zero(c, 0, f[4]));
    } else if (ainv_o) {
      LQ_TRY(op_hop_xpay(c, 0, 1, f[3], f[1], nullptr, w->y64, c->kappa));
      LQ_TRY(launch_site(c, 0, ainv_o, w->y64, f[4]));
    } else {
      LQ_TRY(op_hop_xpay(c, 0, 1, f[3], f[1], nullptr, f[4], c->kappa));
    }
    LQ_TRY(op_full(c, 0, f[3], f[4], w->v64, w->y64));
    double* part = w->inner[0].partials;
    double* nrm = B.snorm + 16 * s;
    LQ_TRY(blas_sub_norm(c, f[0], w->v64, w->v64, part));
    LQ_TRY(fin_norm(c, nrm + 9, part, blas_blocks(c->g.vh), 1, 0));
    LQ_TRY(blas_sub_norm(c, f[1], w->y64, w->y64, part));
    LQ_TRY(fin_norm(c, nrm + 12, part, blas_blocks(c->g.vh), 1, 0));
    double* xs = x[l] + (size_t)r * n;
    if (!prm.on_device) LQ_TRY(ensure_canon(c));
    double* dx = prm.on_device ? xs : reinterpret_cast<double*>(c->canon_b);
    LQ_TRY(launch_export_spinor(c, 0, 0, f[3], dx));
    LQ_TRY(launch_export_spinor(c, 0, 1, f[4], dx));
    if (!prm.on_device) {
      LQ_HIP(hipMemcpyAsync(xs, dx, n * sizeof(double), hipMemcpyDeviceToHost, stream));
      LQ_HIP(hipStreamSynchronize(stream));
    }
  }
  LQ_HIP(hipMemcpyAsync(B.htmp, B.snorm, (size_t)nseg * 16 * sizeof(double), hipMemcpyDeviceToHost, stream));
  LQ_HIP(hipStreamSynchronize(stream));
  const auto t1 = clk::now();
  const double total_s = std::chrono::duration<double>(t1 - t0).count();
  const double setup_s = t_setup0 + std::chrono::duration<double>(t1 - t_rec).count();
  if (stats)
    for (int s = 0; s < nseg; ++s) {
      lqcd_solve_stats& st = stats[s];
      st.outer_iters = outer_it[s];
      st.inner_iters = inner_it[s];
      st.restarts = restarts[s];
      st.true_rel_resid = bnorm2[s] > 0 ? std::sqrt((B.htmp[16 * s + 9] + B.htmp[16 * s + 12]) / bnorm2[s]) : 0.0;
      st.seconds_solve = total_s;
      st.seconds_setup = setup_s;
    }
  return status;
}
