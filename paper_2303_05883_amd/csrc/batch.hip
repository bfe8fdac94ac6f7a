// Batched solves: several lattices of different sizes, each with several
// right-hand sides (e.g. the 12 spin-colour point sources of a propagator),
// solved together. Each right-hand side ("segment") runs its own BiCGStab (own
// rho, alpha, omega; not block Krylov), but every operator step of every
// unconverged segment of every lattice is ONE persistent kernel launch:
//
//  * the hop (bhop.h) walks a tile list of (lattice, 64-site block); the
//    wavefronts of a workgroup take the groups of right-hand sides of its tile
//    and a lane computes its site for the nb right-hand sides of its group,
//    so links and clover blocks come from HBM once per site for all
//    right-hand sides of the lattice (the paper's motivation: many equations
//    on one gauge field, Sec. 3);
//  * its launch shape (right-hand sides per lane, wavefronts per workgroup,
//    workgroups per XCD) is picked by timing the candidates on the batch
//    itself the first time a batch shape is seen, and kept in the tune cache;
//  * vector updates and the fused reductions are batched the same way, with
//    per-segment partial sums and per-segment finalize blocks;
//  * converged segments are masked: their waves skip the work;
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
#include <sstream>
#include <string>
#include <vector>

#include "bhop.h"
#include "blascore.h"
#include "internal.h"
#include "ops.h"
#include "solver.h"
#include "tune.h"

namespace lq {

namespace {

constexpr int MAXLAT = 16;
constexpr int BS = 256;  // sites per workgroup of the batched vector updates

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

// kinds of batched hop, each with a launch shape of its own
enum BKind { BK_SC = 0, BK_DOT = 1, BK_TS = 2, BK_N = 3 };

inline int bkind(int epi, int red) { return epi != EPI_XPAY ? BK_SC : (red == RED_DOT ? BK_DOT : BK_TS); }

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
  int bound[BK_N][9] = {};
  bool clover = false;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_k = 0;
  // shape key: (sites per parity, nrhs) per lattice, inner precision, clover
  std::vector<std::pair<int, int>> key;
  Scal* dscal_all = nullptr;
  bool ready = false;  // every buffer allocated
  // launch shape and device tile list of each kind of batched hop (the
  // A_oo^-1 H_oe hop, the XPAY hop with <rhat, v>, the XPAY hop with <t, s>
  // and <t, t>): the XPAY forms hold more registers and are tuned apart
  BShape shape[BK_N];
  bool tuned = false;           // shapes chosen for this batch
  int2* dtiles[BK_N] = {};      // device tile lists of the current shapes
  size_t tile_cap = 0;          // capacity of each (tiles of the largest shape)
  std::vector<int2> htiles[BK_N];
  double hop_us = 0;  // average duration of the A_oo^-1 H_oe hop when timed (microseconds)
  int max_rhs = 1;

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
  const int kind = bkind(epi, red);
  a.tiles = B.dtiles[kind];
  a.nlat = (int)B.hlat.size();
  a.in_sel = in_sel;
  a.out_sel = out_sel;
  a.own_sel = own_sel;
  a.w_sel = w_sel;
  a.out_parity = parity;
  a.clov_slot = clov_slot;
  a.scale_mode = scale_mode;
  for (int k = 0; k < 9; ++k) a.bound[k] = B.bound[kind][k];
  if (B.prec == 1) return launch_bhop<1>(a, B.shape[kind], epi, red, B.clover, s);
  if (B.prec == 2) return launch_bhop<2>(a, B.shape[kind], epi, red, B.clover, s);
  return launch_bhop<0>(a, B.shape[kind], epi, red, B.clover, s);
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

// Make sh the batch's launch shape: the tile list of its walk and group sets,
// dealt to the XCDs in 8 contiguous chunks, uploaded (on the batch's stream)
// and a captured iteration graph dropped (its launches hold the old shape).
int set_shape(Batch& B, int kind, const BShape& sh) {
  std::vector<int2>& tl = B.htiles[kind];
  tl.clear();
  for (int k = 0; k < 8; ++k) {
    B.bound[kind][k] = (int)tl.size();
    for (size_t l = 0; l < B.hlat.size(); ++l) {
      const BLat& L = B.hlat[l];
      const int ngroup = (L.nrhs + sh.nb - 1) / sh.nb;
      const int nset = (ngroup + sh.nw - 1) / sh.nw;
      const size_t vh = L.g.vh;
      const size_t per_t = vh / (size_t)L.g.lt;  // sites of one parity in a time slice
      auto push = [&](int blk) {
        for (int gs = 0; gs < nset; ++gs) tl.push_back(make_int2((int)l | (gs << 8), blk));
      };
      if (sh.walk >= 1 && per_t % SB == 0) {
        // slab walk: this XCD's range of blocks in every time slice, slices in
        // order; walk w > 1 cuts the range into 2^(w-1) sub-ranges walked one
        // after the other (a smaller working set per time step)
        const int nbt = (int)(per_t / SB);
        const int lo = (int)((long long)nbt * k / 8), hi = (int)((long long)nbt * (k + 1) / 8);
        const int nsub = 1 << (sh.walk - 1);
        for (int q = 0; q < nsub; ++q) {
          const int slo = lo + (int)((long long)(hi - lo) * q / nsub);
          const int shi = lo + (int)((long long)(hi - lo) * (q + 1) / nsub);
          for (int t = 0; t < L.g.lt; ++t)
            for (int bb = slo; bb < shi; ++bb) push(t * nbt + bb);
        }
      } else {
        const int lo = (int)((long long)L.nsb * k / 8), hi = (int)((long long)L.nsb * (k + 1) / 8);
        for (int bb = lo; bb < hi; ++bb) push(bb);
      }
    }
  }
  B.bound[kind][8] = (int)tl.size();
  if (tl.size() > B.tile_cap) return set_error(LQCD_EINVAL, "batched hop tile list exceeds its buffer");
  LQ_HIP(hipMemcpyAsync(B.dtiles[kind], tl.data(), tl.size() * sizeof(int2), hipMemcpyHostToDevice, B.stream));
  B.shape[kind] = sh;
  if (B.exec) {
    (void)hipStreamSynchronize(B.stream);
    (void)hipGraphExecDestroy(B.exec);
    B.exec = nullptr;
  }
  if (B.graph) {
    (void)hipGraphDestroy(B.graph);
    B.graph = nullptr;
  }
  return LQCD_OK;
}

// Check a batch's contexts (one stream, all clover or all Wilson, gauge and
// clover set, no context twice).
int batch_check(lqcd_ctx* const* ctxs, const int* nrhs, int nlattices, bool* clover) {
  if (!ctxs || !nrhs || nlattices < 1 || nlattices > MAXLAT)
    return set_error(LQCD_EINVAL, "bad batch arguments (1 to 16 lattices)");
  hipStream_t stream = ctxs[0] ? ctxs[0]->stream : nullptr;
  for (int l = 0; l < nlattices; ++l) {
    lqcd_ctx* c = ctxs[l];
    if (!c || nrhs[l] < 1) return set_error(LQCD_EINVAL, "null context or nrhs < 1");
    if (!c->have_gauge || !c->have_clover) return set_error(LQCD_ESTATE, "set_gauge and set_clover must come first");
    if (c->stream != stream) return set_error(LQCD_EINVAL, "all contexts of a batch must share one stream");
    if (l == 0) *clover = !c->is_wilson;
    else if (*clover != !c->is_wilson) return set_error(LQCD_EINVAL, "a batch is all clover or all Wilson");
    for (int m = 0; m < l; ++m)
      if (ctxs[m] == c) return set_error(LQCD_EINVAL, "a context appears twice in the batch");
  }
  return LQCD_OK;
}

// The batch of these contexts at inner precision IP: descriptors rebuilt from
// the current contexts, buffers allocated when the batch shape is new (kept
// on the first context for the next call with the same shape).
int batch_prepare(lqcd_ctx* const* ctxs, const int* nrhs, int nlattices, int IP, bool clover, Batch** out) {
  hipStream_t stream = ctxs[0]->stream;
  std::vector<std::pair<int, int>> key;
  for (int l = 0; l < nlattices; ++l) {
    const Geom& g = ctxs[l]->g;
    key.push_back({g.lx | (g.ly << 16), g.lz | (g.lt << 16)});
    key.push_back({g.vh, nrhs[l]});
  }
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
  int total_seg = 0;
  for (int l = 0; l < nlattices; ++l) total_seg += nrhs[l];
  if (!reuse) {
    B.key = key;
    LQ_TRY(B.dev_alloc(reinterpret_cast<void**>(&B.dscal_all), (size_t)total_seg * sizeof(Scal)));
  }
  B.hlat.clear();
  B.ctx.clear();
  B.max_rhs = 1;
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
    L.nsb = (int)(padded_sites(c->g.vh) / SB);
    L.nbb = (c->g.vh + BS - 1) / BS;
    L.nrhs = nrhs[l];
    L.tile0 = tile;
    L.btile0 = btile;
    L.seg0 = seg;
    tile += L.nsb;
    btile += L.nbb * L.nrhs;
    B.max_rhs = std::max(B.max_rhs, L.nrhs);
    B.hlat.push_back(L);
    B.ctx.push_back(c);
    for (int r = 0; r < nrhs[l]; ++r, ++seg) {
      if (reuse) continue;
      BSeg S{};
      const size_t vh = c->g.vh;
      for (int f = 0; f < F_COUNT; ++f)
        LQ_TRY(B.dev_alloc(&S.f[f], spinor_bytes(f == F_X ? B.xprec : IP, vh)));
      S.sc = B.dscal_all + seg;
      // partial sums: 3 per 64-site hop block (more than per BS-site vector block)
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
  if (!reuse) {
    size_t cap = 0;
    for (const BLat& L : B.hlat) cap += (size_t)L.nsb * L.nrhs;
    B.tile_cap = cap;
    for (int k = 0; k < BK_N; ++k) LQ_TRY(B.dev_alloc(reinterpret_cast<void**>(&B.dtiles[k]), cap * sizeof(int2)));
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
  *out = &B;
  return LQCD_OK;
}


std::string batch_key(const Batch& B) {
  std::ostringstream o;
  o << "batch:" << B.prec << ":" << (B.clover ? 1 : 0) << ":";
  for (size_t l = 0; l < B.hlat.size(); ++l) {
    const Geom& g = B.hlat[l].g;
    o << (l ? "," : "") << g.lx << "." << g.ly << "." << g.lz << "." << g.lt << "x" << B.hlat[l].nrhs;
  }
  return o.str();
}

bool shape_ok(const Batch& B, const BShape& sh) {
  const int max_nb = B.prec == 0 ? 2 : 4;
  return sh.nb >= 1 && sh.nb <= max_nb && sh.nw >= 1 && sh.nw <= BHOP_MAX_WAVES && sh.nslot >= 1 &&
         sh.nslot <= 4096 && sh.walk >= 0 && sh.walk <= 3 && (sh.nt == 0 || sh.nt == 1);
}

// Average duration (us) of one kind of batched hop with shape sh, HIP events
// on the batch's stream, reps launches after two warm-up launches: the
// A_oo^-1 H_oe hop (F_P -> F_Y) or one of the two XPAY hops of the solver's
// iteration (F_Y -> F_V with <rhat, v>, F_Y -> F_T with <t, s>, <t, t>).
int time_bhop(Batch& B, int kind, const BShape& sh, int reps, double* us) {
  LQ_TRY(set_shape(B, kind, sh));
  auto launch = [&]() {
    if (kind == BK_SC) return batch_hop(B, B.stream, F_P, F_Y, -1, -1, 1, EPI_SCALE_CLOV, RED_NONE, 3, 0);
    if (kind == BK_DOT) return batch_hop(B, B.stream, F_Y, F_V, F_P, F_RHAT, 0, EPI_XPAY, RED_DOT, 0, 1);
    return batch_hop(B, B.stream, F_Y, F_T, F_S, -1, 0, EPI_XPAY, RED_TS, 0, 1);
  };
  hipEvent_t e0, e1;
  LQ_HIP(hipEventCreate(&e0));
  LQ_HIP(hipEventCreate(&e1));
  int st = LQCD_OK;
  for (int k = 0; k < 2 && st == LQCD_OK; ++k) st = launch();
  (void)hipEventRecord(e0, B.stream);
  for (int k = 0; k < reps && st == LQCD_OK; ++k) st = launch();
  (void)hipEventRecord(e1, B.stream);
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  LQ_TRY(st);
  *us = 1000.0 * ms / reps;
  return LQCD_OK;
}

// Pick the launch shape of each kind of batched hop for this batch
// (right-hand sides per lane x wavefronts per workgroup x workgroups per XCD x
// walk) by timing the candidates on the batch's own fields; a forced shape
// (nb > 0) is used for every kind and only the A_oo^-1 H_oe hop is timed.
// The choices are read from and written to the tune cache (LQCD_TUNE_CACHE),
// one entry per kind.
int batch_tune(Batch& B, bool sweep, const BShape* forced = nullptr) {
  const std::string base = batch_key(B);
  const std::string keys[BK_N] = {base, base + ":xpay_dot", base + ":xpay_ts"};
  auto unpack = [](const int v[4]) {
    BShape sh;
    sh.nw = v[0] / 64;
    sh.nb = v[1];
    sh.nslot = v[2];
    sh.walk = v[3] & 3;
    sh.nt = (v[3] >> 2) & 1;
    return sh;
  };
  if (!sweep && !forced) {
    BShape got[BK_N];
    bool all = true;
    for (int k = 0; k < BK_N && all; ++k) {
      int v[4];
      all = tune_cache_get(keys[k], v) && shape_ok(B, got[k] = unpack(v));
    }
    if (all) {
      for (int k = 0; k < BK_N; ++k) LQ_TRY(set_shape(B, k, got[k]));
      B.tuned = true;
      return LQCD_OK;
    }
  }
  // the timed launches read zeroed fields of every segment, none masked
  for (size_t s = 0; s < B.hseg.size(); ++s) {
    lqcd_ctx* c = B.ctx[B.seg_lat[s]];
    for (int f : {F_P, F_Y, F_S, F_RHAT}) LQ_TRY(blas_zero(c, B.prec, B.hseg[s].f[f]));
  }
  LQ_HIP(hipMemsetAsync(B.dscal_all, 0, B.hseg.size() * sizeof(Scal), B.stream));
  if (forced) {
    if (!shape_ok(B, *forced)) return set_error(LQCD_EINVAL, "bad batched hop launch shape");
    for (int k = BK_N - 1; k >= 0; --k) LQ_TRY(set_shape(B, k, *forced));
    LQ_TRY(time_bhop(B, BK_SC, *forced, 5, &B.hop_us));
    B.tuned = true;
    return LQCD_OK;
  }
  const bool verbose = std::getenv("LQCD_TUNE_VERBOSE") != nullptr;
  for (int kind = 0; kind < BK_N; ++kind) {
    // candidates: 1-4 right-hand sides per lane (1-2 in FP64) x 1, 2, 3, 4, 6
    // or all groups per workgroup (at most 8 waves) x 128, 256, 512
    // workgroups per XCD x the walks (the XPAY forms: linear and slab, the
    // split slabs never won for them); streaming loads measured slower
    std::vector<BShape> cand;
    for (int nb = 1; nb <= (B.prec == 0 ? 2 : 4); ++nb) {
      const int ngroup = (B.max_rhs + nb - 1) / nb;
      for (int nw : {1, 2, 3, 4, 6, ngroup}) {
        if (nw > ngroup || nw > BHOP_MAX_WAVES) continue;
        for (int nslot : {128, 256, 512})
          for (int walk = 0; walk < (kind == BK_SC ? 4 : 2); ++walk) {
            BShape sh;
            sh.nb = nb;
            sh.nw = nw;
            sh.nslot = nslot;
            sh.walk = walk;
            sh.nt = 0;
            bool dup = false;
            for (const BShape& c : cand)
              dup = dup || (c.nb == sh.nb && c.nw == sh.nw && c.nslot == sh.nslot && c.walk == sh.walk);
            if (!dup) cand.push_back(sh);
          }
      }
    }
    BShape best = cand[0];
    double best_us = 1e30;
    for (const BShape& sh : cand) {
      double us = 0;
      LQ_TRY(time_bhop(B, kind, sh, 5, &us));
      if (verbose)
        std::fprintf(stderr, "[lqcd tune] %s nb %d nw %d nslot %d walk %d nt %d: %.1f us\n", keys[kind].c_str(),
                     sh.nb, sh.nw, sh.nslot, sh.walk, sh.nt, us);
      if (us < best_us) {
        best_us = us;
        best = sh;
      }
    }
    LQ_TRY(set_shape(B, kind, best));
    if (kind == BK_SC) B.hop_us = best_us;
    const int v[4] = {64 * best.nw, best.nb, best.nslot, best.walk | (best.nt << 2)};
    LQ_TRY(tune_cache_put(keys[kind], v, best_us));
  }
  B.tuned = true;
  return LQCD_OK;
}

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
  for (int l = 0; l < nlattices; ++l)
    if (!b[l] || !x[l]) return set_error(LQCD_EINVAL, "null vector");
  bool clover = false;
  LQ_TRY(batch_check(ctxs, nrhs, nlattices, &clover));
  hipStream_t stream = ctxs[0]->stream;
  const int IP = prm.inner_prec;
  Batch* Bp = nullptr;
  LQ_TRY(batch_prepare(ctxs, nrhs, nlattices, IP, clover, &Bp));
  Batch& B = *Bp;
  if (!B.tuned) LQ_TRY(batch_tune(B, false));
  Scal* dscal_all = B.dscal_all;
  const int nseg = (int)B.hseg.size();
  const int check = prm.check_every > 0 ? prm.check_every : 8;
  // default inner tolerances: FP32 1e-6; FP16 5e-3 (measured on 36 point
  // sources on three clover lattices: 355 iterations against 397 at 1e-2)
  const double delta = prm.inner_tol > 0 ? prm.inner_tol : (IP == 1 ? 1e-6 : (IP == 2 ? 5e-3 : 1e-10));

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

extern "C" int lqcd_batch_autotune(lqcd_ctx* const* ctxs, const int* nrhs, int nlattices, int prec, int shape[5],
                                   double* us) {
  if (prec < 0 || prec > 2) return set_error(LQCD_EINVAL, "bad precision");
  bool clover = false;
  LQ_TRY(batch_check(ctxs, nrhs, nlattices, &clover));
  Batch* Bp = nullptr;
  LQ_TRY(batch_prepare(ctxs, nrhs, nlattices, prec, clover, &Bp));
  Batch& B = *Bp;
  if (shape && shape[0] > 0) {
    BShape sh;
    sh.nb = shape[0];
    sh.nw = shape[1];
    sh.nslot = shape[2];
    sh.walk = shape[3];
    sh.nt = shape[4];
    LQ_TRY(batch_tune(B, false, &sh));
  } else {
    B.tuned = false;
    LQ_TRY(batch_tune(B, false));
  }
  // time the chosen shape of the A_oo^-1 H_oe hop on its own (also after a cache hit)
  const BShape sh = B.shape[BK_SC];
  double t = 0;
  LQ_TRY(time_bhop(B, BK_SC, sh, 20, &t));
  B.hop_us = t;
  if (us) *us = t;
  if (shape) {
    shape[0] = sh.nb;
    shape[1] = sh.nw;
    shape[2] = sh.nslot;
    shape[3] = sh.walk;
    shape[4] = sh.nt;
  }
  LQ_HIP(hipStreamSynchronize(B.stream));
  return LQCD_OK;
}

extern "C" int lqcd_batch_apply_schur(lqcd_ctx* const* ctxs, const int* nrhs, int nlattices, int prec,
                                      const double* const* in, double* const* out) {
  if (prec < 0 || prec > 2) return set_error(LQCD_EINVAL, "bad precision");
  if (!in || !out) return set_error(LQCD_EINVAL, "null vector list");
  bool clover = false;
  LQ_TRY(batch_check(ctxs, nrhs, nlattices, &clover));
  for (int l = 0; l < nlattices; ++l)
    if (!in[l] || !out[l]) return set_error(LQCD_EINVAL, "null vector");
  Batch* Bp = nullptr;
  LQ_TRY(batch_prepare(ctxs, nrhs, nlattices, prec, clover, &Bp));
  Batch& B = *Bp;
  if (!B.tuned) LQ_TRY(batch_tune(B, false));
  // every segment active: S in -> out through the two batched hops of the solver
  LQ_HIP(hipMemsetAsync(B.dscal_all, 0, B.hseg.size() * sizeof(Scal), B.stream));
  for (size_t s = 0; s < B.hseg.size(); ++s) {
    const int l = B.seg_lat[s];
    lqcd_ctx* c = B.ctx[l];
    const size_t n = (size_t)c->g.vh * 2 * 24;
    const double* src = in[l] + (size_t)(s - B.hlat[l].seg0) * n;
    LQ_TRY(launch_import_spinor(c, prec, 0, src, B.hseg[s].f[F_P]));
  }
  LQ_TRY(batch_hop(B, B.stream, F_P, F_Y, -1, -1, 1, EPI_SCALE_CLOV, RED_NONE, 3, 0));
  LQ_TRY(batch_hop(B, B.stream, F_Y, F_T, F_P, -1, 0, EPI_XPAY, RED_TS, 0, 1));
  for (size_t s = 0; s < B.hseg.size(); ++s) {
    const int l = B.seg_lat[s];
    lqcd_ctx* c = B.ctx[l];
    const size_t n = (size_t)c->g.vh * 2 * 24;
    double* dst = out[l] + (size_t)(s - B.hlat[l].seg0) * n;
    LQ_HIP(hipMemsetAsync(dst, 0, n * sizeof(double), B.stream));
    LQ_TRY(launch_export_spinor(c, prec, 0, B.hseg[s].f[F_T], dst));
  }
  LQ_HIP(hipStreamSynchronize(B.stream));
  return LQCD_OK;
}
