// Even-odd preconditioned BiCGStab and the mixed-precision outer loop.
//
// The paper benchmarks BiCGStab for the clover operator and a
// mixed-precision BiCGStab (Sec. 3) and uses the even-odd preconditioned
// operator of Eq. (1) in its solvers. Here:
//   * source preparation  b' = b_e - D_eo D_oo^-1 b_o = b_e + kappa H_eo A_oo^-1 b_o,
//   * BiCGStab (van der Vorst 1992) on S x_e = b' with every scalar kept on the
//     device, <rhat, v> and <t, s>, <t, t> fused into the operator's last hop and
//     <rhat, r>, <r, r> into the x/r update; CHECK iterations are enqueued (or
//     replayed from one captured hipGraph) between host reads of the
//     convergence flag,
//   * precision: FP64 BiCGStab, or FP32 / FP16-storage inner BiCGStab inside an
//     FP64 defect-correction loop (r = b' - S x in FP64, inner solve of
//     S e = r/|r| to a loose tolerance, x += |r| e), FP64 only for the true
//     residual, the outer update and the reductions,
//   * reconstruction   x_o = D_oo^-1 (b_o - D_oe x_e) = A_oo^-1 (b_o + kappa H_oe x_e),
//     then the true residual |b - D x| / |b| with the full FP64 operator.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "blas.h"
#include "internal.h"
#include "ops.h"
#include "solver.h"

namespace lq {

static int alloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return set_error(LQCD_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return LQCD_OK;
}

int InnerVecs::init(lqcd_ctx* c, int p, int xp) {
  prec = p;
  xprec = xp;
  const size_t vh = c->g.vh;
  void** v[] = {&r, &rhat, &pv, &v_, &s, &t, &y};
  for (void** q : v) LQ_TRY(alloc(q, spinor_bytes(prec, vh)));
  LQ_TRY(alloc(&x, spinor_bytes(xprec, vh)));
  LQ_TRY(alloc(reinterpret_cast<void**>(&sc), sizeof(Scal)));
  const size_t np = std::max((size_t)blas_blocks(vh), max_hop_blocks(vh)) * 3;
  LQ_TRY(alloc(reinterpret_cast<void**>(&partials), np * sizeof(double)));
  return LQCD_OK;
}

void InnerVecs::release() {
  void* v[] = {r, rhat, pv, v_, s, t, y, x, sc, partials};
  for (void* q : v)
    if (q) (void)hipFree(q);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  *this = InnerVecs();
}

int Workspace::init(lqcd_ctx* c) {
  const size_t vh = c->g.vh;
  void** v[] = {&b_e, &b_o, &bhat, &x_e, &x_o, &r64, &v64, &y64};
  for (void** q : v) LQ_TRY(alloc(q, spinor_bytes(0, vh)));
  LQ_TRY(alloc(reinterpret_cast<void**>(&norms), 64 * sizeof(double)));
  LQ_TRY(hipHostMalloc(reinterpret_cast<void**>(&hnorms), 64 * sizeof(double) + sizeof(Scal)) == hipSuccess
             ? LQCD_OK
             : set_error(LQCD_ENOMEM, "hipHostMalloc failed"));
  return LQCD_OK;
}

void Workspace::release() {
  void* v[] = {b_e, b_o, bhat, x_e, x_o, r64, v64, y64, norms};
  for (void* q : v)
    if (q) (void)hipFree(q);
  if (hnorms) (void)hipHostFree(hnorms);
  for (auto& iv : inner) iv.release();
}

int ensure_workspace(lqcd_ctx* c, int inner_prec) {
  if (!c->ws) {
    c->ws = new Workspace();
    int s = c->ws->init(c);
    if (s != LQCD_OK) {
      c->ws->release();
      delete c->ws;
      c->ws = nullptr;
      return s;
    }
  }
  InnerVecs& iv = c->ws->inner[inner_prec];
  if (!iv.r) {
    const int xp = inner_prec == 2 ? 1 : inner_prec;
    int s = iv.init(c, inner_prec, xp);
    if (s != LQCD_OK) {
      iv.release();
      return s;
    }
  }
  return LQCD_OK;
}

// |a|^2 of an FP64 half field into norms[slot..slot+2] (sum, 1/sqrt, sqrt)
static int norm64(lqcd_ctx* c, const void* a, double* dst) {
  Workspace* w = c->ws;
  InnerVecs& iv = w->inner[0].r ? w->inner[0] : w->inner[1].r ? w->inner[1] : w->inner[2];
  LQ_TRY(blas_dot_norm(c, 0, a, a, iv.partials));
  return fin_norm(c, dst, iv.partials, blas_blocks(c->g.vh), 3, 2);
}

static double* scratch_partials(lqcd_ctx* c) {
  Workspace* w = c->ws;
  return w->inner[0].r ? w->inner[0].partials : w->inner[1].r ? w->inner[1].partials : w->inner[2].partials;
}

// r = b' - S x (FP64), |r|^2 -> dst
static int residual64(lqcd_ctx* c, const void* x, void* r, double* dst) {
  Workspace* w = c->ws;
  double* part = scratch_partials(c);
  LQ_TRY(op_schur(c, 0, x, w->v64, w->y64, RED_NONE, nullptr, nullptr, nullptr, nullptr));
  LQ_TRY(blas_sub_norm(c, w->bhat, w->v64, r, part));
  return fin_norm(c, dst, part, blas_blocks(c->g.vh), 1, 0);
}

// The BiCGStab iteration body: everything after p is known.
static int bicg_iteration(lqcd_ctx* c, InnerVecs& v) {
  const int P = v.prec;
  const int* skip = &v.sc->done;
  int nb = 0;
  LQ_TRY(op_schur(c, P, v.pv, v.v_, v.y, RED_DOT, v.rhat, v.partials, skip, &nb));
  LQ_TRY(fin_alpha(c, v.sc, v.partials, nb));
  LQ_TRY(blas_s_update(c, P, v.r, v.v_, v.s, v.sc));
  LQ_TRY(op_schur(c, P, v.s, v.t, v.y, RED_TS, nullptr, v.partials, skip, &nb));
  LQ_TRY(fin_omega(c, v.sc, v.partials, nb));
  LQ_TRY(blas_xr_update(c, P, v.xprec, v.x, v.pv, v.s, v.t, v.r, v.rhat, v.sc, v.partials));
  LQ_TRY(fin_rho(c, v.sc, v.partials, blas_blocks(c->g.vh)));
  return blas_p_update(c, P, v.r, v.pv, v.v_, v.sc);
}

static int run_chunk(lqcd_ctx* c, InnerVecs& v, int k, bool use_graph) {
  if (!use_graph) {
    for (int j = 0; j < k; ++j) LQ_TRY(bicg_iteration(c, v));
    return LQCD_OK;
  }
  if (!v.exec || v.graph_k != k || v.graph_block != c->hop_block[v.prec] || v.graph_remap != c->hop_remap[v.prec] ||
      v.graph_nt != c->hop_nt[v.prec] || v.graph_split != c->hop_split[v.prec]) {
    if (v.exec) (void)hipGraphExecDestroy(v.exec);
    if (v.graph) (void)hipGraphDestroy(v.graph);
    v.exec = nullptr;
    v.graph = nullptr;
    if (!c->cap_stream) LQ_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t saved = c->stream;
    c->stream = c->cap_stream;
    LQ_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int st = LQCD_OK;
    for (int j = 0; j < k && st == LQCD_OK; ++j) st = bicg_iteration(c, v);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = saved;
    if (st != LQCD_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return set_error(LQCD_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    v.graph = g;
    LQ_HIP(hipGraphInstantiate(&v.exec, v.graph, nullptr, nullptr, 0));
    v.graph_k = k;
    v.graph_block = c->hop_block[v.prec];
    v.graph_remap = c->hop_remap[v.prec];
    v.graph_nt = c->hop_nt[v.prec];
    v.graph_split = c->hop_split[v.prec];
  }
  LQ_HIP(hipGraphLaunch(v.exec, c->stream));
  return LQCD_OK;
}

// BiCGStab on S x = rhs in precision v.prec; rhs in v.r on entry; x in v.x
// (caller initialises). Runs until the iterated |r|^2 <= target2 or the
// iteration budget is spent. Returns the iterations done in *iters.
static int bicg_run(lqcd_ctx* c, InnerVecs& v, double target2, int max_iters, int check, bool use_graph,
                    int* iters, int* breakdown, double* rr) {
  const int P = v.prec;
  LQ_TRY(blas_copy(c, P, v.r, v.rhat));
  LQ_TRY(blas_copy(c, P, v.r, v.pv));
  LQ_TRY(blas_dot_norm(c, P, v.rhat, v.r, v.partials));
  LQ_TRY(fin_init(c, v.sc, v.partials, blas_blocks(c->g.vh), target2, max_iters));
  Scal* hs = reinterpret_cast<Scal*>(c->ws->hnorms + 32);
  const bool verbose = log_level() >= 2;
  int last_logged = 0;
  for (;;) {
    LQ_HIP(hipMemcpyAsync(hs, v.sc, sizeof(Scal), hipMemcpyDeviceToHost, c->stream));
    LQ_HIP(hipStreamSynchronize(c->stream));
    if (verbose && (hs->done || hs->iters / 256 != last_logged / 256)) {
      std::fprintf(stderr, "[lqcd] inner prec %d iter %d |r|^2 %.3e (target %.3e)\n", P, hs->iters, hs->rr,
                   target2);
      last_logged = hs->iters;
    }
    if (hs->done) break;
    LQ_TRY(run_chunk(c, v, check, use_graph));
  }
  *iters = hs->iters;
  *breakdown = hs->breakdown;
  *rr = hs->rr;
  return LQCD_OK;
}

// Mixed precision with reliable updates (Sleijpen and van der Vorst, 1996):
// one low-precision BiCGStab runs on the residual equation normalised by the
// last true residual; whenever its iterated residual has dropped by DELTA_R
// since then (or it reports convergence), the low-precision solution is added
// to x in FP64, the true residual b' - S x is recomputed in FP64 and put back
// into the iteration (p and v rescaled to the new normalisation, rho
// recomputed), so that the Krylov space is kept instead of restarted. On a
// breakdown the iteration restarts from the true residual.
static int reliable_mixed(lqcd_ctx* c, const lqcd_solve_params& prm, InnerVecs& iv, double target, double bnorm2,
                          double& rnorm, int& total_iters, int& restarts, int& updates, int& status) {
  const double DELTA_R = prm.inner_tol > 0 && prm.inner_tol < 1 ? prm.inner_tol : 0.1;
  Workspace* w = c->ws;
  const int IP = iv.prec;
  double* hn = w->hnorms;
  Scal* hs = reinterpret_cast<Scal*>(hn + 32);
  const int check = prm.check_every > 0 ? prm.check_every : 8;
  const bool graph = prm.use_graph != 0;
  const int nb = blas_blocks(c->g.vh);
  bool restart = true;
  int base_iters = 0;  // iterations of earlier restarts
  double prev = rnorm;
  int fails = 0;
  while (rnorm > target) {
    if (restart) {
      if (total_iters >= prm.max_iter) break;
      LQ_TRY(blas_scale_down(c, IP, w->r64, iv.r, w->norms + 7, 0.0));
      LQ_TRY(blas_zero(c, iv.xprec, iv.x));
      LQ_TRY(blas_copy(c, IP, iv.r, iv.rhat));
      LQ_TRY(blas_copy(c, IP, iv.r, iv.pv));
      LQ_TRY(blas_dot_norm(c, IP, iv.rhat, iv.r, iv.partials));
      const double t = target / rnorm;
      LQ_TRY(fin_init(c, iv.sc, iv.partials, nb, t * t, prm.max_iter - total_iters));
      base_iters = total_iters;
      restart = false;
    }
    // iterate until the iterated residual has dropped by DELTA_R (it starts at 1)
    for (;;) {
      LQ_HIP(hipMemcpyAsync(hs, iv.sc, sizeof(Scal), hipMemcpyDeviceToHost, c->stream));
      LQ_HIP(hipStreamSynchronize(c->stream));
      if (hs->done || hs->rr <= DELTA_R * DELTA_R) break;
      LQ_TRY(run_chunk(c, iv, check, graph));
    }
    total_iters = base_iters + hs->iters;
    const bool breakdown = hs->breakdown != 0;
    const bool exhausted = hs->iters >= hs->max_iters;
    // reliable update: x += |r| e (FP64), e = 0, r = b' - S x (FP64)
    LQ_TRY(blas_accum_up(c, iv.xprec, w->x_e, iv.x, w->norms + 8));
    LQ_TRY(blas_zero(c, iv.xprec, iv.x));
    LQ_TRY(residual64(c, w->x_e, w->r64, w->norms + 6));
    LQ_HIP(hipMemcpyAsync(hn + 6, w->norms + 6, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LQ_HIP(hipStreamSynchronize(c->stream));
    const double rold = rnorm;
    rnorm = hn[8];
    ++updates;
    if (log_level() >= 1)
      std::fprintf(stderr, "[lqcd] reliable update %d (inner prec %d): %d iterations, |r|/|b| %.3e\n", updates, IP,
                   total_iters, rnorm / std::sqrt(bnorm2));
    if (rnorm <= target) break;
    if (exhausted || total_iters >= prm.max_iter) break;
    if (!(rnorm < prev)) {
      if (++fails > 5) {
        status = set_error(LQCD_EBREAKDOWN, "reliable updates stopped reducing the residual");
        return LQCD_OK;
      }
    } else {
      prev = rnorm;
    }
    if (breakdown || !(rnorm < rold)) {
      ++restarts;
      restart = true;
      continue;
    }
    // put the true residual back: r = r64 / |r64|, p and v to the new normalisation
    LQ_TRY(blas_scale_down(c, IP, w->r64, iv.r, w->norms + 7, 0.0));
    LQ_TRY(blas_scale2(c, IP, iv.pv, iv.v_, rold / rnorm));
    LQ_TRY(blas_dot_norm(c, IP, iv.rhat, iv.r, iv.partials));
    const double t = target / rnorm;
    LQ_TRY(fin_reliable(c, iv.sc, iv.partials, nb, t * t));
  }
  if (rnorm > target && status == LQCD_OK)
    status = set_error(LQCD_ENOCONV, "mixed-precision solve did not reach the tolerance");
  return LQCD_OK;
}

int solve_native(lqcd_ctx* c, const lqcd_solve_params& prm, lqcd_solve_stats& st) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  Workspace* w = c->ws;
  const int IP = prm.inner_prec;
  InnerVecs& iv = w->inner[IP];
  const double k = c->kappa;
  double* hn = w->hnorms;
  const int check = prm.check_every > 0 ? prm.check_every : 8;
  const bool graph = prm.use_graph != 0;

  // |b|^2 over both parities
  LQ_TRY(norm64(c, w->b_e, w->norms + 0));
  LQ_TRY(norm64(c, w->b_o, w->norms + 3));
  // source preparation: b' = b_e + kappa H_eo A_oo^-1 b_o
  const void* ainv_o = clover_slot(c, 0, 3);
  const void* src_o = w->b_o;
  if (ainv_o) {
    LQ_TRY(launch_site(c, 0, ainv_o, w->b_o, w->y64));
    src_o = w->y64;
  }
  LQ_TRY(op_hop_xpay(c, 0, 0, src_o, w->b_e, nullptr, w->bhat, k));
  LQ_HIP(hipMemcpyAsync(hn, w->norms, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  const double bnorm2 = hn[0] + hn[3];
  const auto t_prep = clk::now();
  double setup_s = std::chrono::duration<double>(t_prep - t0).count();
  st = lqcd_solve_stats{};
  if (bnorm2 == 0.0) {
    LQ_TRY(blas_zero(c, 0, w->x_e));
    LQ_TRY(blas_zero(c, 0, w->x_o));
    LQ_HIP(hipStreamSynchronize(c->stream));
    st.true_rel_resid = 0.0;
    st.seconds_setup = setup_s;
    st.seconds_solve = std::chrono::duration<double>(clk::now() - t0).count();
    return LQCD_OK;
  }
  const double target = prm.tol * std::sqrt(bnorm2);
  int status = LQCD_OK;

  // initial residual r = b' - S x_e (x_e holds the initial guess, zero by default)
  LQ_TRY(residual64(c, w->x_e, w->r64, w->norms + 6));
  LQ_HIP(hipMemcpyAsync(hn + 6, w->norms + 6, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  double rnorm = hn[8];
  int total_iters = 0, restarts = 0, outer = 0, fails = 0;

  if (IP == 0) {
    // plain FP64 BiCGStab on S, accumulating into x_e directly; restart from the
    // true residual when the iterated one has converged but the true one has not
    while (rnorm > target) {
      if (total_iters >= prm.max_iter || outer >= prm.max_outer) {
        status = set_error(LQCD_ENOCONV, "FP64 BiCGStab did not reach the tolerance");
        break;
      }
      LQ_TRY(blas_copy(c, 0, w->r64, iv.r));
      LQ_TRY(blas_copy(c, 0, w->x_e, iv.x));
      int it = 0, bd = 0;
      double rr = 0;
      LQ_TRY(bicg_run(c, iv, target * target, prm.max_iter - total_iters, check, graph, &it, &bd, &rr));
      total_iters += it;
      ++outer;
      LQ_TRY(blas_copy(c, 0, iv.x, w->x_e));
      LQ_TRY(residual64(c, w->x_e, w->r64, w->norms + 6));
      LQ_HIP(hipMemcpyAsync(hn + 6, w->norms + 6, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      LQ_HIP(hipStreamSynchronize(c->stream));
      const double prev = rnorm;
      rnorm = hn[8];
      if (log_level() >= 1)
        std::fprintf(stderr, "[lqcd] FP64 pass %d: %d iterations, |r|/|b| %.3e\n", outer, total_iters,
                     rnorm / std::sqrt(bnorm2));
      if (rnorm > target) ++restarts;
      if (bd) ++fails;
      if (!(rnorm < prev) && ++fails > 5) {
        status = set_error(LQCD_EBREAKDOWN, "BiCGStab stagnated or broke down repeatedly");
        break;
      }
    }
  } else {
    if (prm.reliable_update) {
      LQ_TRY(reliable_mixed(c, prm, iv, target, bnorm2, rnorm, total_iters, restarts, outer, status));
    } else {
    // mixed precision: FP64 defect correction around FP32 / FP16 BiCGStab
    const double delta = prm.inner_tol > 0 ? prm.inner_tol : (IP == 1 ? 1e-6 : 1e-2);
    while (rnorm > target) {
      if (total_iters >= prm.max_iter || outer >= prm.max_outer) {
        status = set_error(LQCD_ENOCONV, "mixed-precision solve did not reach the tolerance");
        break;
      }
      // inner rhs = r / |r| in the inner precision; inner x = 0
      LQ_TRY(blas_scale_down(c, IP, w->r64, iv.r, w->norms + 7, 0.0));
      LQ_TRY(blas_zero(c, iv.xprec, iv.x));
      // do not ask the inner solve for more than the outer loop still needs
      double d = delta;
      const double need = target / rnorm;
      if (need > d) d = need * 0.5;
      int it = 0, bd = 0;
      double rr = 0;
      LQ_TRY(bicg_run(c, iv, d * d, prm.max_iter - total_iters, check, graph, &it, &bd, &rr));
      total_iters += it;
      ++outer;
      // x += |r| e
      LQ_TRY(blas_accum_up(c, iv.xprec, w->x_e, iv.x, w->norms + 8));
      LQ_TRY(residual64(c, w->x_e, w->r64, w->norms + 6));
      LQ_HIP(hipMemcpyAsync(hn + 6, w->norms + 6, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      LQ_HIP(hipStreamSynchronize(c->stream));
      const double prev = rnorm;
      rnorm = hn[8];
      if (log_level() >= 1)
        std::fprintf(stderr, "[lqcd] outer %d (inner prec %d): %d inner iterations, |r|/|b| %.3e\n", outer, IP,
                     total_iters, rnorm / std::sqrt(bnorm2));
      if (bd) ++restarts;
      if (!(rnorm < prev) && ++fails > 5) {
        status = set_error(LQCD_EBREAKDOWN, "defect correction stopped reducing the residual");
        break;
      }
    }
    }
  }
  const auto t_solved = clk::now();

  // reconstruction x_o = A_oo^-1 (b_o + kappa H_oe x_e)
  if (ainv_o) {
    LQ_TRY(op_hop_xpay(c, 0, 1, w->x_e, w->b_o, nullptr, w->y64, k));
    LQ_TRY(launch_site(c, 0, ainv_o, w->y64, w->x_o));
  } else {
    LQ_TRY(op_hop_xpay(c, 0, 1, w->x_e, w->b_o, nullptr, w->x_o, k));
  }
  // true residual with the full FP64 operator
  LQ_TRY(op_full(c, 0, w->x_e, w->x_o, w->v64, w->y64));
  double* part = scratch_partials(c);
  LQ_TRY(blas_sub_norm(c, w->b_e, w->v64, w->v64, part));
  LQ_TRY(fin_norm(c, w->norms + 9, part, blas_blocks(c->g.vh), 1, 0));
  LQ_TRY(blas_sub_norm(c, w->b_o, w->y64, w->y64, part));
  LQ_TRY(fin_norm(c, w->norms + 12, part, blas_blocks(c->g.vh), 1, 0));
  LQ_HIP(hipMemcpyAsync(hn + 9, w->norms + 9, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  const auto t1 = clk::now();
  setup_s += std::chrono::duration<double>(t1 - t_solved).count();
  st.outer_iters = outer;
  st.inner_iters = total_iters;
  st.restarts = restarts;
  st.true_rel_resid = std::sqrt((hn[9] + hn[12]) / bnorm2);
  st.seconds_setup = setup_s;
  st.seconds_solve = std::chrono::duration<double>(t1 - t0).count();
  return status;
}

}  // namespace lq
