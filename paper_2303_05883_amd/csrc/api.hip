// The C ABI (include/lqcd.h): context life cycle, field set-up, operator
// application through the canonical layout, and the solve entry points.
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "blas.h"
#include "internal.h"
#include "ops.h"
#include "sap.h"
#include "stag.h"
#include "dwf.h"
#include "mg.h"
#include "solver.h"
#include "tune.h"

namespace lq {

// Scratch of lqcd_apply_native_noalloc: the odd half field between the two
// hops of the Schur operator, in a file-scope device array instead of a
// library allocation. Each GPU the library runs on holds its own copy (from
// the first use of this code object on that GPU to the end of the process);
// host code reaches it only through the per-device address that
// hipGetSymbolAddress returns (the array's name is a host-side stand-in).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static void* g_scratch_addr[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_scratch_mutex;

// The scratch array's address on the current device (looked up once per device).
static int noalloc_scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return set_error(LQCD_EHIP, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return set_error(LQCD_EHIP, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
    }
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return LQCD_OK;
}

static thread_local std::string g_last_error;

int set_error(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

static int dalloc(void** p, size_t bytes) {
  if (*p) return LQCD_OK;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return set_error(LQCD_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return LQCD_OK;
}

static void dfree(void*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

static size_t full_sites(const lqcd_ctx* c) { return (size_t)c->g.vh * 2; }

int ensure_canon(lqcd_ctx* c) {
  LQ_TRY(dalloc(&c->canon_a, full_sites(c) * 192));
  return dalloc(&c->canon_b, full_sites(c) * 192);
}

static int ensure_apply_buffers(lqcd_ctx* c, int prec) {
  LQ_TRY(ensure_canon(c));
  const size_t b = spinor_bytes(prec, c->g.vh);
  LQ_TRY(dalloc(&c->half_a[prec], b));
  LQ_TRY(dalloc(&c->half_b[prec], b));
  LQ_TRY(dalloc(&c->half_c[prec], b));
  LQ_TRY(dalloc(&c->half_d[prec], b));
  return LQCD_OK;
}

static void invalidate_graphs(lqcd_ctx* c) {
  if (!c->ws) return;
  for (auto& iv : c->ws->inner) {
    if (iv.exec) (void)hipGraphExecDestroy(iv.exec);
    if (iv.graph) (void)hipGraphDestroy(iv.graph);
    iv.exec = nullptr;
    iv.graph = nullptr;
    iv.graph_k = 0;
  }
}

// Copy a canonical vector (n doubles) to device staging if it lives on the host.
static int stage_in(lqcd_ctx* c, const double* src, int on_device, void* staging, size_t bytes, const double** dev) {
  if (on_device) {
    *dev = src;
    return LQCD_OK;
  }
  LQ_HIP(hipMemcpyAsync(staging, src, bytes, hipMemcpyHostToDevice, c->stream));
  *dev = reinterpret_cast<const double*>(staging);
  return LQCD_OK;
}

static int check_finite(lqcd_ctx* c, const double* p, size_t n) {
  unsigned long long* flag = reinterpret_cast<unsigned long long*>(c->dscal) + 4;
  LQ_HIP(hipMemsetAsync(flag, 0, sizeof(unsigned long long), c->stream));
  LQ_TRY(launch_check_finite(c, p, n, reinterpret_cast<double*>(flag)));
  unsigned long long h = 0;
  LQ_HIP(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  if (h) return set_error(LQCD_EINVAL, "input holds NaN or Inf");
  return LQCD_OK;
}

}  // namespace lq

using namespace lq;

extern "C" {

const char* lqcd_strerror(int s) {
  switch (s) {
    case LQCD_OK: return "ok";
    case LQCD_EINVAL: return "invalid argument";
    case LQCD_ENOMEM: return "out of device memory";
    case LQCD_EHIP: return "HIP runtime error";
    case LQCD_ESTATE: return "call out of order";
    case LQCD_ENOCONV: return "solver did not converge";
    case LQCD_EBREAKDOWN: return "solver breakdown";
    case LQCD_ENOTSU3: return "gauge link is not SU(3)";
    case LQCD_ESINGULAR: return "singular clover block";
  }
  return "unknown status";
}

const char* lqcd_last_error(void) { return g_last_error.c_str(); }

void lqcd_default_params(lqcd_solve_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->tol = 1e-10;
  p->max_iter = 100000;
  p->max_outer = 100;
  p->inner_prec = LQCD_F64;
  p->inner_tol = 0.0;
  p->check_every = 8;
  p->use_graph = 1;
  p->x0 = nullptr;
  p->on_device = 0;
  p->reliable_update = 0;
  p->even_odd = 1;
}

int lqcd_create(const int dims[4], int t_bc, void* hip_stream, lqcd_ctx** out) {
  if (!dims || !out) return set_error(LQCD_EINVAL, "null argument");
  *out = nullptr;
  size_t v = 1;
  for (int k = 0; k < 4; ++k) {
    if (dims[k] < 2 || dims[k] % 2 != 0)
      return set_error(LQCD_EINVAL, "every lattice extent must be even and >= 2");
    v *= (size_t)dims[k];
  }
  if (v / 2 >= (size_t)1 << 31) return set_error(LQCD_EINVAL, "lattice too large (2^31 sites per parity max)");
  if (t_bc != 1 && t_bc != -1) return set_error(LQCD_EINVAL, "t_bc must be +1 or -1");
  lqcd_ctx* c = new lqcd_ctx();
  c->g.lx = dims[0];
  c->g.ly = dims[1];
  c->g.lz = dims[2];
  c->g.lt = dims[3];
  c->g.lxh = dims[0] / 2;
  c->g.vh = (int)(v / 2);
  c->g.t_bc = t_bc;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return set_error(LQCD_EHIP, "no HIP device");
  }
  if (hip_stream) {
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return set_error(LQCD_EHIP, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  int s = noalloc_scratch_address(c->device, &c->noalloc_scratch);
  for (int p = 0; p < 3 && s == LQCD_OK; ++p) s = dalloc(&c->gauge[p], 8 * link_bytes(p, c->g.vh));
  if (s == LQCD_OK) s = dalloc(reinterpret_cast<void**>(&c->dscal), 64 * sizeof(double));
  if (s == LQCD_OK && hipHostMalloc(reinterpret_cast<void**>(&c->hscal), 64 * sizeof(double)) != hipSuccess)
    s = set_error(LQCD_ENOMEM, "hipHostMalloc failed");
  if (s == LQCD_OK) s = tune_load_defaults(c);
  if (s != LQCD_OK) {
    lqcd_destroy(c);
    return s;
  }
  *out = c;
  return LQCD_OK;
}

static void drop_mg(lqcd_ctx* c) {
  if (c->mg && c->mg_free) {
    (void)hipStreamSynchronize(c->stream);
    c->mg_free(c->mg);
  }
  c->mg = nullptr;
  c->mg_free = nullptr;
}

int lqcd_destroy(lqcd_ctx* c) {
  if (!c) return LQCD_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->batch && c->batch_free) c->batch_free(c->batch);
  if (c->mg && c->mg_free) c->mg_free(c->mg);
  if (c->ws) {
    c->ws->release();
    delete c->ws;
  }
  for (int p = 0; p < 3; ++p) {
    dfree(c->gauge[p]);
    for (int s = 0; s < 4; ++s) dfree(c->clov[p][s]);
    dfree(c->half_a[p]);
    dfree(c->half_b[p]);
    dfree(c->half_c[p]);
    dfree(c->half_d[p]);
  }
  dfree(c->canon_a);
  dfree(c->canon_b);
  dfree(c->sap_res);
  dfree(c->sap_delta);
  void* d = c->dscal;
  dfree(d);
  if (c->hscal) (void)hipHostFree(c->hscal);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return LQCD_OK;
}

int lqcd_set_gauge(lqcd_ctx* c, const double* U, int on_device) {
  if (!c || !U) return set_error(LQCD_EINVAL, "null argument");
  c->have_gauge = false;
  c->have_clover = false;
  invalidate_graphs(c);
  drop_mg(c);
  const size_t bytes = full_sites(c) * 72 * sizeof(double);  // 4 links x 9 complex per site
  void* staging = nullptr;
  const double* dev = U;
  if (!on_device) {
    LQ_TRY(dalloc(&staging, bytes));
    if (hipMemcpyAsync(staging, U, bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
      dfree(staging);
      return set_error(LQCD_EHIP, "gauge upload failed");
    }
    dev = reinterpret_cast<const double*>(staging);
  }
  int s = check_finite(c, dev, full_sites(c) * 72);
  if (s == LQCD_OK) {
    double* chk = c->dscal;
    if (hipMemsetAsync(chk, 0, 2 * sizeof(unsigned long long), c->stream) != hipSuccess)
      s = set_error(LQCD_EHIP, "memset failed");
    if (s == LQCD_OK) s = launch_import_gauge(c, dev, chk);
    unsigned long long h[2] = {0, 0};
    if (s == LQCD_OK && hipMemcpyAsync(h, chk, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      s = set_error(LQCD_EHIP, "readback failed");
    if (s == LQCD_OK && hipStreamSynchronize(c->stream) != hipSuccess) s = set_error(LQCD_EHIP, "sync failed");
    if (s == LQCD_OK) {
      double err;
      std::memcpy(&err, &h[0], sizeof(err));
      if (h[1]) s = set_error(LQCD_EINVAL, "gauge field holds NaN or Inf");
      else if (!(err <= 1e-12))
        s = set_error(LQCD_ENOTSU3, "a link is not SU(3): max deviation " + std::to_string(err));
    }
  }
  if (staging) {
    (void)hipStreamSynchronize(c->stream);
    dfree(staging);
  }
  if (s == LQCD_OK) c->have_gauge = true;
  return s;
}

int lqcd_set_clover(lqcd_ctx* c, double kappa, double csw) {
  if (!c) return set_error(LQCD_EINVAL, "null argument");
  if (!std::isfinite(kappa) || !std::isfinite(csw)) return set_error(LQCD_EINVAL, "kappa and c_SW must be finite");
  if (!c->have_gauge) return set_error(LQCD_ESTATE, "set_gauge must come first");
  invalidate_graphs(c);
  drop_mg(c);
  c->have_clover = false;
  c->kappa = kappa;
  c->csw = csw;
  c->is_wilson = (csw == 0.0 || kappa == 0.0);
  if (!c->is_wilson) {
    for (int p = 0; p < 3; ++p)
      for (int s = 0; s < 4; ++s) LQ_TRY(dalloc(&c->clov[p][s], clover_bytes(p, c->g.vh)));
    LQ_TRY(build_clover(c, kappa, csw));
  }
  c->have_clover = true;
  return LQCD_OK;
}

static int apply_halves(lqcd_ctx* c, int op, int prec, void* in_e, void* in_o, void* out_e, void* out_o,
                        bool* write_e, bool* write_o) {
  const double k = c->kappa;
  *write_e = *write_o = true;
  switch (op) {
    case LQCD_D: return op_full(c, prec, in_e, in_o, out_e, out_o);
    case LQCD_DEE: *write_o = false; return launch_site(c, prec, clover_slot(c, prec, 0), in_e, out_e);
    case LQCD_DOO: *write_e = false; return launch_site(c, prec, clover_slot(c, prec, 1), in_o, out_o);
    case LQCD_DEE_INV: *write_o = false; return launch_site(c, prec, clover_slot(c, prec, 2), in_e, out_e);
    case LQCD_DOO_INV: *write_e = false; return launch_site(c, prec, clover_slot(c, prec, 3), in_o, out_o);
    case LQCD_DEO: *write_o = false; return op_hop(c, prec, 0, in_o, out_e, -k);
    case LQCD_DOE: *write_e = false; return op_hop(c, prec, 1, in_e, out_o, -k);
    case LQCD_HOP_EO: *write_o = false; return op_hop(c, prec, 0, in_o, out_e, 1.0);
    case LQCD_HOP_OE: *write_e = false; return op_hop(c, prec, 1, in_e, out_o, 1.0);
    case LQCD_DPREC_SCHUR:
      *write_o = false;
      return op_schur(c, prec, in_e, out_e, out_o, RED_NONE, nullptr, nullptr, nullptr, nullptr);
    case LQCD_DPREC_PAPER:
      // D^(eo) = A_ee^-1 S; S into in_o's buffer (free once the input's odd part is unused)
      *write_o = false;
      LQ_TRY(op_schur(c, prec, in_e, in_o, out_o, RED_NONE, nullptr, nullptr, nullptr, nullptr));
      return launch_site(c, prec, clover_slot(c, prec, 2), in_o, out_e);
  }
  return set_error(LQCD_EINVAL, "unknown operator");
}

int lqcd_apply(lqcd_ctx* c, int op, int prec, const double* in, double* out, int on_device) {
  if (!c || !in || !out) return set_error(LQCD_EINVAL, "null argument");
  if (prec < 0 || prec > 2) return set_error(LQCD_EINVAL, "bad precision");
  if (op < LQCD_D || op > LQCD_HOP_OE) return set_error(LQCD_EINVAL, "unknown operator");
  if (!c->have_gauge || !c->have_clover) return set_error(LQCD_ESTATE, "set_gauge and set_clover must come first");
  LQ_TRY(ensure_apply_buffers(c, prec));
  const size_t bytes = full_sites(c) * 192;
  const double* din = nullptr;
  LQ_TRY(stage_in(c, in, on_device, c->canon_a, bytes, &din));
  double* dout = on_device ? out : reinterpret_cast<double*>(c->canon_b);
  void *ie = c->half_a[prec], *io = c->half_b[prec], *oe = c->half_c[prec], *oo = c->half_d[prec];
  LQ_TRY(launch_import_spinor(c, prec, 0, din, ie));
  LQ_TRY(launch_import_spinor(c, prec, 1, din, io));
  bool we = true, wo = true;
  LQ_TRY(apply_halves(c, op, prec, ie, io, oe, oo, &we, &wo));
  if (we) LQ_TRY(launch_export_spinor(c, prec, 0, oe, dout));
  else LQ_TRY(launch_zero_parity(c, 0, dout));
  if (wo) LQ_TRY(launch_export_spinor(c, prec, 1, oo, dout));
  else LQ_TRY(launch_zero_parity(c, 1, dout));
  if (!on_device) {
    LQ_HIP(hipMemcpyAsync(out, dout, bytes, hipMemcpyDeviceToHost, c->stream));
    LQ_HIP(hipStreamSynchronize(c->stream));
  }
  return LQCD_OK;
}

static int validate_params(const lqcd_solve_params* p) {
  if (!p) return LQCD_OK;
  if (!(p->tol > 0) || p->inner_prec < 0 || p->inner_prec > 2 || p->max_iter < 1 || p->max_outer < 1 ||
      p->inner_tol < 0 || !(p->inner_tol < 1) || p->even_odd < 0 || p->even_odd > 1)
    return set_error(LQCD_EINVAL, "bad solver parameters");
  return LQCD_OK;
}

int lqcd_solve(lqcd_ctx* c, const double* b, double* x, const lqcd_solve_params* prm_in, lqcd_solve_stats* stats) {
  if (!c || !b || !x) return set_error(LQCD_EINVAL, "null argument");
  LQ_TRY(validate_params(prm_in));
  lqcd_solve_params prm;
  if (prm_in) prm = *prm_in;
  else lqcd_default_params(&prm);
  if (!c->have_gauge || !c->have_clover) return set_error(LQCD_ESTATE, "set_gauge and set_clover must come first");
  if (!prm.even_odd && prm.inner_prec != LQCD_F64)
    return set_error(LQCD_EINVAL, "the unpreconditioned solve (even_odd = 0) runs in FP64 only");
  LQ_TRY(ensure_apply_buffers(c, 0));
  LQ_TRY(ensure_workspace(c, prm.inner_prec));
  Workspace* w = c->ws;
  const size_t bytes = full_sites(c) * 192;
  const double* db = nullptr;
  LQ_TRY(stage_in(c, b, prm.on_device, c->canon_a, bytes, &db));
  LQ_TRY(check_finite(c, db, full_sites(c) * 24));
  LQ_TRY(launch_import_spinor(c, 0, 0, db, w->b_e));
  LQ_TRY(launch_import_spinor(c, 0, 1, db, w->b_o));
  if (prm.x0) {
    const double* dx0 = nullptr;
    LQ_TRY(stage_in(c, prm.x0, prm.on_device, c->canon_b, bytes, &dx0));
    LQ_TRY(launch_import_spinor(c, 0, 0, dx0, w->x_e));
    if (!prm.even_odd) LQ_TRY(launch_import_spinor(c, 0, 1, dx0, w->x_o));
  } else {
    LQ_TRY(blas_zero(c, 0, w->x_e));
  }
  lqcd_solve_stats st{};
  int status;
  if (prm.even_odd) {
    status = solve_native(c, prm, st);
  } else {
    // BiCGStab on the full operator D: the flexible BiCGStab without a
    // preconditioner; its counts mapped to lqcd_solve's (iterations, passes)
    status = solve_flexible(c, prm, FlexPrecond(), "plain", w->b_e, w->b_o, w->x_e, w->x_o, !prm.x0, st);
    st.inner_iters = st.outer_iters;
    st.outer_iters = st.restarts + 1;
  }
  if (status != LQCD_OK && status != LQCD_ENOCONV && status != LQCD_EBREAKDOWN) return status;
  double* dx = prm.on_device ? x : reinterpret_cast<double*>(c->canon_b);
  LQ_TRY(launch_export_spinor(c, 0, 0, w->x_e, dx));
  LQ_TRY(launch_export_spinor(c, 0, 1, w->x_o, dx));
  if (!prm.on_device) LQ_HIP(hipMemcpyAsync(x, dx, bytes, hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  if (stats) *stats = st;
  return status;
}

static int validate_sap(const lqcd_ctx* c, const lqcd_sap_params* sp) {
  if (!sp) return set_error(LQCD_EINVAL, "null SAP parameters");
  if (!sap_shape_ok(c->g, sp->block))
    return set_error(LQCD_EINVAL, "SAP blocks must tile the lattice with an even number per direction and "
                                  "64, 128, 192 or 256 sites per block");
  if (sp->ncycles < 1 || sp->nmr < 1) return set_error(LQCD_EINVAL, "SAP needs ncycles >= 1 and nmr >= 1");
  return LQCD_OK;
}

int lqcd_apply_sap(lqcd_ctx* c, const lqcd_sap_params* sp, const double* eta, double* psi, int on_device) {
  if (!c || !eta || !psi) return set_error(LQCD_EINVAL, "null argument");
  LQ_TRY(validate_sap(c, sp));
  if (!c->have_gauge || !c->have_clover) return set_error(LQCD_ESTATE, "set_gauge and set_clover must come first");
  LQ_TRY(ensure_apply_buffers(c, 1));
  const size_t bytes = full_sites(c) * 192;
  const double* din = nullptr;
  LQ_TRY(stage_in(c, eta, on_device, c->canon_a, bytes, &din));
  double* dout = on_device ? psi : reinterpret_cast<double*>(c->canon_b);
  void *ie = c->half_a[1], *io = c->half_b[1], *oe = c->half_c[1], *oo = c->half_d[1];
  LQ_TRY(launch_import_spinor(c, 1, 0, din, ie));
  LQ_TRY(launch_import_spinor(c, 1, 1, din, io));
  LQ_TRY(sap_apply(c, sp->block, sp->ncycles, sp->nmr, ie, io, oe, oo));
  LQ_TRY(launch_export_spinor(c, 1, 0, oe, dout));
  LQ_TRY(launch_export_spinor(c, 1, 1, oo, dout));
  if (!on_device) {
    LQ_HIP(hipMemcpyAsync(psi, dout, bytes, hipMemcpyDeviceToHost, c->stream));
    LQ_HIP(hipStreamSynchronize(c->stream));
  }
  return LQCD_OK;
}

int lqcd_solve_sap(lqcd_ctx* c, const double* b, double* x, const lqcd_solve_params* prm_in,
                   const lqcd_sap_params* sp, lqcd_solve_stats* stats) {
  if (!c || !b || !x) return set_error(LQCD_EINVAL, "null argument");
  LQ_TRY(validate_params(prm_in));
  LQ_TRY(validate_sap(c, sp));
  lqcd_solve_params prm;
  if (prm_in) prm = *prm_in;
  else lqcd_default_params(&prm);
  if (!c->have_gauge || !c->have_clover) return set_error(LQCD_ESTATE, "set_gauge and set_clover must come first");
  LQ_TRY(ensure_apply_buffers(c, 0));
  const size_t bytes = full_sites(c) * 192;
  const double* db = nullptr;
  LQ_TRY(stage_in(c, b, prm.on_device, c->canon_a, bytes, &db));
  LQ_TRY(check_finite(c, db, full_sites(c) * 24));
  void *be = c->half_a[0], *bo = c->half_b[0], *xe = c->half_c[0], *xo = c->half_d[0];
  LQ_TRY(launch_import_spinor(c, 0, 0, db, be));
  LQ_TRY(launch_import_spinor(c, 0, 1, db, bo));
  if (prm.x0) {
    const double* dx0 = nullptr;
    LQ_TRY(stage_in(c, prm.x0, prm.on_device, c->canon_b, bytes, &dx0));
    LQ_TRY(launch_import_spinor(c, 0, 0, dx0, xe));
    LQ_TRY(launch_import_spinor(c, 0, 1, dx0, xo));
  }
  lqcd_solve_stats st{};
  const int status = solve_sap(c, prm, sp->block, sp->ncycles, sp->nmr, be, bo, xe, xo, prm.x0 == nullptr, st);
  if (status != LQCD_OK && status != LQCD_ENOCONV && status != LQCD_EBREAKDOWN) return status;
  double* dx = prm.on_device ? x : reinterpret_cast<double*>(c->canon_b);
  LQ_TRY(launch_export_spinor(c, 0, 0, xe, dx));
  LQ_TRY(launch_export_spinor(c, 0, 1, xo, dx));
  if (!prm.on_device) LQ_HIP(hipMemcpyAsync(x, dx, bytes, hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  if (stats) *stats = st;
  return status;
}

int lqcd_stag_apply(lqcd_ctx* c, int op, int prec, double mass, const double* in, double* out, int on_device) {
  if (!c || !in || !out) return set_error(LQCD_EINVAL, "null argument");
  if (prec != 0 && prec != 1) return set_error(LQCD_EINVAL, "staggered operator: precision must be F64 or F32");
  if (op != LQCD_STAG_D && op != LQCD_STAG_SCHUR) return set_error(LQCD_EINVAL, "unknown staggered operator");
  if (!std::isfinite(mass)) return set_error(LQCD_EINVAL, "mass must be finite");
  if (!c->have_gauge) return set_error(LQCD_ESTATE, "set_gauge must come first");
  LQ_TRY(ensure_canon(c));
  const size_t bytes = full_sites(c) * 48;
  const double* din = nullptr;
  LQ_TRY(stage_in(c, in, on_device, c->canon_a, bytes, &din));
  double* dout = on_device ? out : reinterpret_cast<double*>(c->canon_b);
  const size_t hb = stag_field_bytes(prec, c->g.vh);
  void* h[5] = {};
  int st = LQCD_OK;
  for (auto& p : h) {
    if (hipMalloc(&p, hb) != hipSuccess) {
      (void)hipGetLastError();
      st = set_error(LQCD_ENOMEM, "staggered apply buffers");
      break;
    }
  }
  if (st == LQCD_OK) st = stag_import(c, prec, 0, din, h[0]);
  if (st == LQCD_OK) st = stag_import(c, prec, 1, din, h[1]);
  if (st == LQCD_OK && op == LQCD_STAG_D) {
    st = stag_hop(c, prec, 0, h[1], h[0], mass, 1.0, h[2]);
    if (st == LQCD_OK) st = stag_hop(c, prec, 1, h[0], h[1], mass, 1.0, h[3]);
    if (st == LQCD_OK) st = stag_export(c, prec, 0, h[2], dout);
    if (st == LQCD_OK) st = stag_export(c, prec, 1, h[3], dout);
  } else if (st == LQCD_OK) {
    st = stag_schur(c, prec, mass, h[0], h[4], h[2]);
    if (st == LQCD_OK && hipMemsetAsync(dout, 0, bytes, c->stream) != hipSuccess) st = set_error(LQCD_EHIP, "memset");
    if (st == LQCD_OK) st = stag_export(c, prec, 0, h[2], dout);
  }
  if (st == LQCD_OK && !on_device) {
    if (hipMemcpyAsync(out, dout, bytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      st = set_error(LQCD_EHIP, "copy back");
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess && st == LQCD_OK) st = set_error(LQCD_EHIP, "synchronise");
  for (void* p : h)
    if (p) (void)hipFree(p);
  return st;
}

int lqcd_stag_solve(lqcd_ctx* c, double mass, const double* b, double* x, const lqcd_solve_params* prm_in,
                    lqcd_solve_stats* stats) {
  if (!c || !b || !x) return set_error(LQCD_EINVAL, "null argument");
  LQ_TRY(validate_params(prm_in));
  if (!(mass > 0) || !std::isfinite(mass)) return set_error(LQCD_EINVAL, "staggered solve needs a finite mass > 0");
  lqcd_solve_params prm;
  if (prm_in) prm = *prm_in;
  else lqcd_default_params(&prm);
  if (prm.inner_prec != LQCD_F64 && prm.inner_prec != LQCD_F32)
    return set_error(LQCD_EINVAL, "staggered solve: inner precision must be F64 or F32");
  if (!c->have_gauge) return set_error(LQCD_ESTATE, "set_gauge must come first");
  LQ_TRY(ensure_canon(c));
  const size_t bytes = full_sites(c) * 48;
  const double* db = nullptr;
  LQ_TRY(stage_in(c, b, prm.on_device, c->canon_a, bytes, &db));
  LQ_TRY(check_finite(c, db, full_sites(c) * 6));
  const size_t hb = stag_field_bytes(0, c->g.vh);
  void* h[4] = {};
  int st = LQCD_OK;
  for (auto& p : h) {
    if (hipMalloc(&p, hb) != hipSuccess) {
      (void)hipGetLastError();
      st = set_error(LQCD_ENOMEM, "staggered solve buffers");
      break;
    }
  }
  if (st == LQCD_OK) st = stag_import(c, 0, 0, db, h[0]);
  if (st == LQCD_OK) st = stag_import(c, 0, 1, db, h[1]);
  lqcd_solve_stats ss{};
  int status = st;
  if (st == LQCD_OK) {
    status = stag_solve(c, mass, prm, h[0], h[1], h[2], h[3], ss);
    if (status == LQCD_OK || status == LQCD_ENOCONV || status == LQCD_EBREAKDOWN) {
      double* dx = prm.on_device ? x : reinterpret_cast<double*>(c->canon_b);
      st = stag_export(c, 0, 0, h[2], dx);
      if (st == LQCD_OK) st = stag_export(c, 0, 1, h[3], dx);
      if (st == LQCD_OK && !prm.on_device &&
          hipMemcpyAsync(x, dx, bytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        st = set_error(LQCD_EHIP, "copy back");
      if (st != LQCD_OK) status = st;
    }
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess && status == LQCD_OK) status = set_error(LQCD_EHIP, "synchronise");
  for (void* p : h)
    if (p) (void)hipFree(p);
  if (stats) *stats = ss;
  return status;
}

static int validate_dwf(const lqcd_dwf_params* d) {
  if (!d) return set_error(LQCD_EINVAL, "null domain-wall parameters");
  if (d->Ls < 1 || d->Ls > 256 || !std::isfinite(d->M5) || !std::isfinite(d->mf) || !std::isfinite(d->b5) ||
      !std::isfinite(d->c5))
    return set_error(LQCD_EINVAL, "domain wall: Ls must be 1..256, M5, mf, b5 and c5 finite");
  return LQCD_OK;
}

// device buffers freed on scope exit
struct Bufs {
  std::vector<void*> p;
  ~Bufs() {
    for (void* q : p) (void)hipFree(q);
  }
  int get(lqcd_ctx* c, size_t bytes, void** out) {
    if (hipMalloc(out, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(LQCD_ENOMEM, "device buffer allocation failed");
    }
    p.push_back(*out);
    LQ_HIP(hipMemsetAsync(*out, 0, bytes, c->stream));
    return LQCD_OK;
  }
};

int lqcd_dwf_apply(lqcd_ctx* c, const lqcd_dwf_params* d, int dag, int prec, const double* in, double* out,
                   int on_device) {
  if (!c || !in || !out) return set_error(LQCD_EINVAL, "null argument");
  LQ_TRY(validate_dwf(d));
  if (prec != 0 && prec != 1) return set_error(LQCD_EINVAL, "domain-wall operator: precision must be F64 or F32");
  if (dag != 0 && dag != 1) return set_error(LQCD_EINVAL, "dag must be 0 or 1");
  if (!c->have_gauge) return set_error(LQCD_ESTATE, "set_gauge must come first");
  const size_t cbytes = full_sites(c) * 192 * (size_t)d->Ls;
  const size_t fb = dwf_field_bytes(prec, c->g.vh, d->Ls);
  Bufs b;
  void *cin = nullptr, *cout = nullptr, *f[3];
  const double* din = in;
  double* dout = out;
  if (!on_device) {
    LQ_TRY(b.get(c, cbytes, &cin));
    LQ_TRY(b.get(c, cbytes, &cout));
    LQ_HIP(hipMemcpyAsync(cin, in, cbytes, hipMemcpyHostToDevice, c->stream));
    din = reinterpret_cast<const double*>(cin);
    dout = reinterpret_cast<double*>(cout);
  }
  for (auto& q : f) LQ_TRY(b.get(c, fb, &q));
  LQ_TRY(dwf_import(c, prec, d->Ls, din, f[0]));
  LQ_TRY(dwf_apply(c, prec, *d, dag, f[0], f[1], f[2]));
  LQ_TRY(dwf_export(c, prec, d->Ls, f[1], dout));
  if (!on_device) LQ_HIP(hipMemcpyAsync(out, dout, cbytes, hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  return LQCD_OK;
}

int lqcd_dwf_solve(lqcd_ctx* c, const lqcd_dwf_params* d, const double* b, double* x,
                   const lqcd_solve_params* prm_in, lqcd_solve_stats* stats) {
  if (!c || !b || !x) return set_error(LQCD_EINVAL, "null argument");
  LQ_TRY(validate_dwf(d));
  LQ_TRY(validate_params(prm_in));
  lqcd_solve_params prm;
  if (prm_in) prm = *prm_in;
  else lqcd_default_params(&prm);
  if (!c->have_gauge) return set_error(LQCD_ESTATE, "set_gauge must come first");
  const size_t cbytes = full_sites(c) * 192 * (size_t)d->Ls;
  const size_t fb = dwf_field_bytes(0, c->g.vh, d->Ls);
  Bufs bf;
  void *cb = nullptr, *cx_ = nullptr, *fbn, *fx;
  const double* db = b;
  double* dx = x;
  if (!prm.on_device) {
    LQ_TRY(bf.get(c, cbytes, &cb));
    LQ_TRY(bf.get(c, cbytes, &cx_));
    LQ_HIP(hipMemcpyAsync(cb, b, cbytes, hipMemcpyHostToDevice, c->stream));
    db = reinterpret_cast<const double*>(cb);
    dx = reinterpret_cast<double*>(cx_);
  }
  LQ_TRY(check_finite(c, db, full_sites(c) * 24 * (size_t)d->Ls));
  LQ_TRY(bf.get(c, fb, &fbn));
  LQ_TRY(bf.get(c, fb, &fx));
  LQ_TRY(dwf_import(c, 0, d->Ls, db, fbn));
  lqcd_solve_stats st{};
  const int status = dwf_solve(c, *d, prm, fbn, fx, st);
  if (status != LQCD_OK && status != LQCD_ENOCONV && status != LQCD_EBREAKDOWN) return status;
  LQ_TRY(dwf_export(c, 0, d->Ls, fx, dx));
  if (!prm.on_device) LQ_HIP(hipMemcpyAsync(x, dx, cbytes, hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  if (stats) *stats = st;
  return status;
}

int lqcd_dwf_apply_schur(lqcd_ctx* c, const lqcd_dwf_params* d, int dag, int prec, const double* in, double* out,
                         int on_device) {
  if (!c || !in || !out) return set_error(LQCD_EINVAL, "null argument");
  LQ_TRY(validate_dwf(d));
  if (prec != 0 && prec != 1) return set_error(LQCD_EINVAL, "domain-wall operator: precision must be F64 or F32");
  if (dag != 0 && dag != 1) return set_error(LQCD_EINVAL, "dag must be 0 or 1");
  if (!c->have_gauge) return set_error(LQCD_ESTATE, "set_gauge must come first");
  const size_t cbytes = full_sites(c) * 192 * (size_t)d->Ls;
  const size_t fb = dwf_field_bytes(prec, c->g.vh, d->Ls);
  Bufs b;
  void *cin = nullptr, *cout = nullptr, *f[4];
  const double* din = in;
  double* dout = out;
  if (!on_device) {
    LQ_TRY(b.get(c, cbytes, &cin));
    LQ_TRY(b.get(c, cbytes, &cout));
    LQ_HIP(hipMemcpyAsync(cin, in, cbytes, hipMemcpyHostToDevice, c->stream));
    din = reinterpret_cast<const double*>(cin);
    dout = reinterpret_cast<double*>(cout);
  }
  for (auto& q : f) LQ_TRY(b.get(c, fb, &q));  // zeroed: the odd half of the result stays zero
  LQ_TRY(dwf_import(c, prec, d->Ls, din, f[0]));
  LQ_TRY(dwf_schur_apply(c, prec, *d, dag, f[0], f[1], f[2], f[3]));
  LQ_TRY(dwf_export(c, prec, d->Ls, f[1], dout));
  if (!on_device) LQ_HIP(hipMemcpyAsync(out, dout, cbytes, hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  return LQCD_OK;
}

int lqcd_dwf_solve_eo(lqcd_ctx* c, const lqcd_dwf_params* d, const double* b, double* x,
                      const lqcd_solve_params* prm_in, lqcd_solve_stats* stats) {
  if (!c || !b || !x) return set_error(LQCD_EINVAL, "null argument");
  LQ_TRY(validate_dwf(d));
  LQ_TRY(validate_params(prm_in));
  lqcd_solve_params prm;
  if (prm_in) prm = *prm_in;
  else lqcd_default_params(&prm);
  if (prm.inner_prec != LQCD_F64 && prm.inner_prec != LQCD_F32)
    return set_error(LQCD_EINVAL, "domain-wall even-odd solve: inner precision must be F64 or F32");
  if (!c->have_gauge) return set_error(LQCD_ESTATE, "set_gauge must come first");
  const size_t cbytes = full_sites(c) * 192 * (size_t)d->Ls;
  const size_t fb = dwf_field_bytes(0, c->g.vh, d->Ls);
  Bufs bf;
  void *cb = nullptr, *cx_ = nullptr, *fbn, *fx;
  const double* db = b;
  double* dx = x;
  if (!prm.on_device) {
    LQ_TRY(bf.get(c, cbytes, &cb));
    LQ_TRY(bf.get(c, cbytes, &cx_));
    LQ_HIP(hipMemcpyAsync(cb, b, cbytes, hipMemcpyHostToDevice, c->stream));
    db = reinterpret_cast<const double*>(cb);
    dx = reinterpret_cast<double*>(cx_);
  }
  LQ_TRY(check_finite(c, db, full_sites(c) * 24 * (size_t)d->Ls));
  LQ_TRY(bf.get(c, fb, &fbn));
  LQ_TRY(bf.get(c, fb, &fx));
  LQ_TRY(dwf_import(c, 0, d->Ls, db, fbn));
  lqcd_solve_stats st{};
  const int status = dwf_solve_eo(c, *d, prm, fbn, fx, st);
  if (status != LQCD_OK && status != LQCD_ENOCONV && status != LQCD_EBREAKDOWN) return status;
  LQ_TRY(dwf_export(c, 0, d->Ls, fx, dx));
  if (!prm.on_device) LQ_HIP(hipMemcpyAsync(x, dx, cbytes, hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  if (stats) *stats = st;
  return status;
}

size_t lqcd_dwf_field_bytes(lqcd_ctx* c, int prec, int Ls) {
  if (!c || (prec != 0 && prec != 1) || Ls < 1 || Ls > 256) return 0;
  return dwf_field_bytes(prec, c->g.vh, Ls);
}

int lqcd_dwf_import(lqcd_ctx* c, int prec, int Ls, const double* canon, void* native) {
  if (!c || !canon || !native) return set_error(LQCD_EINVAL, "null argument");
  if ((prec != 0 && prec != 1) || Ls < 1 || Ls > 256) return set_error(LQCD_EINVAL, "bad precision or Ls");
  return dwf_import(c, prec, Ls, canon, native);
}

int lqcd_dwf_export(lqcd_ctx* c, int prec, int Ls, const void* native, double* canon) {
  if (!c || !canon || !native) return set_error(LQCD_EINVAL, "null argument");
  if ((prec != 0 && prec != 1) || Ls < 1 || Ls > 256) return set_error(LQCD_EINVAL, "bad precision or Ls");
  return dwf_export(c, prec, Ls, native, canon);
}

int lqcd_dwf_apply_native(lqcd_ctx* c, const lqcd_dwf_params* d, int dag, int prec, const void* in, void* out,
                          void* tmp) {
  if (!c || !in || !out) return set_error(LQCD_EINVAL, "null argument");
  if (in == out || (tmp && (tmp == in || tmp == out)))
    return set_error(LQCD_EINVAL, "domain-wall operator: in, out and tmp must be different fields");
  LQ_TRY(validate_dwf(d));
  if ((prec != 0 && prec != 1) || (dag != 0 && dag != 1)) return set_error(LQCD_EINVAL, "bad precision or dag");
  if (!c->have_gauge) return set_error(LQCD_ESTATE, "set_gauge must come first");
  return dwf_apply(c, prec, *d, dag, in, out, tmp);
}

static int validate_mg(const lqcd_ctx* c, const lqcd_mg_params* mp) {
  if (!mp) return set_error(LQCD_EINVAL, "null multigrid parameters");
  if (!mg_shape_ok(c->g, mp->agg))
    return set_error(LQCD_EINVAL, "aggregates must have extents >= 2, tile the lattice with an even number per "
                                  "direction and hold at most 256 sites");
  if (mp->nvec < 1 || mp->nvec > 24) return set_error(LQCD_EINVAL, "multigrid needs 1 to 24 test vectors");
  if (mp->setup_iters < 0 || mp->setup_iters > 100) return set_error(LQCD_EINVAL, "setup_iters must be 0..100");
  if (!(mp->coarse_tol > 0.0 && mp->coarse_tol < 1.0) || mp->coarse_max_iter < 1)
    return set_error(LQCD_EINVAL, "coarse_tol must be in (0, 1) and coarse_max_iter >= 1");
  return validate_sap(c, &mp->sap);
}

int lqcd_mg_setup(lqcd_ctx* c, const lqcd_mg_params* mp, const double* start, int on_device) {
  if (!c || !start) return set_error(LQCD_EINVAL, "null argument");
  LQ_TRY(validate_mg(c, mp));
  if (!c->have_gauge || !c->have_clover) return set_error(LQCD_ESTATE, "set_gauge and set_clover must come first");
  LQ_TRY(ensure_apply_buffers(c, 1));
  const size_t n = full_sites(c) * 24 * (size_t)mp->nvec;
  Bufs bf;
  const double* ds = start;
  if (!on_device) {
    void* d = nullptr;
    LQ_TRY(bf.get(c, n * sizeof(double), &d));
    LQ_HIP(hipMemcpyAsync(d, start, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    ds = reinterpret_cast<const double*>(d);
  }
  LQ_TRY(check_finite(c, ds, n));
  const int status = mg_setup(c, *mp, ds);
  if (status != LQCD_OK) drop_mg(c);
  return status;
}

size_t lqcd_mg_coarse_size(lqcd_ctx* c) { return c ? mg_coarse_size(c) : 0; }

// canonical fine field (host or device) -> FP32 native halves half_a[1], half_b[1]
static int mg_stage_fine(lqcd_ctx* c, const double* in, int on_device) {
  LQ_TRY(ensure_apply_buffers(c, 1));
  const double* din = nullptr;
  LQ_TRY(stage_in(c, in, on_device, c->canon_a, full_sites(c) * 192, &din));
  LQ_TRY(launch_import_spinor(c, 1, 0, din, c->half_a[1]));
  return launch_import_spinor(c, 1, 1, din, c->half_b[1]);
}

// FP32 native halves half_c[1], half_d[1] -> canonical fine field (host or device)
static int mg_unstage_fine(lqcd_ctx* c, double* out, int on_device) {
  const size_t bytes = full_sites(c) * 192;
  double* dout = on_device ? out : reinterpret_cast<double*>(c->canon_b);
  LQ_TRY(launch_export_spinor(c, 1, 0, c->half_c[1], dout));
  LQ_TRY(launch_export_spinor(c, 1, 1, c->half_d[1], dout));
  if (!on_device) LQ_HIP(hipMemcpyAsync(out, dout, bytes, hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  return LQCD_OK;
}

// a coarse complex128 vector (host or device) -> FP32 complex device vector
static int mg_stage_coarse(lqcd_ctx* c, Bufs& bf, const double* in, int on_device, void** f32) {
  const size_t nc = mg_coarse_size(c);
  LQ_TRY(bf.get(c, nc * 8, f32));
  const double* din = in;
  if (!on_device) {
    void* d = nullptr;
    LQ_TRY(bf.get(c, nc * 16, &d));
    LQ_HIP(hipMemcpyAsync(d, in, nc * 16, hipMemcpyHostToDevice, c->stream));
    din = reinterpret_cast<const double*>(d);
  }
  return mg_coarse_convert(c, din, true, *f32, nc);
}

static int mg_unstage_coarse(lqcd_ctx* c, Bufs& bf, const void* f32, double* out, int on_device) {
  const size_t nc = mg_coarse_size(c);
  double* dout = out;
  if (!on_device) {
    void* d = nullptr;
    LQ_TRY(bf.get(c, nc * 16, &d));
    dout = reinterpret_cast<double*>(d);
  }
  LQ_TRY(mg_coarse_convert(c, f32, false, dout, nc));
  if (!on_device) LQ_HIP(hipMemcpyAsync(out, dout, nc * 16, hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  return LQCD_OK;
}

int lqcd_mg_restrict(lqcd_ctx* c, const double* fine, double* coarse, int on_device) {
  if (!c || !fine || !coarse) return set_error(LQCD_EINVAL, "null argument");
  if (!c->mg) return set_error(LQCD_ESTATE, "lqcd_mg_setup must come first");
  LQ_TRY(mg_stage_fine(c, fine, on_device));
  Bufs bf;
  void* rc = nullptr;
  LQ_TRY(bf.get(c, mg_coarse_size(c) * 8, &rc));
  LQ_TRY(mg_restrict(c, c->half_a[1], c->half_b[1], rc));
  return mg_unstage_coarse(c, bf, rc, coarse, on_device);
}

int lqcd_mg_prolong(lqcd_ctx* c, const double* coarse, double* fine, int on_device) {
  if (!c || !fine || !coarse) return set_error(LQCD_EINVAL, "null argument");
  if (!c->mg) return set_error(LQCD_ESTATE, "lqcd_mg_setup must come first");
  LQ_TRY(ensure_apply_buffers(c, 1));
  Bufs bf;
  void* ec = nullptr;
  LQ_TRY(mg_stage_coarse(c, bf, coarse, on_device, &ec));
  LQ_TRY(mg_prolong(c, ec, c->half_c[1], c->half_d[1]));
  return mg_unstage_fine(c, fine, on_device);
}

int lqcd_mg_coarse_apply(lqcd_ctx* c, const double* in, double* out, int on_device) {
  if (!c || !in || !out) return set_error(LQCD_EINVAL, "null argument");
  if (!c->mg) return set_error(LQCD_ESTATE, "lqcd_mg_setup must come first");
  Bufs bf;
  void *x = nullptr, *y = nullptr;
  LQ_TRY(mg_stage_coarse(c, bf, in, on_device, &x));
  LQ_TRY(bf.get(c, mg_coarse_size(c) * 8, &y));
  LQ_TRY(mg_coarse_apply(c, x, y));
  return mg_unstage_coarse(c, bf, y, out, on_device);
}

int lqcd_mg_apply(lqcd_ctx* c, const double* r, double* x, int on_device) {
  if (!c || !r || !x) return set_error(LQCD_EINVAL, "null argument");
  if (!c->mg) return set_error(LQCD_ESTATE, "lqcd_mg_setup must come first");
  LQ_TRY(mg_stage_fine(c, r, on_device));
  LQ_TRY(mg_precond(c, c->half_a[1], c->half_b[1], c->half_c[1], c->half_d[1], nullptr));
  return mg_unstage_fine(c, x, on_device);
}

int lqcd_solve_mg(lqcd_ctx* c, const double* b, double* x, const lqcd_solve_params* prm_in, lqcd_solve_stats* stats) {
  if (!c || !b || !x) return set_error(LQCD_EINVAL, "null argument");
  LQ_TRY(validate_params(prm_in));
  if (!c->mg) return set_error(LQCD_ESTATE, "lqcd_mg_setup must come first");
  lqcd_solve_params prm;
  if (prm_in) prm = *prm_in;
  else lqcd_default_params(&prm);
  LQ_TRY(ensure_apply_buffers(c, 0));
  const size_t bytes = full_sites(c) * 192;
  const double* db = nullptr;
  LQ_TRY(stage_in(c, b, prm.on_device, c->canon_a, bytes, &db));
  LQ_TRY(check_finite(c, db, full_sites(c) * 24));
  void *be = c->half_a[0], *bo = c->half_b[0], *xe = c->half_c[0], *xo = c->half_d[0];
  LQ_TRY(launch_import_spinor(c, 0, 0, db, be));
  LQ_TRY(launch_import_spinor(c, 0, 1, db, bo));
  if (prm.x0) {
    const double* dx0 = nullptr;
    LQ_TRY(stage_in(c, prm.x0, prm.on_device, c->canon_b, bytes, &dx0));
    LQ_TRY(launch_import_spinor(c, 0, 0, dx0, xe));
    LQ_TRY(launch_import_spinor(c, 0, 1, dx0, xo));
  }
  lqcd_solve_stats st{};
  long coarse = 0;
  const int status = solve_mg(c, prm, be, bo, xe, xo, prm.x0 == nullptr, st, &coarse);
  if (status != LQCD_OK && status != LQCD_ENOCONV && status != LQCD_EBREAKDOWN) return status;
  double* dx = prm.on_device ? x : reinterpret_cast<double*>(c->canon_b);
  LQ_TRY(launch_export_spinor(c, 0, 0, xe, dx));
  LQ_TRY(launch_export_spinor(c, 0, 1, xo, dx));
  if (!prm.on_device) LQ_HIP(hipMemcpyAsync(x, dx, bytes, hipMemcpyDeviceToHost, c->stream));
  LQ_HIP(hipStreamSynchronize(c->stream));
  if (stats) *stats = st;
  return status;
}

size_t lqcd_stag_field_bytes(lqcd_ctx* c, int prec) {
  if (!c || (prec != 0 && prec != 1)) return 0;
  return stag_field_bytes(prec, c->g.vh);
}

int lqcd_stag_import(lqcd_ctx* c, int prec, int parity, const double* canon, void* native) {
  if (!c || !canon || !native) return set_error(LQCD_EINVAL, "null argument");
  if ((prec != 0 && prec != 1) || (parity != 0 && parity != 1)) return set_error(LQCD_EINVAL, "bad precision or parity");
  return stag_import(c, prec, parity, canon, native);
}

int lqcd_stag_export(lqcd_ctx* c, int prec, int parity, const void* native, double* canon) {
  if (!c || !canon || !native) return set_error(LQCD_EINVAL, "null argument");
  if ((prec != 0 && prec != 1) || (parity != 0 && parity != 1)) return set_error(LQCD_EINVAL, "bad precision or parity");
  return stag_export(c, prec, parity, native, canon);
}

int lqcd_stag_hop_native(lqcd_ctx* c, int prec, int out_parity, const void* in, void* out) {
  if (!c || !in || !out) return set_error(LQCD_EINVAL, "null argument");
  if ((prec != 0 && prec != 1) || (out_parity != 0 && out_parity != 1))
    return set_error(LQCD_EINVAL, "bad precision or parity");
  if (!c->have_gauge) return set_error(LQCD_ESTATE, "set_gauge must come first");
  return stag_hop(c, prec, out_parity, in, nullptr, 0.0, 1.0, out);
}

size_t lqcd_field_bytes(lqcd_ctx* c, int prec) {
  if (!c || prec < 0 || prec > 2) return 0;
  return spinor_bytes(prec, c->g.vh);
}

int lqcd_import(lqcd_ctx* c, int prec, int parity, const double* canon, void* native) {
  if (!c || !canon || !native) return set_error(LQCD_EINVAL, "null argument");
  if (prec < 0 || prec > 2 || (parity != 0 && parity != 1)) return set_error(LQCD_EINVAL, "bad precision or parity");
  return launch_import_spinor(c, prec, parity, canon, native);
}

int lqcd_export(lqcd_ctx* c, int prec, int parity, const void* native, double* canon) {
  if (!c || !canon || !native) return set_error(LQCD_EINVAL, "null argument");
  if (prec < 0 || prec > 2 || (parity != 0 && parity != 1)) return set_error(LQCD_EINVAL, "bad precision or parity");
  return launch_export_spinor(c, prec, parity, native, canon);
}

int lqcd_apply_native(lqcd_ctx* c, int op, int prec, const void* in, void* out) {
  if (!c || !in || !out) return set_error(LQCD_EINVAL, "null argument");
  if (prec < 0 || prec > 2) return set_error(LQCD_EINVAL, "bad precision");
  if (in == out) return set_error(LQCD_EINVAL, "in and out must differ");
  if (!c->have_gauge || !c->have_clover) return set_error(LQCD_ESTATE, "set_gauge and set_clover must come first");
  void* tmp = nullptr;
  if (op == LQCD_DPREC_SCHUR) {
    LQ_TRY(dalloc(&c->half_d[prec], spinor_bytes(prec, c->g.vh)));
    tmp = c->half_d[prec];
  }
  return op_native(c, op, prec, in, out, tmp);
}

int lqcd_apply_native_noalloc(lqcd_ctx* c, int op, int prec, const void* in, void* out) {
  if (!c || !in || !out) return set_error(LQCD_EINVAL, "null argument");
  if (prec < 0 || prec > 2) return set_error(LQCD_EINVAL, "bad precision");
  if (in == out) return set_error(LQCD_EINVAL, "in and out must differ");
  void* tmp = nullptr;
  if (op == LQCD_DPREC_SCHUR) {
    const size_t need = spinor_bytes(prec, c->g.vh);
    if (need > NOALLOC_SCRATCH_BYTES)
      return set_error(LQCD_EINVAL, "the Schur operator needs a " + std::to_string(need) +
                                        "-byte half field, more than the " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                                        "-byte scratch of lqcd_apply_native_noalloc");
    if (!c->noalloc_scratch) return set_error(LQCD_ESTATE, "no scratch address for this context");
    tmp = c->noalloc_scratch;
  }
  if (!c->have_gauge || !c->have_clover) return set_error(LQCD_ESTATE, "set_gauge and set_clover must come first");
  return op_native(c, op, prec, in, out, tmp);
}

int lqcd_solve_batch(lqcd_ctx* const* ctxs, const int* nrhs, const double* const* b, double* const* x,
                     int nlattices, const lqcd_solve_params* prm, lqcd_solve_stats* stats);

}  // extern "C"
