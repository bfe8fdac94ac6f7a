/*
 * lqcd.h -- C ABI of the MI355X (gfx950) even-odd Wilson/clover operator and
 * its Krylov solvers.
 *
 * The library takes over the calculation of fermion propagators from a host
 * application, converting data to its own layout on the way in and back on the
 * way out (the paper, Sec. 1 and Sec. 2: machine-specific code plugged in as an
 * alternative to the generic code, with data conversion before and after).
 *
 * Operator (Sec. 2, Eq. (1); matrix elements are the textbook Wilson and
 * Sheikholeslami-Wohlert ones, which the paper names but does not print):
 *
 *   D psi(x) = A(x) psi(x) - kappa * sum_mu [ eta (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                           + eta (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *   A(x)     = 1 + kappa c_SW sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x)   (A = 1 for c_SW = 0)
 *   sigma_{mu nu} = [gamma_mu, gamma_nu]/(2i),  F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dag)/(8i),
 *   Q_{mu nu} = sum of the four plaquettes in the (mu, nu) plane that start and end at x.
 *
 * gamma matrices are Dirac-Pauli: gamma_j = [[0, -i s_j], [i s_j, 0]] (j = x, y, z),
 * gamma_t = diag(1, 1, -1, -1). eta = t_bc on a hop in t that crosses the
 * lattice boundary, 1 otherwise; all other directions are periodic.
 *
 * Even-odd blocks (Eq. (1)): with P_e, P_o the projectors on even
 * ((x+y+z+t) mod 2 = 0) and odd sites, D_pq = P_p D P_q. The solver works on
 * the Schur complement S = D_ee - D_eo D_oo^-1 D_oe; the paper's form is
 * D^(eo) = 1 - D_ee^-1 D_eo D_oo^-1 D_oe = D_ee^-1 S.
 *
 * Canonical layouts at this boundary (complex128 = two doubles, re then im):
 *   spinor  psi[t][z][y][x][spin 0..3][colour 0..2]            (12 complex per site)
 *   gauge   U[t][z][y][x][mu 0..3 = x,y,z,t][row 0..2][col 0..2] (9 complex per link)
 * Parity operators take and return full-lattice vectors; D_pq reads parity q of
 * its input and writes parity p of its output, and sets the other parity of the
 * output to zero, so D = D_ee + D_eo + D_oe + D_oo holds exactly.
 *
 * Conventions for every call:
 *   - Return value: LQCD_OK (0) or a negative lqcd_status. No exception crosses
 *     the ABI. lqcd_strerror() names a status; lqcd_last_error() gives detail.
 *   - Ownership: the caller owns every pointer it passes; the library copies what
 *     it keeps (gauge, clover) and keeps no caller pointer after a call returns.
 *   - on_device = 1: the pointer is device memory of the context's GPU (e.g. a
 *     torch tensor's data_ptr()); on_device = 0: host memory.
 *   - Streams: all GPU work is enqueued on the context's stream. Calls with host
 *     pointers, lqcd_solve* and lqcd_set_* return after that stream is
 *     synchronised; lqcd_apply_native and device-pointer lqcd_apply return
 *     without synchronising.
 *   - Threads: a context is used by one host thread at a time.
 */
#ifndef LQCD_H
#define LQCD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lqcd_ctx lqcd_ctx;

enum lqcd_status {
  LQCD_OK = 0,
  LQCD_EINVAL = -1,     /* bad argument: dims, null pointer, NaN/Inf input, unknown op */
  LQCD_ENOMEM = -2,     /* device allocation failed */
  LQCD_EHIP = -3,       /* a HIP runtime call failed */
  LQCD_ESTATE = -4,     /* call out of order (e.g. apply before set_gauge) */
  LQCD_ENOCONV = -5,    /* solver hit max_iter / max_outer; stats are filled */
  LQCD_EBREAKDOWN = -6, /* BiCGStab breakdown persisted after restarts */
  LQCD_ENOTSU3 = -7,    /* a link is not special unitary to 1e-12 */
  LQCD_ESINGULAR = -8   /* a clover block is singular */
};

enum lqcd_prec { LQCD_F64 = 0, LQCD_F32 = 1, LQCD_F16 = 2 };

enum lqcd_op {
  LQCD_D = 0,            /* full operator D */
  LQCD_DEE = 1,          /* D_ee = P_e A P_e */
  LQCD_DOO = 2,          /* D_oo = P_o A P_o */
  LQCD_DEO = 3,          /* D_eo = -kappa P_e H P_o */
  LQCD_DOE = 4,          /* D_oe = -kappa P_o H P_e */
  LQCD_DPREC_PAPER = 5,  /* Eq. (1): D^(eo) = 1 - D_ee^-1 D_eo D_oo^-1 D_oe on even sites */
  LQCD_DPREC_SCHUR = 6,  /* S = D_ee - D_eo D_oo^-1 D_oe on even sites */
  LQCD_DEE_INV = 7,      /* D_ee^-1 */
  LQCD_DOO_INV = 8,      /* D_oo^-1 */
  LQCD_HOP_EO = 9,       /* P_e H P_o (the bare hopping term, "Dslash", no -kappa) */
  LQCD_HOP_OE = 10       /* P_o H P_e */
};

/* Create a context for an Lx x Ly x Lz x Lt lattice (dims = {Lx, Ly, Lz, Lt},
 * every extent even and >= 2; up to 2^31 sites per parity). t_bc = -1
 * (antiperiodic in t) or +1 (periodic). hip_stream: a hipStream_t to enqueue
 * on, or NULL for a stream the context creates and owns. On success *out owns
 * all device state; release it with lqcd_destroy. EINVAL on bad dims or t_bc. */
int lqcd_create(const int dims[4], int t_bc, void* hip_stream, lqcd_ctx** out);

/* Free every device buffer of the context (NULL is accepted). */
int lqcd_destroy(lqcd_ctx* ctx);

/* Load the gauge field (canonical layout, 36 complex = 72 doubles per site). Every link is
 * checked to be SU(3) (max |U U^dag - 1| and |det U - 1| below 1e-12) and
 * finite; otherwise ENOTSU3 or EINVAL and the context has no gauge field
 * (later calls return ESTATE until a valid field is set). Stored as
 * rows 0 and 1 of each link (row 2 = conj(row0 x row1) is rebuilt in
 * registers) in FP64, FP32 and FP16. Invalidates the clover term: call
 * lqcd_set_clover next. */
int lqcd_set_gauge(lqcd_ctx* ctx, const double* U, int on_device);

/* Set kappa and c_SW and build the site matrices A from the stored gauge field
 * (c_SW = 0 gives the Wilson operator, A = 1, and nothing is built). Builds
 * A and A^-1 on both parities in FP64, FP32 and FP16 as two 6x6 Hermitian
 * blocks per site (A commutes with gamma5). ESTATE before set_gauge; ESINGULAR if a
 * block cannot be inverted; EINVAL for non-finite kappa or c_SW. */
int lqcd_set_clover(lqcd_ctx* ctx, double kappa, double csw);

/* out = op(in) on canonical full-lattice spinors (12 complex per site) in
 * precision prec (LQCD_F64/F32/F16: the precision of the stored fields and of
 * the arithmetic; FP16 uses FP16 storage with FP32 arithmetic). in and out must
 * not overlap. */
int lqcd_apply(lqcd_ctx* ctx, int op, int prec, const double* in, double* out, int on_device);

typedef struct {
  double tol;           /* stop when ||b - D x|| <= tol ||b|| (full FP64 D); default 1e-10 */
  int max_iter;         /* cap on inner BiCGStab iterations over the whole solve */
  int max_outer;        /* cap on outer (defect-correction) iterations */
  int inner_prec;       /* LQCD_F64: plain FP64 BiCGStab; F32/F16: mixed precision
                           (the staggered and even-odd domain-wall CG solves take
                           F64 or F32) */
  double inner_tol;     /* relative tolerance of each inner solve (mixed only); with
                           reliable_update, the drop of the iterated residual
                           between two reliable updates (0: 0.1) */
  int check_every;      /* iterations between host convergence checks (>= 1) */
  int use_graph;        /* 1: replay check_every iterations from a captured hipGraph */
  const double* x0;     /* optional initial guess (canonical, same residency as b) */
  int on_device;        /* 1: b, x and x0 are device pointers; 0: host pointers */
  int reliable_update;  /* mixed only: 1 = reliable updates (one low-precision Krylov
                           space, the FP64 true residual re-injected each time the
                           iterated one drops by inner_tol, 10x by default); 0 =
                           defect correction (restart
                           the inner solve from each FP64 residual) */
  int even_odd;         /* lqcd_solve only: 1 = even-odd preconditioned (Eq. (1));
                           0 = BiCGStab on the full operator D, FP64 only
                           (inner_prec must be LQCD_F64, else EINVAL) */
} lqcd_solve_params;

typedef struct {
  int outer_iters;      /* defect-correction passes (1 for plain FP64) */
  int inner_iters;      /* BiCGStab iterations, summed over passes */
  int restarts;         /* BiCGStab restarts (true-residual or breakdown) */
  double true_rel_resid;/* ||b - D x|| / ||b||, full operator, FP64, on return */
  double seconds_solve; /* wall time from entry to return */
  double seconds_setup; /* part of it spent on source preparation and reconstruction */
} lqcd_solve_stats;

/* Fill *p with the defaults (tol 1e-10, max_iter 100000, max_outer 100,
 * inner_prec LQCD_F64, inner_tol 1e-6 for F32 / 1e-2 for F16 when 0,
 * check_every 8, use_graph 1, x0 NULL, on_device 0, reliable_update 0,
 * even_odd 1). */
void lqcd_default_params(lqcd_solve_params* p);

/* Solve D x = b (canonical full-lattice vectors), the propagator solve the
 * paper benchmarks (Sec. 3: BiCGStab for the clover operator and its
 * mixed-precision variant), by even-odd preconditioning (Eq. (1)):
 * b_e' = b_e - D_eo D_oo^-1 b_o, S x_e = b_e' by BiCGStab (FP64, or FP32/FP16
 * iterations with FP64 reliable updates or an FP64 defect-correction loop), then
 * x_o = D_oo^-1 (b_o - D_oe x_e). With prm->even_odd = 0, FP64 BiCGStab on the
 * full operator D instead (stats: inner_iters = iterations, outer_iters =
 * passes restarted from the true residual). Returns after the stream is
 * synchronised. ENOCONV if the caps are hit (x holds the last iterate, stats
 * are filled). */
int lqcd_solve(lqcd_ctx* ctx, const double* b, double* x, const lqcd_solve_params* prm,
               lqcd_solve_stats* stats);

/* Batched solve (Sec. 3: many equations on one gauge configuration, e.g. the
 * 12 spin-colour sources of a propagator, solved together to share the
 * operator's data): for each lattice k < nlattices, nrhs[k] right-hand sides
 * b[k] (nrhs[k] canonical vectors back to back) on context ctxs[k]; solutions
 * to x[k], by the even-odd preconditioned (mixed-precision) BiCGStab of
 * lqcd_solve (even_odd = 0 is EINVAL here; with inner_tol 0 the FP16 inner
 * solves default to 5e-3 instead of 1e-2). All contexts must share one stream. Each RHS runs its own
 * BiCGStab (own alpha, beta, omega; not block Krylov) but every operator step
 * of every unconverged RHS of every lattice is one persistent kernel launch in
 * which a lane applies each link and clover block it loads to several RHS and
 * the waves of a workgroup share a site block's loads (launch shapes tuned per
 * batch, see lqcd_batch_autotune). Converged RHS are masked out. stats has one
 * entry per RHS, lattice-major. */
int lqcd_solve_batch(lqcd_ctx* const* ctxs, const int* nrhs, const double* const* b,
                     double* const* x, int nlattices, const lqcd_solve_params* prm,
                     lqcd_solve_stats* stats);

/* Launch shape of the batched hop for a batch (the same contexts and nrhs
 * as a later lqcd_solve_batch call) at inner precision prec, chosen by a
 * project-written autotuner (the counterpart of the paper's tiling sweep,
 * Sec. 3): shape = {right-hand sides per lane (1..4; 1..2 in FP64),
 * wavefronts per workgroup (1..8, one group of right-hand sides each),
 * workgroups per XCD, tile walk (0: linear in the site index, 1: every XCD
 * walks its range of blocks of each time slice, slice after slice; 2, 3: the
 * same with the range cut into 2 or 4 parts walked one after the other), 1 for
 * non-temporal loads of links and clover blocks}. A batch holds one shape
 * per kind of batched hop: the A_oo^-1 H_oe hop and the two XPAY hops of the
 * BiCGStab iteration (with <rhat, v>, and with <t, s>, <t, t>), whose extra
 * reads and sums hold more registers. With shape NULL or shape[0] <= 0 each
 * kind's shape comes from the tune cache (LQCD_TUNE_CACHE) or, without an
 * entry, from timing its candidates with HIP events on the batch's own fields
 * (the choices are then written to the cache); otherwise the given shape is
 * used as is for every kind. The batch keeps the shapes for the next
 * lqcd_solve_batch of the same contexts, nrhs and precision (which tunes by
 * itself when no shape was set). On return shape (if not NULL) holds the
 * shape of the A_oo^-1 H_oe hop and *us (if not NULL) its average duration in
 * microseconds over all right-hand sides of all lattices, timed with HIP
 * events on the contexts' stream over 20 launches. Allocates the batch's
 * fields; EINVAL for a bad shape or precision, otherwise as lqcd_solve_batch. */
int lqcd_batch_autotune(lqcd_ctx* const* ctxs, const int* nrhs, int nlattices, int prec, int shape[5], double* us);

/* out = S in for every right-hand side of a batch, through the batched hop
 * kernels of lqcd_solve_batch in precision prec (S = D_ee - D_eo D_oo^-1 D_oe
 * as LQCD_DPREC_SCHUR; Eq. (1)): in[k] and out[k] hold nrhs[k] canonical
 * full-lattice vectors of lattice k back to back, in device memory; the odd
 * sites of in are ignored and those of out set to zero. Uses the batch's launch
 * shape (tuned as in lqcd_solve_batch if none is set). For checking the batched
 * kernels against single-field applies and the oracle; returns after the
 * stream is synchronised. EINVAL / ESTATE as lqcd_solve_batch. */
int lqcd_batch_apply_schur(lqcd_ctx* const* ctxs, const int* nrhs, int nlattices, int prec,
                           const double* const* in, double* const* out);

/* Schwarz alternating procedure (SAP) preconditioner, the smoother of the
 * paper's multigrid solver (Sec. 3): the lattice is cut into blocks of
 * block[0] x block[1] x block[2] x block[3] sites (x, y, z, t), every extent
 * holding an even number of blocks, 64, 128, 192 or 256 sites per block;
 * blocks are coloured like a checkerboard. One application M eta runs
 * ncycles cycles from psi = 0; a cycle updates the colour-0 blocks, then the
 * colour-1 blocks, each by nmr minimal-residual iterations on the block
 * equation D_B delta = P_B (eta - D psi), D_B = D with the hops that enter or
 * leave the block removed, one MR coefficient per block. M works in FP32 on
 * the FP32 copies of the links and clover term (the full operator D, both
 * parities, not the even-odd Schur complement). */
typedef struct {
  int block[4];   /* block extents (x, y, z, t) */
  int ncycles;    /* SAP cycles per application (>= 1) */
  int nmr;        /* minimal-residual iterations per block solve (>= 1) */
} lqcd_sap_params;

/* psi = M eta, canonical full-lattice vectors (as lqcd_apply); on_device as
 * in lqcd_apply. EINVAL for a block shape that does not tile the lattice as
 * stated above; ESTATE before set_gauge / set_clover. */
int lqcd_apply_sap(lqcd_ctx* ctx, const lqcd_sap_params* sap, const double* eta, double* psi, int on_device);

/* Solve D x = b on the full lattice by flexible BiCGStab in FP64 with M as a
 * right preconditioner, until the true residual ||b - D x|| / ||b|| <= prm->tol.
 * From prm: tol, max_iter (outer iterations), max_outer (restarts), on_device,
 * x0. stats: outer_iters = flexible BiCGStab iterations, inner_iters =
 * applications of M, restarts, true_rel_resid, timings. Returns ENOCONV /
 * EBREAKDOWN as lqcd_solve does, with x the last iterate. */
int lqcd_solve_sap(lqcd_ctx* ctx, const double* b, double* x, const lqcd_solve_params* prm,
                   const lqcd_sap_params* sap, lqcd_solve_stats* stats);

/* Two-level aggregation multigrid (the paper's headline solver, Sec. 3, in
 * the DD-alpha-AMG style) for the full clover operator D on the gauge field
 * and clover term already set.
 *   aggregates: blocks of extents agg[] (each >= 2, an even number of them per
 *     direction, at most 256 sites each), coarse index a = ax + nax (ay +
 *     nay (az + naz at));
 *   chirality: gamma5 of the Dirac-Pauli basis mixes the upper (u) and lower
 *     (l) spin pairs; the chiral parts are c_+ = (u - l)/sqrt2 and
 *     c_- = (u + l)/sqrt2;
 *   P: one column per (a, chi, k), the chiral part chi of test vector k on a,
 *     the n columns of each (a, chi) orthonormalised in the order k = 0..n-1
 *     (Gram-Schmidt); coarse vectors are complex128 of mg_coarse_size entries,
 *     index (a * 2 + chi) * n + k;
 *   D_c = P^dag D P (a nearest-neighbour stencil on the aggregates), in FP32;
 *   setup: from nvec start vectors, setup_iters rounds of one SAP-smoothing
 *     step of D v = 0, v_k <- v_k - M_SAP D v_k, for every k, each followed by
 *     the orthonormalisation (0 rounds: the start vectors themselves);
 *   preconditioner: x = P D_c^-1 P^dag r with the coarse system solved by
 *     FP32 BiCGStab to a relative residual coarse_tol (or coarse_max_iter
 *     iterations), then x += M_SAP (r - D x); all in FP32.
 * The setup belongs to the context and is dropped by lqcd_set_gauge and
 * lqcd_set_clover. */
typedef struct {
  int agg[4];             /* aggregate extents (x, y, z, t) */
  int nvec;               /* test vectors per chirality (1 .. 24) */
  int setup_iters;        /* SAP smoothing rounds in the setup (0 .. 100) */
  lqcd_sap_params sap;    /* the smoother (setup and post-smoothing) */
  double coarse_tol;      /* relative residual of the coarse BiCGStab, in (0, 1) */
  int coarse_max_iter;    /* iteration cap of the coarse BiCGStab (>= 1) */
} lqcd_mg_params;

/* Set up the test vectors and the coarse operator from nvec canonical spinor
 * fields at start (back to back, host or device; random vectors in the usual
 * use). EINVAL for bad parameters or non-finite start vectors, ESTATE before
 * set_gauge / set_clover, ENOMEM. On failure no setup remains. */
int lqcd_mg_setup(lqcd_ctx* ctx, const lqcd_mg_params* mg, const double* start, int on_device);
/* Entries of a coarse vector; 0 without a setup. */
size_t lqcd_mg_coarse_size(lqcd_ctx* ctx);
/* coarse = P^dag fine, fine = P coarse, out = D_c in, x = the two-level
 * preconditioner applied to r (all in FP32 inside; canonical fine fields and
 * complex128 coarse vectors, host or device). ESTATE without a setup. */
int lqcd_mg_restrict(lqcd_ctx* ctx, const double* fine, double* coarse, int on_device);
int lqcd_mg_prolong(lqcd_ctx* ctx, const double* coarse, double* fine, int on_device);
int lqcd_mg_coarse_apply(lqcd_ctx* ctx, const double* in, double* out, int on_device);
int lqcd_mg_apply(lqcd_ctx* ctx, const double* r, double* x, int on_device);
/* Solve D x = b (canonical fields, host or device) by FP64 flexible BiCGStab
 * with the two-level preconditioner on the right, until the true residual
 * ||b - D x|| / ||b|| <= prm->tol. stats: outer_iters = flexible BiCGStab
 * iterations, inner_iters = preconditioner applications. ESTATE without a
 * setup; ENOCONV / EBREAKDOWN as lqcd_solve. */
int lqcd_solve_mg(lqcd_ctx* ctx, const double* b, double* x, const lqcd_solve_params* prm,
                  lqcd_solve_stats* stats);

/* Staggered fermions (one of the operator kinds the paper lists, Sec. 2), on
 * the gauge field already set: D = m + H with
 *   (H psi)(x) = 1/2 sum_mu eta_mu(x) [U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu)],
 * eta_x = 1, eta_y = (-1)^x, eta_z = (-1)^(x+y), eta_t = (-1)^(x+y+z), the
 * context's time boundary factor on hops across the t boundary. Vectors are
 * canonical full-lattice colour vectors: complex128 [Lt][Lz][Ly][Lx][3]
 * (48 bytes per site), host or device as on_device says. */
typedef enum {
  LQCD_STAG_D = 0,      /* out = D in on the whole lattice */
  LQCD_STAG_SCHUR = 1   /* out_e = (m^2 - H_eo H_oe) in_e, out_o = 0 (even-odd normal operator) */
} lqcd_stag_op;

/* prec LQCD_F64 or LQCD_F32 (FP32 links and vectors, FP32 arithmetic).
 * EINVAL for another precision, op or a non-finite mass; ESTATE before
 * set_gauge. */
int lqcd_stag_apply(lqcd_ctx* ctx, int op, int prec, double mass, const double* in, double* out, int on_device);

/* Solve D x = b (mass > 0) by CG on the even-odd normal system
 * (m^2 + H_eo H_eo^dag on the even sites, Hermitian positive definite), x_o
 * rebuilt as (b_o - H_oe x_e) / m, until the true residual
 * ||b - D x|| / ||b|| <= prm->tol. From prm: tol, max_iter (CG iterations),
 * max_outer (CG restarts from the true residual), on_device, and inner_prec:
 * LQCD_F64, CG in FP64; LQCD_F32, defect correction in the manner of the
 * paper's mixed-precision solver (Sec. 3): each pass solves for the FP64
 * residual by FP32 CG until its iterated residual has dropped by
 * prm->inner_tol (1e-6 when 0) and adds the correction in FP64; LQCD_F16:
 * EINVAL. stats: inner_iters = CG iterations, outer_iters = passes,
 * true_rel_resid, timings. */
int lqcd_stag_solve(lqcd_ctx* ctx, double mass, const double* b, double* x, const lqcd_solve_params* prm,
                    lqcd_solve_stats* stats);

/* Domain-wall fermions, Moebius form (the operator kind the paper lists and
 * benchmarks, Sec. 2-3), on the gauge field already set:
 *   D = D_W (b5 + c5 S) + (1 - S),   D_W = (4 - M5) - 1/2 H on every slice,
 *   (S psi)_s = P_- psi_{s+1} + P_+ psi_{s-1},
 * H the Wilson hopping term (the context's boundary factor in t),
 * P_+- = (1 +- gamma5)/2, s = 0..Ls-1, walls psi_{Ls} -> -mf psi_0 and
 * psi_{-1} -> -mf psi_{Ls-1}. b5 = 1, c5 = 0 is the Shamir operator
 * (5 - M5) psi_s - 1/2 H psi_s - (S psi)_s. Vectors are canonical 5-d spinor
 * fields complex128 [Ls][Lt][Lz][Ly][Lx][4][3] (s slowest), host or device. */
typedef struct {
  int Ls;        /* 1 .. 256 */
  double M5;     /* domain-wall height */
  double mf;     /* quark mass at the walls */
  double b5, c5; /* Moebius coefficients (Shamir: 1, 0) */
} lqcd_dwf_params;

/* out = D in (dag = 0) or D^dagger in (dag = 1), prec LQCD_F64 or LQCD_F32.
 * EINVAL for Ls outside 1..256, non-finite M5 / mf / b5 / c5 or another precision;
 * ESTATE before set_gauge. */
int lqcd_dwf_apply(lqcd_ctx* ctx, const lqcd_dwf_params* dwf, int dag, int prec, const double* in, double* out,
                   int on_device);

/* Solve D x = b by FP64 CG on the normal equations D^dag D x = D^dag b (D is
 * not positive definite: its Wilson kernel has mass -M5) until the true
 * residual ||b - D x|| / ||b|| <= prm->tol. From prm: tol, max_iter (CG
 * iterations), max_outer (passes restarted from the true residual),
 * on_device. stats: inner_iters = CG iterations, outer_iters = passes. */
int lqcd_dwf_solve(lqcd_ctx* ctx, const lqcd_dwf_params* dwf, const double* b, double* x,
                   const lqcd_solve_params* prm, lqcd_solve_stats* stats);

/* Even-odd form over the 4-d parity of the sites (the paper's even-odd
 * decomposition, Sec. 2, Eq. (1)): D = M5op + Dhop with the site-local
 * M5op = (4 - M5)(b5 + c5 S) + 1 - S and Dhop = -1/2 H (b5 + c5 S).
 * out = S_ee in (dag 0) or S_ee^dag in (dag 1) with
 * S_ee = M5op - Dhop_eo M5op^-1 Dhop_oe on the even sites of canonical 5-d
 * fields (host or device); the odd sites of in are ignored and those of out
 * are set to zero. ESINGULAR if M5op is singular; otherwise as lqcd_dwf_apply. */
int lqcd_dwf_apply_schur(lqcd_ctx* ctx, const lqcd_dwf_params* dwf, int dag, int prec, const double* in, double* out,
                         int on_device);
/* Solve D x = b through S_ee x_e = b_e - Dhop_eo M5op^-1 b_o, solved by CG
 * on its normal equations, and x_o = M5op^-1 (b_o - Dhop_oe x_e), restarted
 * from the true residual until ||b - D x|| / ||b|| <= prm->tol. Parameters
 * and stats as lqcd_dwf_solve, and prm->inner_prec: LQCD_F64, CG in FP64;
 * LQCD_F32, defect correction in the manner of the paper's mixed-precision
 * solver (Sec. 3): each pass solves the normal equations of the FP64 residual
 * by FP32 CG until its iterated residual has dropped by prm->inner_tol (1e-6
 * when 0) and adds the correction to x in FP64; LQCD_F16: EINVAL. */
int lqcd_dwf_solve_eo(lqcd_ctx* ctx, const lqcd_dwf_params* dwf, const double* b, double* x,
                      const lqcd_solve_params* prm, lqcd_solve_stats* stats);

/* Native domain-wall fields (benchmarks), on the device: the fifth coordinate
 * is the fastest index of a site (5-d index i Ls + s, i the 4-d checkerboard
 * index of the library's spinor layout), two parity halves in the
 * site-blocked layout, the even half first. 0 for a bad precision or Ls. */
size_t lqcd_dwf_field_bytes(lqcd_ctx* ctx, int prec, int Ls);
/* canonical 5-d device field -> native 5-d field */
int lqcd_dwf_import(lqcd_ctx* ctx, int prec, int Ls, const double* canon, void* native);
/* native 5-d field -> canonical 5-d device field */
int lqcd_dwf_export(lqcd_ctx* ctx, int prec, int Ls, const void* native, double* canon);
/* out = D in (dag 0) or D^dag in (dag 1) on native 5-d fields, enqueued
 * without synchronising (one kernel; two for D with c5 != 0). tmp is a
 * caller-owned native 5-d scratch field, needed by D with c5 != 0 only (NULL
 * allowed otherwise). in, out and tmp must be different fields (EINVAL
 * otherwise). Padding sites of out are not written. */
int lqcd_dwf_apply_native(lqcd_ctx* ctx, const lqcd_dwf_params* dwf, int dag, int prec, const void* in, void* out,
                          void* tmp);

/* Native staggered fields (benchmarks): half-lattice colour-vector fields of
 * one parity in the library's site-blocked layout on the device. */
size_t lqcd_stag_field_bytes(lqcd_ctx* ctx, int prec);
/* canonical full-lattice device colour vector -> native half field of a parity */
int lqcd_stag_import(lqcd_ctx* ctx, int prec, int parity, const double* canon, void* native);
/* native half field of a parity -> its sites of a canonical device colour
 * vector (the other parity's sites are left untouched) */
int lqcd_stag_export(lqcd_ctx* ctx, int prec, int parity, const void* native, double* canon);
/* out = H in (the staggered hopping term, from parity 1 - out_parity to
 * out_parity) on native device fields, enqueued without synchronising. */
int lqcd_stag_hop_native(lqcd_ctx* ctx, int prec, int out_parity, const void* in, void* out);

/* Native fast path (benchmarks, solvers in the caller): half-lattice fields of
 * one parity in the library's internal layout on the device (site-blocked:
 * sites in blocks of 64, the count per parity rounded up to whole blocks). */
size_t lqcd_field_bytes(lqcd_ctx* ctx, int prec);
/* canonical full-lattice device vector -> native half field of the given parity */
int lqcd_import(lqcd_ctx* ctx, int prec, int parity, const double* canon, void* native);
/* native half field of the given parity -> parity sites of a canonical device
 * vector (the other parity's sites are left untouched) */
int lqcd_export(lqcd_ctx* ctx, int prec, int parity, const void* native, double* canon);
/* out = op(in) on native half fields, enqueued without synchronising. op is one
 * of LQCD_DEO, LQCD_DOE, LQCD_HOP_EO, LQCD_HOP_OE (one hop), LQCD_DEE, LQCD_DOO,
 * LQCD_DEE_INV, LQCD_DOO_INV (site terms) or LQCD_DPREC_SCHUR (even -> even). */
int lqcd_apply_native(lqcd_ctx* ctx, int op, int prec, const void* in, void* out);

/* lqcd_apply_native without allocating: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Same operators, arguments and results as
 * lqcd_apply_native; the Schur operator's intermediate odd half field lives in
 * a file-scope device array of the library (NOALLOC limit: 128 MiB per GPU,
 * e.g. FP32 up to 32^3 x 64, FP64 up to 32^3 x 32), held on each GPU from the
 * first context created on it to the end of the process. No hipMalloc, hipFree
 * or allocating library call is made. EINVAL when the operator's half field
 * exceeds the limit (with the sizes in lqcd_last_error); ESTATE before
 * set_gauge / set_clover. All calls on one GPU share that array, so calls
 * that overlap in time on one GPU (other streams or threads) race; calls
 * ordered on one stream are safe. Enqueued without synchronising. */
int lqcd_apply_native_noalloc(lqcd_ctx* ctx, int op, int prec, const void* in, void* out);

/* Autotune the launch shape of the hop for (op, prec) on this lattice: times
 * each candidate workgroup size and block-to-XCD mapping on native scratch
 * fields and keeps the fastest in the context. If path is not NULL the choice
 * is merged into that JSON cache file and read back from it by later contexts
 * of the same lattice and precision. */
int lqcd_autotune(lqcd_ctx* ctx, int prec, const char* path);

/* Fix the launch shape of the hop kernels for one precision (the knobs the
 * autotuner searches). Site-parallel kernels: block = workgroup size (64, 128,
 * 192 or 256 threads), split = lanes per output site (1; 2 with the forward
 * hops in one lane and the backward hops in the other; 4 with one lattice
 * direction per lane), xcd_map = 0 for blocks in site order, 1 to give each of
 * the chip's 8 XCDs one contiguous range of sites, 2 to give each XCD one slab
 * of Lz/8 z-planes walked z before t (needs Lz divisible by 8).
 * split = 0 selects the plane march: one workgroup per tile of whole x rows of
 * an xy plane, marching in z with each plane's input staged in LDS; block =
 * lanes = (Lx/2) x rows (rows dividing Ly, at most 512 lanes), xcd_map = z
 * planes per workgroup (dividing Lz).
 * nt = 1 to load the links non-temporally. EINVAL for any shape that is not
 * valid on this lattice. The results do not depend on the shape beyond the
 * rounding of the order in which the hops of a site and the fused reductions
 * are added. */
int lqcd_set_hop_shape(lqcd_ctx* ctx, int prec, int block, int split, int xcd_map, int nt);
/* The launch shape in use for one precision (as lqcd_set_hop_shape takes it);
 * any output pointer may be NULL. */
int lqcd_get_hop_shape(lqcd_ctx* ctx, int prec, int* block, int* split, int* xcd_map, int* nt);

/* Streaming bandwidth of the context's GPU, the practical ceiling the
 * roofline figures are read against (measurement support, not a step of the
 * method): kind 0 streams `bytes` of device memory once through a read-only
 * kernel (a sum of 16-byte words, 2048 workgroups of 256 lanes walking the
 * buffer in grid-sized strides), kind 1 copies them to a second buffer. The
 * library allocates the buffers (zeroed) and frees them before returning;
 * *gbs receives the best of reps launches in GB/s of bytes moved (read plus
 * written), timed with HIP events on the context's stream. bytes is rounded
 * down to a multiple of 16 and must be at least 1 MiB; EINVAL for a bad
 * kind, size or reps, ENOMEM if the buffers cannot be allocated. */
int lqcd_bandwidth_probe(lqcd_ctx* ctx, int kind, size_t bytes, int reps, double* gbs);

/* Name of a status code; detail of the last error on this thread. */
const char* lqcd_strerror(int status);
const char* lqcd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LQCD_H */
