// Solver workspaces and the even-odd solve (solver.hip).
#pragma once

#include "blas.h"
#include "internal.h"

namespace lq {

// Vectors of one BiCGStab in precision prec (x in xprec), its device scalars,
// reduction partials and the captured graph of `graph_k` iterations.
struct InnerVecs {
  int prec = 0, xprec = 0;
  void *r = nullptr, *rhat = nullptr, *pv = nullptr, *v_ = nullptr, *s = nullptr, *t = nullptr, *y = nullptr,
       *x = nullptr;
  Scal* sc = nullptr;
  double* partials = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_k = 0, graph_block = 0, graph_remap = -1, graph_nt = -1, graph_split = -1;
  int init(lqcd_ctx* c, int prec, int xprec);
  void release();
};

// FP64 half fields of the outer loop, plus one InnerVecs per inner precision.
struct Workspace {
  void *b_e = nullptr, *b_o = nullptr, *bhat = nullptr, *x_e = nullptr, *x_o = nullptr, *r64 = nullptr,
       *v64 = nullptr, *y64 = nullptr;
  double* norms = nullptr;   // device: small results
  double* hnorms = nullptr;  // pinned host mirror (+ a Scal at offset 32 doubles)
  InnerVecs inner[3];
  int init(lqcd_ctx* c);
  void release();
};

int ensure_workspace(lqcd_ctx* c, int inner_prec);
// Solve with b in ws->b_e / b_o and the initial guess in ws->x_e; result in ws->x_e / x_o.
int solve_native(lqcd_ctx* c, const lqcd_solve_params& prm, lqcd_solve_stats& st);

}  // namespace lq
