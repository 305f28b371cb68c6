// Second-order (nodal, 3D) solver runtime interface, used by the C ABI layer.
#pragma once

#include "cmcg_internal.h"

namespace cmcg {

struct F2Params {
  int n[3];            // cells per axis; nodes are n+1 per axis
  double h, dt, omega;
  int N;               // leapfrog steps per period
  int prec;            // CMCG_FP64 or CMCG_FP32_MIXED
  int kblock;          // steps per launch (temporal blocking)
  int abs_face[6];     // 1 if -x,+x,-y,+y,-z,+z is absorbing
  double tol;
  int max_iter;
  double riesz_tol;    // 0 -> default
  int riesz_max_iter;  // 0 -> default
};

struct F2Solver;

cmcg_status f2_create(F2Solver **out, const F2Params &p, const cmcg_problem *P, hipStream_t s);
void f2_destroy(F2Solver *S);
size_t f2_device_bytes(const F2Solver *S);
cmcg_status f2_begin(F2Solver *S);
cmcg_status f2_iterate(F2Solver *S, int iters, int *converged);
cmcg_status f2_finish(F2Solver *S, double *u_re, double *u_im);
cmcg_status f2_solve(F2Solver *S, double *u_re, double *u_im);
cmcg_status f2_apply(F2Solver *S, int op, const double *in, double *out);
cmcg_status f2_filter(F2Solver *S, const double *z, double *u_re, double *u_im);
cmcg_status f2_get_state(F2Solver *S, int which, double *out);
void f2_report(const F2Solver *S, cmcg_report *rep);

}  // namespace cmcg
