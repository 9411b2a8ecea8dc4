// Arguments of the analytic-field kernels (Van der Pol and linear instances).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace bode {

// Scalar state of a joint (coupled) solve: the batch's members share it.
struct JointState {
  double t, t_end, h, err_prev, err_prev2;
  int32_t n_att, n_acc, n_rej, status, cursor, prev_rej, ref, n_total, probe;
};

template <typename R>
struct AnalyticArgs {
  int32_t B, D, E;
  const R* y0;
  const double* t0;
  const double* t_end;
  const double* rtol;
  const double* atol;
  const double* t_eval;
  const double* h0;
  const int32_t* kind;
  const int32_t* dim;
  const R* mu;
  const R* A;
  R* y_eval;
  R* y_final;
  State<R> st;
  // Work queue: instances still running after initialisation, Van der Pol
  // ones from the front of `list`, linear ones from the back.
  // counts = {n_vdp, n_linear, head_vdp, head_linear}.
  int32_t* list;
  int32_t* counts;
  double* h_rec;  // [B, rec_cap] attempted step sizes (rejected < 0)
  double* e_rec;  // [B, rec_cap] their error norms
  int32_t rec_cap;
  DenseKeep<R> dk;
  int32_t keep_dense;
  Ctrl ctrl;
  int32_t budget;  // attempts per instance in one solve call
  // joint mode: shared scalar state, stages k_2..k_7 [6, B, D] and the
  // candidate solution [B, D] of the current attempt (null otherwise)
  JointState* js;
  R* jK;
  R* jY;
};

template <typename R>
hipError_t launch_analytic_init(const AnalyticArgs<R>& a, int method,
                                hipStream_t s);
template <typename R>
hipError_t launch_analytic_solve(const AnalyticArgs<R>& a, int method,
                                 int kind, int lanes, int block,
                                 hipStream_t s);
template <typename R>
hipError_t launch_dense_eval(const DenseKeep<R>& dk, const State<R>& st,
                             int B, int D, const double* t_query, R* y_out,
                             int32_t* qstatus, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s);
// Joint (coupled) mode: one workgroup solves the batch as one system.
template <typename R>
hipError_t launch_joint_init(const AnalyticArgs<R>& a, int method,
                             hipStream_t s);
template <typename R>
hipError_t launch_joint_solve(const AnalyticArgs<R>& a, int method,
                              hipStream_t s);

}  // namespace bode
