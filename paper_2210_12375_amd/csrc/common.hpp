// Shared device-side definitions of the batchode HIP library.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

namespace bode {

enum : int32_t {
  kRunning = 0,
  kSuccess = 1,
  kMaxSteps = 2,
  kDtUnderflow = 3,
  kInvalid = 4,
};

enum : int32_t { kKindVdp = 0, kKindLinear = 1 };

// Step-size controller coefficients (PI family, integral when beta2 == 0).
struct Ctrl {
  double beta1, beta2, safety, fac_min, fac_max;
  int32_t max_steps;
  double beta3;
  int32_t fixed;  // fixed step: accept every attempt, keep h
};

// Per-instance solver state kept in the caller's workspace between calls
// (structure of arrays, index = instance).
template <typename R>
struct State {
  double* t;         // current time
  R* h;              // next step size to try
  // error history of the last two accepted steps (PI and PID terms): the
  // norms clamped below at 1e-4, or in the squared-norm FP32 controller of
  // the analytic kernels log2 of the clamped squared norms
  R* err_prev;
  R* err_prev2;
  int32_t* n_att;    // attempted steps
  int32_t* n_acc;    // accepted steps
  int32_t* n_rej;    // rejected steps
  int32_t* n_fe;     // right-hand-side evaluations
  int32_t* status;   // kRunning ...
  int32_t* cursor;   // next evaluation time to answer
  int32_t* prev_rej; // last attempt was rejected
  R* y;              // [B, D] current state
  R* k1;             // [B, D] f(t, y) (first stage, FSAL)
  // [B, D] FP32 analytic kernels: the rounding error of the last update
  // y <- y + h sum b_j k_j (compensated summation), carried into the next
  // update and the dense outputs; unused (may be null) elsewhere
  R* yc;
};

// Interpolant of each instance's last accepted step, kept on request so
// solver_eval can answer queries: y(theta) = y_prev + sum_m q_m theta^m.
template <typename R>
struct DenseKeep {
  double* t_prev;  // [B] start of the last accepted step
  R* h_last;       // [B] its size
  R* y_prev;       // [B, D]
  R* q;            // [4, B, D]
};

template <typename R>
__device__ __forceinline__ R rabs(R x) {
  return x < R(0) ? -x : x;
}

template <typename R>
__device__ __forceinline__ R rmax(R a, R b) {
  return a > b ? a : b;
}

template <typename R>
__device__ __forceinline__ R rmin(R a, R b) {
  return a < b ? a : b;
}

__device__ __forceinline__ double rpow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float rpow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double rsqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float rsqrt_(float x) { return sqrtf(x); }

// Controller and norm arithmetic.  FP64 (the validation mode) stays correctly
// rounded; the reduced-precision modes use the hardware reciprocal, square
// root, log2 and exp2 (about 1 ulp), which is far below the float rounding
// noise of an embedded error estimate.
__device__ __forceinline__ double ctl_div(double a, double b) { return a / b; }
__device__ __forceinline__ float ctl_div(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}
__device__ __forceinline__ double ctl_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float ctl_sqrt(float x) {
  return __builtin_amdgcn_sqrtf(x);
}
__device__ __forceinline__ double ctl_pow(double x, double y) {
  return pow(x, y);
}
__device__ __forceinline__ float ctl_pow(float x, float y) {
  return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x));
}

template <typename R>
__device__ __forceinline__ R quiet_nan();
template <>
__device__ __forceinline__ double quiet_nan<double>() {
  return __builtin_nan("");
}
template <>
__device__ __forceinline__ float quiet_nan<float>() {
  return __builtin_nanf("");
}

}  // namespace bode
