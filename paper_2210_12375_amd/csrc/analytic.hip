// Persistent per-lane solver for analytic right-hand sides.
//
// Paper section 3: every instance of the batch keeps its own time, step size,
// error estimate, controller state and accept/reject decision; section 4.1
// (Eq. eq:vdp) shows why: Van der Pol oscillators of different stiffness
// need very different step sequences.  Here one lane owns one instance at a
// time and keeps its whole state (y, the seven stages, t, h, controller state,
// counters, evaluation cursor) in registers for as long as the instance runs.
// There is no per-step launch, no host round trip and no "overhanging"
// evaluation of finished instances (appendix B): a lane whose instance ends
// takes the next one from a device-side queue (work stealing over instances),
// so uneven step counts do not idle the batch.
//
// The dynamics are cheap (section 4.2 / appendix A: for Van der Pol the loop,
// not the model, is the cost), so the kernel is bound by vector-ALU latency:
// the critical path is the longest instance's steps times the latency of one
// step.  Van der Pol and linear instances run in separate kernels so each gets
// the register allocation its own state needs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "analytic.hpp"
#include "common.hpp"
#include "tableau.hpp"

namespace bode {

// ---- right-hand sides ------------------------------------------------------

template <typename R>
struct VdpField {
  static constexpr int N = 2;
  R mu;
  __device__ __forceinline__ void load(const AnalyticArgs<R>& a, int i, int) {
    mu = a.mu[i];
  }
  // x' = v, v' = mu (1 - x^2) v - x
  __device__ __forceinline__ void operator()(const R* y, R* out) const {
    const R x = y[0], v = y[1];
    out[0] = v;
    out[1] = mu * (R(1) - x * x) * v - x;
  }
};

template <typename R>
struct LinearField {
  static constexpr int N = 8;
  R A[8][8];
  __device__ __forceinline__ void load(const AnalyticArgs<R>& a, int i, int dim) {
    const R* Ai = a.A + (long)i * a.D * a.D;
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int c = 0; c < 8; ++c)
        A[r][c] = (r < dim && c < dim) ? Ai[(long)r * a.D + c] : R(0);
  }
  __device__ __forceinline__ void operator()(const R* y, R* out) const {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      R acc = R(0);
#pragma unroll
      for (int c = 0; c < 8; ++c) acc += A[r][c] * y[c];
      out[r] = acc;
    }
  }
};

// Stage j takes part in the interpolant (Dormand-Prince's stage 2 does not).
template <class M>
__host__ __device__ constexpr bool dense_uses(int j) {
  return M::P[j][0] != 0.0 || M::P[j][1] != 0.0 || M::P[j][2] != 0.0 ||
         M::P[j][3] != 0.0;
}

// ---- one lane's instance -----------------------------------------------------

// Compensated summation (FP32 only): the FP32 kernels carry the rounding
// error of every update y <- y + h sum_j b_j k_j in yc and add it to the next
// update (Kahan's compensation, with the exact error of the sum taken by
// Knuth's branch-free TwoSum), so a long solve does not accumulate one
// float rounding of y per step; the stage inputs and the error estimate
// keep plain float arithmetic.
template <typename R>
constexpr bool kCompensated = std::is_same<R, float>::value;

// TW: evaluation times held in registers.  tw[0] is the instance's next
// evaluation time; each emission shifts the window and requests the time TW
// places ahead, so up to TW - 1 of those loads are in flight.  Two (the
// default) covers an emission per step; solves with many evaluation times
// per step (the paper's loop-time workload: about four) take eight.
template <typename R, int N, int TW = 2>
struct Lane {
  R y[N];
  R yc[N];  // compensation of y (FP32), zero in FP64
  R k[7][N];
  double t, te;
  double tw[TW];
  R h, err_prev, err_prev2, rtol, atol;
  int32_t n_att, n_acc, n_rej, n_fe, status, cursor, prev_rej, dim, inst;
};

template <typename R, int N>
__device__ __forceinline__ void write_row(R* row, int D, const R* v, int dim) {
#pragma unroll
  for (int q = 0; q < N; ++q)
    if (q < D) row[q] = q < dim ? v[q] : R(0);
  for (int q = N; q < D; ++q) row[q] = R(0);
}

// Columns [0, N) only: the padding columns [N, D) of the evaluation rows
// are written once, at initialisation, so an emission stores only what
// the field computes.
template <typename R, int N>
__device__ __forceinline__ void write_row_n(R* row, int D, const R* v,
                                            int dim) {
#pragma unroll
  for (int q = 0; q < N; ++q)
    if (q < D) row[q] = q < dim ? v[q] : R(0);
}

template <typename R, int N>
__device__ __forceinline__ void fill_nan_row(R* row, int D, int dim) {
  for (int q = 0; q < D; ++q) row[q] = q < dim ? quiet_nan<R>() : R(0);
}

template <typename R, int N, int TW>
__device__ __forceinline__ void load_lane(const AnalyticArgs<R>& a, int i,
                                          Lane<R, N, TW>& L) {
  const State<R>& s = a.st;
  L.inst = i;
  L.dim = a.dim[i];
  L.t = s.t[i];
  L.te = a.t_end[i];
  L.h = s.h[i];
  L.err_prev = s.err_prev[i];
  L.err_prev2 = s.err_prev2[i];
  L.rtol = R(a.rtol[i]);
  L.atol = R(a.atol[i]);
  L.n_att = s.n_att[i];
  L.n_acc = s.n_acc[i];
  L.n_rej = s.n_rej[i];
  L.n_fe = s.n_fe[i];
  L.status = s.status[i];
  L.cursor = s.cursor[i];
  L.prev_rej = s.prev_rej[i];
#pragma unroll
  for (int w = 0; w < TW; ++w)
    L.tw[w] = L.cursor + w < a.E ? a.t_eval[(long)i * a.E + L.cursor + w]
                                 : INFINITY;
  const R* yr = s.y + (long)i * a.D;
  const R* kr = s.k1 + (long)i * a.D;
  const R* cr = s.yc + (long)i * a.D;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    L.y[q] = q < L.dim ? yr[q] : R(0);
    L.k[0][q] = q < L.dim ? kr[q] : R(0);
    L.yc[q] = (kCompensated<R> && q < L.dim) ? cr[q] : R(0);
  }
}

template <typename R, int N, int TW>
__device__ __forceinline__ void store_lane(const AnalyticArgs<R>& a,
                                           const Lane<R, N, TW>& L) {
  const State<R>& s = a.st;
  const int i = L.inst;
  s.t[i] = L.t;
  s.h[i] = L.h;
  s.err_prev[i] = L.err_prev;
  s.err_prev2[i] = L.err_prev2;
  s.n_att[i] = L.n_att;
  s.n_acc[i] = L.n_acc;
  s.n_rej[i] = L.n_rej;
  s.n_fe[i] = L.n_fe;
  s.status[i] = L.status;
  s.cursor[i] = L.cursor;
  s.prev_rej[i] = L.prev_rej;
  write_row<R, N>(s.y + (long)i * a.D, a.D, L.y, L.dim);
  write_row<R, N>(s.k1 + (long)i * a.D, a.D, L.k[0], L.dim);
  if (kCompensated<R>) write_row<R, N>(s.yc + (long)i * a.D, a.D, L.yc, L.dim);
}

// Writes the final state, and NaN for evaluation times never reached.
template <typename R, int N, int TW>
__device__ __forceinline__ void finish_lane(const AnalyticArgs<R>& a,
                                            const Lane<R, N, TW>& L) {
  store_lane(a, L);
  write_row<R, N>(a.y_final + (long)L.inst * a.D, a.D, L.y, L.dim);
  if (L.status != kSuccess)
    for (int e = L.cursor; e < a.E; ++e)
      fill_nan_row<R, N>(a.y_eval + ((long)L.inst * a.E + e) * a.D, a.D,
                         L.dim);
}

// One attempted step of one instance (accept or reject), in the order of the
// reference algorithm: stages, error norm, controller, dense output, commit.
// REC: write the attempt record; KEEP: keep the interpolant for solver_eval.
// The controller is branch-free (selects); only the rare paths (dense output,
// the step limit) branch.
template <typename R, class M, class F, bool REC, bool KEEP, int TW>
__device__ __forceinline__ void attempt(const AnalyticArgs<R>& a,
                                        Lane<R, F::N, TW>& L, const F& f) {
  constexpr int N = F::N;
  if (__builtin_expect(L.n_att >= a.ctrl.max_steps, 0)) {
    L.status = kMaxSteps;
    return;
  }
  const bool last = L.t + double(L.h) >= L.te;
  const R hs = last ? R(L.te - L.t) : L.h;

  // Stages 2..7: Y_s = y + h sum_{j<s} a_sj k_j, k_s = f(t + c_s h, Y_s).
  // (The fields here are autonomous, so the stage time is not formed.)
  // The last stage input is the new solution (SSAL); in FP32 it is the
  // compensated sum of y and the update plus the carried error, whose new
  // rounding error goes to Yc.
  R Y[N], Yc[N];
#pragma unroll
  for (int s = 1; s < 7; ++s) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R acc = R(0);
#pragma unroll
      for (int j = 0; j < s; ++j)
        if (M::A[s][j] != 0.0) acc += R(M::A[s][j]) * L.k[j][q];
      if (kCompensated<R> && s == 6) {
        const R inc = hs * acc + L.yc[q];
        const R sum = L.y[q] + inc;
        const R bv = sum - L.y[q];
        const R av = sum - bv;
        Yc[q] = (L.y[q] - av) + (inc - bv);
        Y[q] = sum;
      } else {
        Y[q] = L.y[q] + hs * acc;
      }
    }
    f(Y, L.k[s]);
  }
  L.n_fe += 6;
  L.n_att += 1;

  // Weighted RMS norm of the embedded error estimate over the true dimension.
  R acc = R(0);
#pragma unroll
  for (int q = 0; q < N; ++q) {
    R eq = R(0);
#pragma unroll
    for (int j = 0; j < 7; ++j)
      if (M::E[j] != 0.0) eq += R(M::E[j]) * L.k[j][q];
    eq *= hs;
    const R sc = L.atol + L.rtol * rmax(rabs(L.y[q]), rabs(Y[q]));
    const R r = ctl_div(eq, sc);
    if (N == 2 || q < L.dim) acc += r * r;
  }
  // err^2 (mean of the squares); FP64 takes the root as written, FP32 works
  // with the square: err < 1 iff err^2 < 1, and both powers of the
  // controller come from one log2(err^2)
  const R err2 = N == 2 ? acc * R(0.5) : ctl_div(acc, R(L.dim));
  constexpr bool kSq = std::is_same<R, float>::value;
  const R err = kSq ? err2 : ctl_sqrt(err2);
  const bool accept = a.ctrl.fixed || err < R(1);
  if (REC && L.n_att <= a.rec_cap) {
    const long o = (long)L.inst * a.rec_cap + L.n_att - 1;
    a.h_rec[o] = accept ? double(hs) : -double(hs);
    a.e_rec[o] = kSq ? sqrt(double(err)) : double(err);  // FP32: err holds err^2
  }

  // Controller: on acceptance
  // clamp(safety err^-beta1 err_prev^beta2 err_prev2^beta3), capped at 1
  // after a rejection; on rejection max(fac_min, safety err^-1/5); err = 0
  // gives fac_max, a non-finite err fac_min.  The error history holds the
  // clamped norms of the two previous accepted steps (FP64) or log2 of their
  // clamped squares (FP32), 1 / 0 initially.
  const Ctrl& c = a.ctrl;
  R fac, lg = R(0);
  if constexpr (kSq) {  // one exp2 for the whole factor
    lg = __builtin_amdgcn_logf(err2);  // log2
    const R ex = accept ? R(-0.5 * c.beta1) * lg + R(0.5 * c.beta2) * L.err_prev +
                              R(0.5 * c.beta3) * L.err_prev2
                        : R(-0.1) * lg;
    fac = R(c.safety) * __builtin_amdgcn_exp2f(ex);
  } else {
    fac = R(c.safety) * ctl_pow(err, accept ? R(-c.beta1) : R(-0.2));
    if (accept) {
      if (c.beta2 != 0.0) fac = fac * ctl_pow(L.err_prev, R(c.beta2));
      if (c.beta3 != 0.0) fac = fac * ctl_pow(L.err_prev2, R(c.beta3));
    }
  }
  fac = (accept && err == R(0)) ? R(c.fac_max) : fac;
  fac = rmax(R(c.fac_min), accept ? rmin(R(c.fac_max), fac) : fac);
  fac = (accept && L.prev_rej) ? rmin(R(1), fac) : fac;
  fac = __builtin_isfinite(err) ? fac : R(c.fac_min);
  fac = c.fixed ? R(1) : fac;  // fixed step: h stays

  if (accept) {
    const double tnew = last ? L.te : L.t + double(hs);
    // Dense output at this instance's own evaluation times in (t, t_new]
    // (Horner in theta, then the stage combination).
    while (__builtin_expect(L.tw[0] <= tnew, 0)) {
      // theta = (t_e - t_n) / h: the difference in double, the quotient in
      // the state's precision
      const R th = ctl_div(R(L.tw[0] - L.t), hs);
      R w[7];
#pragma unroll
      for (int j = 0; j < 7; ++j)
        w[j] = th * (R(M::P[j][0]) +
                     th * (R(M::P[j][1]) +
                           th * (R(M::P[j][2]) + th * R(M::P[j][3]))));
      R out[N];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        R s2 = R(0);
#pragma unroll
        for (int j = 0; j < 7; ++j)
          if (dense_uses<M>(j)) s2 += w[j] * L.k[j][q];
        out[q] = L.y[q] + (kCompensated<R> ? hs * s2 + L.yc[q] : hs * s2);
      }
      write_row_n<R, N>(a.y_eval + ((long)L.inst * a.E + L.cursor) * a.D,
                        a.D, out, L.dim);
      L.cursor += 1;
#pragma unroll
      for (int w = 0; w + 1 < TW; ++w) L.tw[w] = L.tw[w + 1];
      L.tw[TW - 1] = L.cursor + TW - 1 < a.E
                         ? a.t_eval[(long)L.inst * a.E + L.cursor + TW - 1]
                         : INFINITY;
    }
    if (KEEP) {
      const int i = L.inst;
      a.dk.t_prev[i] = L.t;
      a.dk.h_last[i] = hs;
      write_row<R, N>(a.dk.y_prev + (long)i * a.D, a.D, L.y, L.dim);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        R qm[N];
#pragma unroll
        for (int q = 0; q < N; ++q) {
          R s2 = R(0);
#pragma unroll
          for (int j = 0; j < 7; ++j)
            if (M::P[j][m] != 0.0) s2 += R(M::P[j][m]) * L.k[j][q];
          qm[q] = hs * s2;
        }
        write_row<R, N>(a.dk.q + ((long)m * a.B + i) * a.D, a.D, qm, L.dim);
      }
    }
    L.t = tnew;
    if (last) L.status = kSuccess;
    L.err_prev2 = L.err_prev;
    if constexpr (kSq)  // log2 max(err, 1e-4)^2 = max(lg, log2 1e-8)
      L.err_prev = rmax(lg, R(-26.575424759098897));
    else
      L.err_prev = rmax(err, R(1e-4));
    L.n_acc += 1;
  }
  L.n_rej += accept ? 0 : 1;
  L.prev_rej = accept ? 0 : 1;
  if (accept) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      L.y[q] = Y[q];
      if (kCompensated<R>) L.yc[q] = Yc[q];
      L.k[0][q] = L.k[6][q];  // FSAL
    }
  }
  L.h = hs * fac;
  if (L.status == kRunning && !(double(L.h) > 16.0 * DBL_EPSILON * fabs(L.t)))
    L.status = kDtUnderflow;
}

template <typename R>
__device__ __forceinline__ int fetch(const AnalyticArgs<R>& a, int kind) {
  const int p = atomicAdd(&a.counts[2 + kind], 1);
  const int n = __atomic_load_n(&a.counts[kind], __ATOMIC_RELAXED);
  if (p >= n) return -1;
  return kind == kKindVdp ? a.list[p] : a.list[a.B - 1 - p];
}

constexpr int kLongRun = 256;

template <typename R, class M, class F, bool REC, bool KEEP, int TW = 2>
__global__ __launch_bounds__(256) void solve_kernel(AnalyticArgs<R> a,
                                                    int kind) {
  Lane<R, F::N, TW> L;
  F f;
  int inst = fetch(a, kind);
  while (inst >= 0) {
    if (a.st.status[inst] == kRunning) {
      load_lane(a, inst, L);
      f.load(a, inst, L.dim);
      // Drain the lane's loads here (vmcnt 0; expcnt, lgkmcnt untouched):
      // otherwise the step loop cannot tell them from the evaluation-time
      // prefetch still in flight and waits for everything on every step.
      __builtin_amdgcn_s_waitcnt(0x0F70);
      int used = 0;
      while (L.status == kRunning && used < a.budget) {
        attempt<R, M, F, REC, KEEP, TW>(a, L, f);
        ++used;
        // An instance still stepping after many attempts is on the batch's
        // critical path (the solve ends with its last step): its wavefront
        // issues ahead of the short-lived ones sharing the SIMD.
        if (used == kLongRun) __builtin_amdgcn_s_setprio(3);
      }
      if (L.status == kRunning)
        store_lane(a, L);
      else
        finish_lane(a, L);
    }
    inst = fetch(a, kind);
  }
}

// ---- initialisation ----------------------------------------------------------

template <typename R>
__device__ __forceinline__ bool instance_ok(const AnalyticArgs<R>& a, int i) {
  const int kind = a.kind[i], dim = a.dim[i];
  if (kind == kKindVdp) {
    if (dim != 2 || a.D < 2 || a.mu == nullptr) return false;
    if (!__builtin_isfinite(double(a.mu[i]))) return false;
  } else if (kind == kKindLinear) {
    if (dim < 1 || dim > 8 || dim > a.D || a.A == nullptr) return false;
  } else {
    return false;
  }
  const double t0 = a.t0[i], te = a.t_end[i];
  if (!__builtin_isfinite(t0) || !__builtin_isfinite(te) || te < t0)
    return false;
  const double rt = a.rtol[i], at = a.atol[i];
  if (!(rt >= 0.0) || !(at >= 0.0) || (rt == 0.0 && at == 0.0)) return false;
  for (int q = 0; q < dim; ++q)
    if (!__builtin_isfinite(double(a.y0[(long)i * a.D + q]))) return false;
  // sorted within [t0, t_end]: eight independent loads in flight at a time
  const double* tr = a.t_eval + (long)i * a.E;
  double prev = t0;
  bool sorted = true;
  int e = 0;
  for (; e + 8 <= a.E; e += 8) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = tr[e + q];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      sorted &= (v[q] >= prev) & (v[q] <= te);
      prev = v[q];
    }
  }
  for (; e < a.E; ++e) {
    const double v = tr[e];
    sorted &= (v >= prev) & (v <= te);
    prev = v;
  }
  if (!sorted) return false;
  if (a.h0 != nullptr && !(a.h0[i] > 0.0)) return false;
  return true;
}

// Hairer's starting step (Solving ODEs I, II.4) from f0 = f(t0, y0).
template <typename R, class F>
__device__ __forceinline__ R start_step(const AnalyticArgs<R>& a, Lane<R, F::N>& L,
                        const F& f) {
  constexpr int N = F::N;
  const double span = L.te - L.t;
  R sc[N], s0 = R(0), s1 = R(0);
#pragma unroll
  for (int q = 0; q < N; ++q) {
    sc[q] = L.atol + rabs(L.y[q]) * L.rtol;
    if (q < L.dim) {
      const R u = L.y[q] / sc[q], v = L.k[0][q] / sc[q];
      s0 += u * u;
      s1 += v * v;
    }
  }
  const R d0 = rsqrt_(s0 / R(L.dim)), d1 = rsqrt_(s1 / R(L.dim));
  R h0 = (d0 < R(1e-5) || d1 < R(1e-5)) ? R(1e-6) : R(0.01) * d0 / d1;
  h0 = rmin(h0, R(span));
  R y1[N], f1[N];
#pragma unroll
  for (int q = 0; q < N; ++q) y1[q] = L.y[q] + h0 * L.k[0][q];
  f(y1, f1);
  L.n_fe += 1;
  R s2 = R(0);
#pragma unroll
  for (int q = 0; q < N; ++q)
    if (q < L.dim) {
      const R u = (f1[q] - L.k[0][q]) / sc[q];
      s2 += u * u;
    }
  const R d2 = rsqrt_(s2 / R(L.dim)) / h0;
  R h1;
  if (d1 <= R(1e-15) && d2 <= R(1e-15))
    h1 = rmax(R(1e-6), h0 * R(1e-3));
  else
    h1 = rpow(R(0.01) / rmax(d1, d2), R(0.2));
  return rmin(rmin(R(100) * h0, h1), R(span));
}

template <typename R, class F>
__device__ __forceinline__ void init_one(const AnalyticArgs<R>& a, int i) {
  constexpr int N = F::N;
  Lane<R, N> L;
  F f;
  L.inst = i;
  L.dim = a.dim[i];
  f.load(a, i, L.dim);
  L.t = a.t0[i];
  L.te = a.t_end[i];
  L.rtol = R(a.rtol[i]);
  L.atol = R(a.atol[i]);
  const R* y0 = a.y0 + (long)i * a.D;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    L.y[q] = q < L.dim ? y0[q] : R(0);
    L.yc[q] = R(0);
  }
  f(L.y, L.k[0]);
  L.n_fe = 1;
  L.n_att = L.n_acc = L.n_rej = 0;
  L.prev_rej = 0;
  L.err_prev = L.err_prev2 = std::is_same<R, float>::value ? R(0) : R(1);
  L.cursor = 0;
  while (L.cursor < a.E && a.t_eval[(long)i * a.E + L.cursor] <= L.t) {
    write_row<R, N>(a.y_eval + ((long)i * a.E + L.cursor) * a.D, a.D, L.y,
                    L.dim);
    L.cursor += 1;
  }
  for (int e = L.cursor; e < a.E; ++e)
    for (int q = N; q < a.D; ++q)
      a.y_eval[((long)i * a.E + e) * a.D + q] = R(0);
  L.h = R(0);
  if (L.te == L.t) {
    L.status = kSuccess;
    finish_lane(a, L);
    return;
  }
  L.status = kRunning;
  L.h = a.h0 != nullptr ? R(a.h0[i]) : start_step(a, L, f);
  store_lane(a, L);
  if (a.kind[i] == kKindVdp) {
    const int p = atomicAdd(&a.counts[0], 1);
    a.list[p] = i;
  } else {
    const int p = atomicAdd(&a.counts[1], 1);
    a.list[a.B - 1 - p] = i;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void init_kernel(AnalyticArgs<R> a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.B) return;
  if (!instance_ok(a, i)) {
    const State<R>& s = a.st;
    s.status[i] = kInvalid;
    s.n_att[i] = s.n_acc[i] = s.n_rej[i] = s.n_fe[i] = 0;
    s.cursor[i] = 0;
    s.t[i] = a.t0[i];
    for (int q = 0; q < a.D; ++q) {
      a.y_final[(long)i * a.D + q] = quiet_nan<R>();
      s.y[(long)i * a.D + q] = quiet_nan<R>();
    }
    for (long e = 0; e < (long)a.E * a.D; ++e)
      a.y_eval[(long)i * a.E * a.D + e] = quiet_nan<R>();
    return;
  }
  if (a.kind[i] == kKindVdp)
    init_one<R, VdpField<R>>(a, i);
  else
    init_one<R, LinearField<R>>(a, i);
}

// ---- dense output of the last accepted step ------------------------------------

template <typename R>
__global__ void dense_eval_kernel(DenseKeep<R> dk, State<R> st, int B, int D,
                                  const double* t_query, R* y_out,
                                  int32_t* qstatus) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const double tq = t_query[i];
  const bool ok = st.n_acc[i] > 0 && tq >= dk.t_prev[i] && tq <= st.t[i];
  qstatus[i] = ok ? 0 : 1;
  const R th = ok ? R((tq - dk.t_prev[i]) / double(dk.h_last[i])) : R(0);
  for (int q = 0; q < D; ++q) {
    const long o = (long)i * D + q;
    if (!ok) {
      y_out[o] = quiet_nan<R>();
      continue;
    }
    const long bd = (long)B * D;
    const R v = dk.q[o] + th * (dk.q[bd + o] + th * (dk.q[2 * bd + o] +
                                                      th * dk.q[3 * bd + o]));
    y_out[o] = dk.y_prev[o] + th * v;
  }
}

__global__ void fill_i32_kernel(int32_t* p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---- launchers -----------------------------------------------------------------

// ---- joint (coupled) mode -----------------------------------------------------
//
// Section 4.1's comparison mode: the members (valid instances with the first
// valid instance's t0, t_end, evaluation times and h0) are one system of
// size sum(dim) with one time, step size, error norm (weighted RMS over all
// their components, each scaled by its own instance's tolerances) and
// accept/reject decision.  One workgroup owns the batch: each thread runs
// its instances' stages in registers, their scaled squared errors meet in a
// block reduction (fixed order), thread 0 takes the decision and the
// controller step, and the threads commit their instances.

constexpr int kJointThreads = 256;

template <typename T>
__device__ __forceinline__ T joint_sum(T v, T* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  T acc = T(0);
  for (int q = 0; q < kJointThreads / 64; ++q) acc += red[q];
  return acc;
}

template <typename R>
__device__ __forceinline__ bool joint_member(const AnalyticArgs<R>& a, int i,
                                             int ref) {
  if (a.st.status[i] == kInvalid) return false;
  if (a.t0[i] != a.t0[ref] || a.t_end[i] != a.t_end[ref]) return false;
  // same evaluation times: eight pairs of loads in flight at a time
  const double* ti = a.t_eval + (long)i * a.E;
  const double* tr = a.t_eval + (long)ref * a.E;
  bool same = true;
  int e = 0;
  for (; e + 8 <= a.E; e += 8) {
    double u[8], v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      u[q] = ti[e + q];
      v[q] = tr[e + q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) same &= u[q] == v[q];
  }
  for (; e < a.E; ++e) same &= ti[e] == tr[e];
  if (!same) return false;
  if (a.h0 != nullptr && a.h0[i] != a.h0[ref]) return false;
  return true;
}

// Stages 2..7 of member i from (t, y_i, k1_i) with step hs: k_2..k_7 and
// the candidate solution go to the workspace; returns the instance's sum
// of squared scaled errors.
template <typename R, class M, class F>
__device__ R joint_stages(const AnalyticArgs<R>& a, int i, double t, R hs) {
  constexpr int N = F::N;
  F f;
  const int dim = a.dim[i];
  f.load(a, i, dim);
  const long B = a.B, D = a.D;
  R y[N], k[7][N], Y[N];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    y[q] = q < dim ? a.st.y[i * D + q] : R(0);
    k[0][q] = q < dim ? a.st.k1[i * D + q] : R(0);
  }
  (void)t;  // the analytic fields are autonomous
#pragma unroll
  for (int s = 1; s < 7; ++s) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R acc = R(0);
#pragma unroll
      for (int j = 0; j < s; ++j)
        if (M::A[s][j] != 0.0) acc += R(M::A[s][j]) * k[j][q];
      Y[q] = y[q] + hs * acc;
    }
    f(Y, k[s]);
  }
  R e2 = R(0);
#pragma unroll
  for (int q = 0; q < N; ++q) {
    if (q >= dim) continue;
    R eq = R(0);
#pragma unroll
    for (int j = 0; j < 7; ++j)
      if (M::E[j] != 0.0) eq += R(M::E[j]) * k[j][q];
    eq *= hs;
    const R sc = R(a.atol[i]) + R(a.rtol[i]) * rmax(rabs(y[q]), rabs(Y[q]));
    const R r = eq / sc;
    e2 += r * r;
    a.jY[i * D + q] = Y[q];
#pragma unroll
    for (int s = 1; s < 7; ++s) a.jK[((s - 1) * B + i) * D + q] = k[s][q];
  }
  return e2;
}

template <typename R>
__device__ void joint_write_stats(const AnalyticArgs<R>& a, int i,
                                  const JointState& j) {
  a.st.n_att[i] = j.n_att;
  a.st.n_acc[i] = j.n_acc;
  a.st.n_rej[i] = j.n_rej;
  a.st.n_fe[i] = 1 + j.probe + 6 * j.n_att;
  a.st.status[i] = j.status;
  a.st.t[i] = j.t;
  a.st.h[i] = R(j.h);
  a.st.cursor[i] = j.cursor;
}

template <typename R>
__device__ void joint_finish(const AnalyticArgs<R>& a, int i,
                             const JointState& j) {
  const int dim = a.dim[i];
  for (int q = 0; q < a.D; ++q)
    a.y_final[(long)i * a.D + q] =
        q < dim ? a.st.y[(long)i * a.D + q] : R(0);
  if (j.status != kSuccess)
    for (int e = j.cursor; e < a.E; ++e)
      for (int q = 0; q < a.D; ++q)
        a.y_eval[((long)i * a.E + e) * a.D + q] =
            q < dim ? quiet_nan<R>() : R(0);
}

template <typename R>
__device__ void joint_rhs(const AnalyticArgs<R>& a, int i, const R* y, R* f) {
  if (a.kind[i] == kKindVdp) {
    VdpField<R> F;
    F.load(a, i, 2);
    F(y, f);
  } else {
    LinearField<R> F;
    F.load(a, i, a.dim[i]);
    F(y, f);
  }
}

template <typename R>
__global__ __launch_bounds__(kJointThreads) void joint_init_kernel(
    AnalyticArgs<R> a) {
  __shared__ double red[kJointThreads / 64];
  __shared__ int32_t ref_s;
  const int tid = threadIdx.x;
  const long D = a.D;
  if (tid == 0) ref_s = a.B;
  __syncthreads();
  for (int i = tid; i < a.B; i += kJointThreads) {
    const bool ok = instance_ok(a, i);
    a.st.status[i] = ok ? kRunning : kInvalid;
    if (ok) atomicMin(&ref_s, i);
  }
  __syncthreads();
  const int ref = ref_s;
  double n_loc = 0.0, s0 = 0.0, s1 = 0.0;
  for (int i = tid; i < a.B; i += kJointThreads) {
    const bool member = ref < a.B && joint_member(a, i, ref);
    const int dim = a.dim[i];
    a.st.n_att[i] = a.st.n_acc[i] = a.st.n_rej[i] = a.st.n_fe[i] = 0;
    a.st.cursor[i] = 0;
    if (!member) {
      a.st.status[i] = kInvalid;
      a.st.t[i] = a.t0[i];
      for (long q = 0; q < D; ++q) {
        a.y_final[i * D + q] = quiet_nan<R>();
        a.st.y[i * D + q] = quiet_nan<R>();
      }
      for (long e = 0; e < (long)a.E * D; ++e)
        a.y_eval[i * a.E * D + e] = quiet_nan<R>();
      continue;
    }
    R y[8], f[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      y[q] = q < dim ? a.y0[i * D + q] : R(0);
    joint_rhs(a, i, y, f);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q >= D) continue;
      a.st.y[i * D + q] = q < dim ? y[q] : R(0);
      a.st.k1[i * D + q] = q < dim ? f[q] : R(0);
    }
    for (int e = 0; e < a.E; ++e) {
      const double te = a.t_eval[(long)i * a.E + e];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (q >= D) continue;
        a.y_eval[((long)i * a.E + e) * D + q] =
            q < dim ? (te <= a.t0[i] ? y[q] : quiet_nan<R>()) : R(0);
      }
    }
    n_loc += dim;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q >= dim) continue;
      const R sc = R(a.atol[i]) + rabs(y[q]) * R(a.rtol[i]);
      s0 += double((y[q] / sc) * (y[q] / sc));
      s1 += double((f[q] / sc) * (f[q] / sc));
    }
  }
  // Hairer's start step on the stacked vector (sums in the state precision
  // for FP32, exactly as the independent solve forms them per instance)
  const double n_tot = joint_sum(n_loc, red);
  const double S0 = joint_sum(s0, red), S1 = joint_sum(s1, red);
  JointState j{};
  j.ref = ref;
  j.n_total = int32_t(n_tot);
  j.status = (ref < a.B) ? kRunning : kInvalid;
  j.err_prev = j.err_prev2 = 1.0;
  j.t = ref < a.B ? a.t0[ref] : 0.0;
  j.t_end = ref < a.B ? a.t_end[ref] : 0.0;
  j.cursor = 0;
  if (ref < a.B)
    while (j.cursor < a.E && a.t_eval[(long)ref * a.E + j.cursor] <= j.t)
      ++j.cursor;
  if (j.status == kRunning && j.t_end == j.t) {
    j.status = kSuccess;
  } else if (j.status == kRunning && a.h0 != nullptr) {
    j.h = a.h0[ref];
  } else if (j.status == kRunning) {
    const double span = j.t_end - j.t;
    const double d0 = sqrt(S0 / n_tot), d1 = sqrt(S1 / n_tot);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    h0 = fmin(h0, span);
    double s2 = 0.0;
    for (int i = tid; i < a.B; i += kJointThreads) {
      if (!joint_member(a, i, ref)) continue;
      const int dim = a.dim[i];
      R y[8], f0[8], y1[8], f1[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        y[q] = q < dim ? a.st.y[i * D + q] : R(0);
        f0[q] = q < dim ? a.st.k1[i * D + q] : R(0);
        y1[q] = y[q] + R(h0) * f0[q];
      }
      joint_rhs(a, i, y1, f1);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (q >= dim) continue;
        const R sc = R(a.atol[i]) + rabs(y[q]) * R(a.rtol[i]);
        const R d = (f1[q] - f0[q]) / sc;
        s2 += double(d * d);
      }
    }
    const double d2 = sqrt(joint_sum(s2, red) / n_tot) / h0;
    const double h1 = (d1 <= 1e-15 && d2 <= 1e-15)
                          ? fmax(1e-6, h0 * 1e-3)
                          : pow(0.01 / fmax(d1, d2), 1.0 / 5.0);
    j.h = fmin(fmin(100.0 * h0, h1), span);
    j.probe = 1;
  }
  for (int i = tid; i < a.B; i += kJointThreads) {
    if (a.st.status[i] == kInvalid) continue;
    joint_write_stats(a, i, j);
    if (j.status != kRunning) joint_finish(a, i, j);
  }
  if (tid == 0) *a.js = j;
}

template <typename R, class M>
__global__ __launch_bounds__(kJointThreads) void joint_solve_kernel(
    AnalyticArgs<R> a) {
  __shared__ double red[kJointThreads / 64];
  __shared__ JointState js;
  __shared__ int32_t acc_s, cur_new;
  __shared__ double tnew_s, fac_s, err_s;
  const int tid = threadIdx.x;
  const long B = a.B, D = a.D;
  if (tid == 0) js = *a.js;
  __syncthreads();
  const int ref = js.ref;
  const Ctrl& c = a.ctrl;
  for (int it = 0; it < a.budget && js.status == kRunning; ++it) {
    if (js.n_att >= c.max_steps) {
      __syncthreads();
      if (tid == 0) js.status = kMaxSteps;
      __syncthreads();
      break;
    }
    const bool last = js.t + js.h >= js.t_end;
    const R hs = last ? R(js.t_end - js.t) : R(js.h);
    double part = 0.0;
    for (int i = tid; i < B; i += kJointThreads) {
      if (a.st.status[i] == kInvalid) continue;
      part += double(a.kind[i] == kKindVdp
                         ? joint_stages<R, M, VdpField<R>>(a, i, js.t, hs)
                         : joint_stages<R, M, LinearField<R>>(a, i, js.t, hs));
    }
    const double acc = joint_sum(part, red);
    __syncthreads();
    if (tid == 0) {
      const double err = sqrt(acc / double(js.n_total));
      const bool accept = err < 1.0;
      double fac;
      if (!__builtin_isfinite(err)) {
        fac = c.fac_min;
      } else if (accept) {
        if (err == 0.0) {
          fac = c.fac_max;
        } else {
          fac = c.safety * pow(err, -c.beta1) * pow(js.err_prev, c.beta2) *
                pow(js.err_prev2, c.beta3);
          fac = fac < c.fac_min ? c.fac_min : (fac > c.fac_max ? c.fac_max : fac);
        }
        if (js.prev_rej) fac = fmin(1.0, fac);
      } else {
        fac = fmax(c.fac_min, c.safety * pow(err, -1.0 / 5.0));
      }
      js.n_att += 1;
      acc_s = accept;
      int cur = js.cursor;
      if (accept) {
        const double tnew = last ? js.t_end : js.t + double(hs);
        while (cur < a.E && a.t_eval[(long)ref * a.E + cur] <= tnew) ++cur;
        tnew_s = tnew;
        js.err_prev2 = js.err_prev;
        js.err_prev = fmax(err, 1e-4);
        js.n_acc += 1;
        js.prev_rej = 0;
        if (last) js.status = kSuccess;
      } else {
        tnew_s = js.t;
        js.n_rej += 1;
        js.prev_rej = 1;
      }
      cur_new = cur;
      fac_s = fac;
      err_s = err;
    }
    __syncthreads();
    if (a.h_rec != nullptr && js.n_att <= a.rec_cap)  // every member's row
      for (int i = tid; i < B; i += kJointThreads) {
        if (a.st.status[i] == kInvalid) continue;
        const long o = (long)i * a.rec_cap + js.n_att - 1;
        a.h_rec[o] = acc_s ? double(hs) : -double(hs);
        a.e_rec[o] = err_s;
      }
    if (acc_s) {  // dense outputs in (t, t_new], then y <- Y7, k1 <- k7
      for (int i = tid; i < B; i += kJointThreads) {
        if (a.st.status[i] == kInvalid) continue;
        const int dim = a.dim[i];
        for (int e = js.cursor; e < cur_new; ++e) {
          const R th = R((a.t_eval[(long)ref * a.E + e] - js.t) / double(hs));
          R w[7];
#pragma unroll
          for (int q = 0; q < 7; ++q)
            w[q] = th * (R(M::P[q][0]) +
                         th * (R(M::P[q][1]) +
                               th * (R(M::P[q][2]) + th * R(M::P[q][3]))));
          for (int q = 0; q < dim; ++q) {
            R s2 = w[0] * a.st.k1[i * D + q];
            for (int st = 1; st < 7; ++st)
              s2 += w[st] * a.jK[((st - 1) * B + i) * D + q];
            a.y_eval[((long)i * a.E + e) * D + q] = a.st.y[i * D + q] + hs * s2;
          }
        }
        for (int q = 0; q < dim; ++q) {
          a.st.y[i * D + q] = a.jY[i * D + q];
          a.st.k1[i * D + q] = a.jK[(5 * B + i) * D + q];
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      if (acc_s) {
        js.t = tnew_s;
        js.cursor = cur_new;
      }
      js.h = double(hs * R(fac_s));  // in the state precision
      if (js.status == kRunning &&
          !(js.h > 16.0 * DBL_EPSILON * fabs(js.t)))
        js.status = kDtUnderflow;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int i = tid; i < B; i += kJointThreads) {
    if (a.st.status[i] == kInvalid) continue;
    joint_write_stats(a, i, js);
    if (js.status != kRunning) joint_finish(a, i, js);
  }
  if (tid == 0) *a.js = js;
}

template <typename R>
hipError_t launch_analytic_init(const AnalyticArgs<R>& a, int, hipStream_t s) {
  const int block = 256;
  const int grid = (a.B + block - 1) / block;
  hipLaunchKernelGGL(init_kernel<R>, dim3(grid), dim3(block), 0, s, a);
  return hipGetLastError();
}

constexpr int kWindowMinE = 64;

template <typename R, class M, class F>
void launch_solve_flags(const AnalyticArgs<R>& a, int kind, dim3 g, dim3 b,
                        hipStream_t s) {
  const bool rec = a.h_rec != nullptr, keep = a.keep_dense != 0;
  // many evaluation times per instance: the eight-time window (measured on
  // the paper's 256-instance, 200-time Van der Pol workload)
  if (!rec && !keep && a.E >= kWindowMinE)
    hipLaunchKernelGGL((solve_kernel<R, M, F, false, false, 8>), g, b, 0, s,
                       a, kind);
  else if (rec && keep)
    hipLaunchKernelGGL((solve_kernel<R, M, F, true, true>), g, b, 0, s, a, kind);
  else if (rec)
    hipLaunchKernelGGL((solve_kernel<R, M, F, true, false>), g, b, 0, s, a,
                       kind);
  else if (keep)
    hipLaunchKernelGGL((solve_kernel<R, M, F, false, true>), g, b, 0, s, a,
                       kind);
  else
    hipLaunchKernelGGL((solve_kernel<R, M, F, false, false>), g, b, 0, s, a,
                       kind);
}

template <typename R>
hipError_t launch_analytic_solve(const AnalyticArgs<R>& a, int method,
                                 int kind, int lanes, int block,
                                 hipStream_t s) {
  if (block <= 0) block = 64;
  if (lanes <= 0) lanes = a.B;
  const int grid = (lanes + block - 1) / block;
  if (grid == 0) return hipSuccess;
  const dim3 g(grid), b(block);
  if (kind == kKindVdp) {
    if (method == 1)
      launch_solve_flags<R, Tsit5, VdpField<R>>(a, kind, g, b, s);
    else
      launch_solve_flags<R, Dopri5, VdpField<R>>(a, kind, g, b, s);
  } else {
    if (method == 1)
      launch_solve_flags<R, Tsit5, LinearField<R>>(a, kind, g, b, s);
    else
      launch_solve_flags<R, Dopri5, LinearField<R>>(a, kind, g, b, s);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_dense_eval(const DenseKeep<R>& dk, const State<R>& st,
                             int B, int D, const double* t_query, R* y_out,
                             int32_t* qstatus, hipStream_t s) {
  const int block = 256;
  hipLaunchKernelGGL(dense_eval_kernel<R>, dim3((B + block - 1) / block),
                     dim3(block), 0, s, dk, st, B, D, t_query, y_out, qstatus);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s,
                     p, n, v);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_joint_init(const AnalyticArgs<R>& a, int, hipStream_t s) {
  if (a.js == nullptr || a.jK == nullptr || a.jY == nullptr)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(joint_init_kernel<R>, dim3(1), dim3(kJointThreads), 0, s,
                     a);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_joint_solve(const AnalyticArgs<R>& a, int method,
                              hipStream_t s) {
  if (a.js == nullptr || a.jK == nullptr || a.jY == nullptr)
    return hipErrorInvalidValue;
  if (method == 1)
    hipLaunchKernelGGL((joint_solve_kernel<R, Tsit5>), dim3(1),
                       dim3(kJointThreads), 0, s, a);
  else
    hipLaunchKernelGGL((joint_solve_kernel<R, Dopri5>), dim3(1),
                       dim3(kJointThreads), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_joint_init<double>(const AnalyticArgs<double>&,
                                              int, hipStream_t);
template hipError_t launch_joint_init<float>(const AnalyticArgs<float>&, int,
                                             hipStream_t);
template hipError_t launch_joint_solve<double>(const AnalyticArgs<double>&,
                                               int, hipStream_t);
template hipError_t launch_joint_solve<float>(const AnalyticArgs<float>&, int,
                                              hipStream_t);
template hipError_t launch_analytic_init<double>(const AnalyticArgs<double>&,
                                                 int, hipStream_t);
template hipError_t launch_analytic_init<float>(const AnalyticArgs<float>&,
                                                int, hipStream_t);
template hipError_t launch_analytic_solve<double>(const AnalyticArgs<double>&,
                                                  int, int, int, int,
                                                  hipStream_t);
template hipError_t launch_analytic_solve<float>(const AnalyticArgs<float>&,
                                                 int, int, int, int,
                                                 hipStream_t);
template hipError_t launch_dense_eval<double>(const DenseKeep<double>&,
                                              const State<double>&, int, int,
                                              const double*, double*,
                                              int32_t*, hipStream_t);
template hipError_t launch_dense_eval<float>(const DenseKeep<float>&,
                                             const State<float>&, int, int,
                                             const double*, float*, int32_t*,
                                             hipStream_t);

}  // namespace bode
