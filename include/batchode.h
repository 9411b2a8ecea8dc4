/*
 * batchode: a batched adaptive explicit Runge-Kutta solver for MI355X (gfx950).
 *
 * It implements the parallel solving method of Lienen & Guennemann,
 * "torchode: A Parallel ODE Solver for PyTorch" (arXiv 2210.12375): a batch of
 * independent initial value problems is advanced together, and every instance
 * keeps its own time, step size, error estimate, step-size-controller state
 * and accept/reject decision (section 3, "Design & Features"; section 4.1
 * shows why a shared step size is wrong for uneven batches).  Evaluation
 * times are per instance and answered by dense output (section 3, "What slows
 * torchode down?").
 *
 * Calling convention
 *  - Plain C ABI: no C++ exception crosses it.  Every call returns BODE_OK (0)
 *    or a negative BODE_E* code; solver_last_error() gives the text.
 *  - Device pointers are HIP device allocations owned by the caller.  Inputs
 *    are borrowed: they must stay valid and unchanged until solver_destroy()
 *    (the backward pass re-reads y0 and the parameters).  The library never
 *    allocates device memory: all scratch lives in the caller's workspace of
 *    solver_workspace_size() bytes (solver_solve_noalloc instead uses one
 *    static device array that the library's code object holds per GPU).
 *  - All device work is enqueued on the caller's stream (a hipStream_t passed
 *    as void*) and is asynchronous unless a call says otherwise.
 *  - Per-instance numerical outcomes are a status (BODE_SUCCESS,
 *    BODE_MAX_STEPS, ...), never an error code.
 *
 * Layout: every per-instance array is instance-major ("[B, D]" means
 * B rows of D elements, row stride D).  State-typed arrays are double in
 * BODE_FP64 mode and float otherwise; times are always double.
 */
#ifndef BATCHODE_H
#define BATCHODE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- enumerations ------------------------------------------------------ */

/* Runge-Kutta pairs (paper appendix A: "dopri5" in every experiment; "tsit5"
 * is also provided).  Both are 7-stage, FSAL, order 5 with an embedded
 * order-4 error estimate and a fourth-order continuous extension.          */
#define BODE_DOPRI5 0
#define BODE_TSIT5 1

/* Arithmetic of the solve.
 *  FP64: state, stages, norm, controller and time in double.
 *  FP32: state, stages, norm and controller in float; time in double.
 *  BF16: as FP32, but neural right-hand sides run their GEMMs on BF16 MFMA
 *        with FP32 accumulation (analytic right-hand sides behave as FP32). */
#define BODE_FP64 0
#define BODE_FP32 1
#define BODE_BF16 2

/* Right-hand-side families.  ANALYTIC batches mix, per instance (kind[]),
 *  BODE_KIND_VDP:    x' = v, v' = mu (1 - x^2) v - x  (section 4.1, Eq. eq:vdp)
 *  BODE_KIND_LINEAR: y' = A y with A of size dim x dim, dim <= 8.          */
#define BODE_RHS_ANALYTIC 0
#define BODE_RHS_MLP 2
#define BODE_RHS_CNF 3

#define BODE_KIND_VDP 0
#define BODE_KIND_LINEAR 1

/* Per-instance status. */
#define BODE_RUNNING 0
#define BODE_SUCCESS 1
#define BODE_MAX_STEPS 2
#define BODE_DT_UNDERFLOW 3
#define BODE_INVALID 4

/* Error codes. */
#define BODE_OK 0
#define BODE_EINVAL (-1)       /* bad argument or configuration              */
#define BODE_EUNSUPPORTED (-2) /* valid but not built (e.g. CNF in FP64 MFMA) */
#define BODE_EHIP (-3)         /* a HIP runtime call failed                   */
#define BODE_ESTATE (-4)       /* call out of order (e.g. eval before a step) */

/* ---- configuration ----------------------------------------------------- */

typedef struct {
  int32_t method;    /* BODE_DOPRI5 | BODE_TSIT5                              */
  int32_t precision; /* BODE_FP64 | BODE_FP32 | BODE_BF16                     */
  int32_t rhs;       /* BODE_RHS_*                                            */
  int32_t B;         /* instances, >= 1                                       */
  int32_t D;         /* row stride of state arrays: ANALYTIC <= 8; MLP = d;
                        CNF = d + 1 (the last component is the log-density)   */
  int32_t E;         /* evaluation times per instance, >= 0                   */
  int32_t max_steps; /* attempted steps per instance before BODE_MAX_STEPS    */
  /* Step-size controller (section 3: the PID family generalises the
   * integral controller; appendix C).  After an accepted step with error
   * norm err the step is scaled by
   *   clamp(safety * err^-beta1 * err_prev^beta2 * err_prev2^beta3,
   *         fac_min, fac_max),
   * err_prev, err_prev2 the norms of the two previous accepted steps
   * (clamped below at 1e-4; 1 before there were any), capped at 1 right
   * after a rejection; after a rejected step by max(fac_min, safety *
   * err^-1/5).  err = 0 gives fac_max.  beta2 = beta3 = 0 is the integral
   * controller; beta1 = 0.14, beta2 = 0.08 is Gustafsson's PI controller; a
   * PID law on log err with gains (kI, kP, kD) for an order-5 error estimate
   * has beta1 = (kI + kP + kD)/5, beta2 = (kP + 2 kD)/5, beta3 = -kD/5.
   * beta3 is the last member of this struct.                               */
  double beta1, beta2, safety, fac_min, fac_max;
  int32_t record_cap; /* attempted step sizes kept per instance (0: none);
                         solver_backward needs >= the largest attempt count */
  int32_t keep_dense; /* 1: keep the last accepted step's interpolant so
                         solver_eval can answer queries                      */
  int32_t mlp_hidden; /* MLP / CNF hidden width (both hidden layers)         */
  int32_t tune_block; /* launch tuning (0 = library / autotuned default)     */
  int32_t tune_lanes;
  int32_t ckpt_every; /* neural fields: keep y_n every ckpt_every accepted
                         steps for solver_backward (0: no checkpoints); the
                         backward recomputes the states in between          */
  double beta3;       /* third controller exponent (PID); 0 for I and PI    */
  int32_t joint;      /* 1: joint (coupled) batch mode of section 4.1, the
                         comparison mode: the members (valid instances with
                         the first valid instance's t0, t_end, t_eval and h0;
                         the others are BODE_INVALID) are solved as one
                         system with one step size, one error norm (RMS over
                         all their components) and one accept/reject
                         decision.  ANALYTIC fields and keep_dense = 0
                         only; with record_cap every member's row holds the
                         joint attempts.  0: independent instances.        */
  int32_t eager;      /* neural fields: 1 launches every kernel of the round
                         loops directly; 0 (default) captures a block of
                         rounds (and of continuous-adjoint attempts) into a
                         HIP graph once per handle / call and replays it.
                         Results are identical.                             */
  int32_t fixed_step; /* 1: fixed-step integration (a validation mode, not
                         one of the paper's controllers; its closed form
                         R(hA)^N y0 checks the stage arithmetic without a
                         controller): every instance steps with its own
                         h0 (bode_problem.h0 is then required), every attempt
                         is accepted, the step that would pass t_end is
                         clipped to end there; the error estimate is not
                         used.  Not with joint mode or solver_cadjoint.
                         0: adaptive (the controller above).                */
  int32_t plain_bf16; /* BF16 mode with MLP / CNF fields: 1 rounds every
                         activation to one BF16 value (8 significant bits;
                         one MFMA per fragment, a third of the matrix-core
                         work); 0 (default) splits it into three BF16 terms
                         (24 bits), so the only BF16 rounding is that of
                         the weights.  Plain BF16 is built for forward
                         solves: solver_backward and solver_cadjoint return
                         BODE_EUNSUPPORTED for it.                           */
} bode_config;

/* Problem description: device pointers (NULL where not used). */
typedef struct {
  const void* y0;       /* [B, D] initial states (padding columns ignored)   */
  const double* t0;     /* [B]                                               */
  const double* t_end;  /* [B], t_end >= t0                                  */
  const double* rtol;   /* [B], >= 0                                         */
  const double* atol;   /* [B], >= 0, not both zero                          */
  const double* t_eval; /* [B, E], each row non-decreasing within [t0, t_end]*/
  const double* h0;     /* [B] first step, or NULL for Hairer's rule          */
  const int32_t* kind;  /* [B] BODE_KIND_* (ANALYTIC only)                    */
  const int32_t* dim;   /* [B] true dimension: VDP 2, LINEAR 1..8 (ANALYTIC)  */
  const void* mu;       /* [B] Van der Pol damping (ANALYTIC)                */
  const void* A;        /* [B, D, D] row-major linear systems (ANALYTIC)     */
  /* MLP / CNF parameters, state-typed, W_l stored [fan_in, fan_out]:
   * x = [y, t] (MLP) or [z, t] (CNF); a1 = tanh(x W1 + b1);
   * a2 = tanh(a1 W2 + b2); out = a2 W3 + b3.                              */
  const void *W1, *b1, *W2, *b2, *W3, *b3;
  const void* eps;      /* [B, D] Rademacher probes (CNF; first D-1 used)    */
  void* y_eval;         /* [B, E, D] output: solution at t_eval              */
  void* y_final;        /* [B, D]    output: state at t_end (or at failure)  */
} bode_problem;

typedef struct bode_solver bode_solver;

/* ---- calls ------------------------------------------------------------- */

/* Bytes of device workspace solver_init needs for cfg (0 if cfg invalid). */
size_t solver_workspace_size(const bode_config* cfg);

/* Validates cfg and the host-visible parts of p, lays out the workspace and
 * enqueues the initialisation of every instance on `stream`: the first stage
 * k1 = f(t0, y0), Hairer's starting step (Solving ODEs I, II.4) unless h0 is
 * given, answers for evaluation times equal to t0, and per-instance checks
 * of the device inputs (a bad instance gets status BODE_INVALID).
 * On success *out is a new handle.                                          */
int solver_init(const bode_config* cfg, const bode_problem* p, void* workspace,
                size_t workspace_bytes, void* stream, bode_solver** out);

/* Every RUNNING instance attempts up to n_attempts further steps (each
 * accepted or rejected by its own error norm).  If n_running_host is not
 * NULL the call synchronises the stream and stores the number of instances
 * still RUNNING there.                                                      */
int solver_step(bode_solver* s, int32_t n_attempts, int32_t* n_running_host);

/* Steps every instance to completion (t_end, max_steps or a failure).
 * Asynchronous.                                                             */
int solver_solve(bode_solver* s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * solver_init + solver_solve in one call with the same kernels and results,
 * but the workspace is a static device array owned by the library
 * (32 MiB per GPU, held from the library's load until the process ends)
 * instead of caller memory; no device memory is allocated or freed.
 * Analytic right-hand sides only (BODE_EUNSUPPORTED otherwise); a
 * configuration whose solver_workspace_size() exceeds 32 MiB is rejected
 * with BODE_EINVAL.  p is as for solver_init (inputs read, y_eval and
 * y_final written).  stats (device int32 [5, B], may be NULL) receives the
 * attempted, accepted and rejected steps, evaluations and status of every
 * instance.  Asynchronous on `stream`.  Every call on one GPU uses that
 * GPU's one array and leaves its contents behind: calls that overlap on one
 * GPU (other streams or threads) race and must be ordered by the caller.
 * There is no handle, so solver_step, solver_eval and the backward passes
 * are not available for such a solve.                                      */
int solver_solve_noalloc(const bode_config* cfg, const bode_problem* p,
                         int32_t* stats, void* stream);

/* Dense output of each instance's last accepted step at its own query time:
 * for t_query[i] in [t_prev_i, t_i] writes y_out[i, :] and qstatus[i] = 0,
 * otherwise qstatus[i] = 1 and y_out[i, :] = NaN.  Needs cfg.keep_dense.
 * t_query [B] double, y_out [B, D] state-typed, qstatus [B] int32: device.  */
int solver_eval(bode_solver* s, const double* t_query, void* y_out,
                int32_t* qstatus);

/* Discrete adjoint through the accepted steps (step sizes and accept
 * decisions frozen; paper section 4.2 trains by backpropagating through the
 * solver).  g_y_eval [B, E, D] (may be NULL) and g_y_final [B, D] are the
 * cotangents of y_eval and y_final; writes dy0 [B, D] and, for MLP / CNF,
 * dtheta = gradients of (W1, b1, W2, b2, W3, b3) concatenated, summed over
 * instances.  Needs a completed solve with cfg.record_cap covering every
 * instance's accepted steps.                                               */
int solver_backward(bode_solver* s, const void* g_y_eval, const void* g_y_final,
                    void* dy0, void* dtheta);

/* Continuous adjoint (appendix A: the CNF is trained through the adjoint
 * equation).  After a completed solve of an MLP or CNF field, the augmented
 * system y' = f, a' = -(df/dy)^T a, g' = -(df/dtheta)^T a is integrated
 * adaptively from t_end back to t0 with the solve's method, controller,
 * tolerances and max_steps, starting from y_final, a = the cotangent of
 * y(t_end) and g = 0; the solve stops at every evaluation time inside
 * (t0, t_end) to add that output's cotangent to a.  joint = 0: every
 * instance integrates its own (y_i, a_i, g_i), 2 D + P variables with its
 * own steps and error norm (the paper's b (f + p) system); joint = 1: the
 * members (instances whose solve succeeded and that share the first such
 * instance's t0, t_end and t_eval) are stacked with one shared g into one
 * system with one step size (the b f + p system).  Each component is scaled
 * by atol + rtol max(|z_n|, |z_n+1|) with its instance's tolerances (the
 * shared g with the first member's); the start step is Hairer's rule on the
 * augmented state.
 * g_y_eval [B, E, D] (may be NULL when E = 0) and g_y_final [B, D] are
 * state-typed device arrays.  Outputs (device): dy0 [B, D] = a(t0) plus the
 * cotangents at t0 (NaN for instances not differentiated), dtheta [P] = the
 * sum of the g_i (per instance) or the shared g, in solver_backward's
 * layout, and, if stats is not NULL, int32 [5, B] of the backward solve:
 * attempted, accepted, rejected steps, augmented evaluations (1 + probe + 6
 * per attempt + 1 per evaluation-time stop) and status (BODE_INVALID for
 * instances not differentiated).  workspace: device memory of at least
 * solver_cadjoint_workspace_bytes(s, joint) bytes, owned by the caller;
 * per instance it holds two [B, P] copies of the parameter adjoints.
 * Synchronises the stream a few times per step.  Errors: BODE_EINVAL
 * (missing argument, joint not 0/1, workspace too small), BODE_ESTATE (no
 * completed solve), BODE_EUNSUPPORTED (analytic right-hand sides).        */
size_t solver_cadjoint_workspace_bytes(const bode_solver* s, int32_t joint);
int solver_cadjoint(bode_solver* s, int32_t joint, const void* g_y_eval,
                    const void* g_y_final, void* workspace,
                    size_t workspace_bytes, void* dy0, void* dtheta,
                    int32_t* stats);

/* Per-instance statistics (section 3: total and accepted steps are collected
 * by default), copied asynchronously into device int32 arrays [B] (any may
 * be NULL): attempted, accepted and rejected steps, right-hand-side
 * evaluations (1 + starting-step probe + 6 per attempt) and status.        */
int solver_get_stats(const bode_solver* s, int32_t* n_attempted,
                     int32_t* n_accepted, int32_t* n_rejected,
                     int32_t* n_feval, int32_t* status);

/* The step record, copied into device arrays h [B, record_cap] (double):
 * the size of every attempted step in order, negated for rejected attempts,
 * and n [B] (int32): the number of attempts (it may exceed record_cap, in
 * which case only the first record_cap are kept).                          */
int solver_get_steps(const bode_solver* s, double* h, int32_t* n);

/* The weighted RMS error norm of every recorded attempt (section 3: each
 * instance decides on its own error estimate), copied into the device array
 * err [B, record_cap] (double) beside solver_get_steps' record: the value
 * the controller used, so an attempt was accepted exactly when its norm is
 * below 1 (always, in fixed-step mode).  In FP32 and BF16 modes the norm is
 * the float value widened to double.  Needs record_cap > 0 (BODE_ESTATE
 * otherwise).                                                              */
int solver_get_errors(const bode_solver* s, double* err);

/* Times launch candidates for this configuration on the caller's problem
 * (outputs are overwritten) and keeps the fastest for later solver_init
 * calls with the same shape: device architecture, right-hand side,
 * precision, method, B, D, E, hidden width and plain_bf16.  Candidates:
 * analytic fields, threads per workgroup {64, 128, 256} x lanes launched
 * {B, B/2, B/4}; matrix-core neural fields, wavefronts per 16-row tile
 * {4, 8}; the per-stage neural path, rounds per captured graph {4, 8, 16}.
 * All candidates give bitwise the same results.  If the environment
 * variable BATCHODE_TUNE_CACHE names a file, the kept shapes are read from
 * it on first use and the file is rewritten after every autotune (one JSON
 * object per line).  Synchronous.  (A performance tool, not a step of the
 * paper's method.)                                                        */
int solver_autotune(const bode_config* cfg, const bode_problem* p,
                    void* workspace, size_t workspace_bytes, void* stream);

/* The launch shape solver_init would use for cfg on the current device:
 * shape[5] (host int32) = threads per workgroup, lanes for Van der Pol and
 * for linear instances (analytic fields), wavefronts per tile and rounds
 * per graph (neural fields); 0 means the library default.               */
int solver_get_tune(const bode_config* cfg, int32_t* shape);

/* Releases the host handle (no device memory is owned). */
void solver_destroy(bode_solver* s);

/* Text of the last error of s, or of the calling thread if s is NULL. */
const char* solver_last_error(const bode_solver* s);

/* Host-side copy of the constants the kernels use, for checks without a GPU:
 * c[7], a[49] row-major, b[7], e[7] (= b - bhat), dense[28] with
 * w_j(theta) = sum_m dense[j*4 + m] theta^(m+1).  Returns BODE_EINVAL for an
 * unknown method.                                                          */
int solver_tableau(int32_t method, double* c, double* a, double* b, double* e,
                   double* dense);

#ifdef __cplusplus
}
#endif
#endif
