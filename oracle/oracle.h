/*
 * Plain FP64 CPU oracle for the batched adaptive Runge-Kutta solver of
 * Lienen & Guennemann, "torchode: A Parallel ODE Solver for PyTorch"
 * (arXiv 2210.12375).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can check the HIP solver against a slow, obviously
 * correct implementation.  It shares no code, header or constant table with
 * the GPU library.
 *
 * What it computes (paper section 3, "Design & Features"): every instance of a
 * batch is an independent initial value problem with its own initial state,
 * integration bounds, tolerances, step size, error estimate, controller state
 * and accept/reject decision.  Instances are solved one at a time by a scalar
 * loop; OpenMP only spreads whole instances over host threads.
 *
 * Pins (tests/test_oracle_*.py): tableau order conditions, stability
 * polynomial, order-5 convergence, scipy's RK45 and initial-step routine
 * (same Dormand-Prince pair, same integral controller), the matrix
 * exponential, harmonic-oscillator energy, the PI controller's closed-form
 * fixed point, Hutchinson brute force and finite differences for the adjoint.
 */
#ifndef BATCHODE_ORACLE_H
#define BATCHODE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Methods (paper appendix A: dopri5 in all experiments, tsit5 available). */
#define ORC_DOPRI5 0
#define ORC_TSIT5 1

/* Right-hand sides. */
#define ORC_RHS_VDP 0      /* x' = v, v' = mu (1 - x^2) v - x   (Eq. eq:vdp) */
#define ORC_RHS_LINEAR 1   /* y' = A y, A per instance                      */
#define ORC_RHS_MLP 2      /* y' = MLP([y, t]) with two tanh hidden layers  */
#define ORC_RHS_CNF 3      /* [z, l]' = [g(z,t), -eps^T (dg/dz) eps]        */
#define ORC_RHS_CNF_DIAG 4 /* test only: CNF augmentation of g(z) = lam * z */

/* Per-instance status codes (same numbering as the GPU library's ABI). */
#define ORC_RUNNING 0
#define ORC_SUCCESS 1
#define ORC_MAX_STEPS 2
#define ORC_DT_UNDERFLOW 3
#define ORC_INVALID 4

typedef struct {
  int32_t B;            /* instances                                         */
  int32_t D;            /* row stride of every [B, D] array                  */
  int32_t E;            /* evaluation times per instance                     */
  const int32_t* kind;  /* [B] ORC_RHS_* per instance                        */
  const int32_t* dim;   /* [B] true state dimension of each instance (<= D)  */
  const double* y0;     /* [B, D]                                            */
  const double* t0;     /* [B]                                               */
  const double* t_end;  /* [B]                                               */
  const double* rtol;   /* [B]                                               */
  const double* atol;   /* [B]                                               */
  const double* t_eval; /* [B, E], each row sorted, inside [t0, t_end]       */
  const double* h0;     /* [B] user initial step, or NULL for Hairer's rule  */
  const double* mu;     /* [B] Van der Pol damping                           */
  const double* A;      /* [B, D, D] linear systems, row-major               */
  /* MLP shared by all instances: n0 = n3 + 1 inputs ([y, t] or [z, t]),
   * hidden widths n1, n2 (tanh), n3 outputs.  W_l is [fan_in, fan_out]
   * row-major, so layer l computes out_j = sum_i in_i W_l[i][j] + b_l[j].  */
  int32_t n0, n1, n2, n3;
  const double *W1, *b1, *W2, *b2, *W3, *b3;
  const double* eps;    /* [B, D] Rademacher probes (CNF: first n3 entries)  */
  const double* lam;    /* [B, D] diagonal rates (CNF_DIAG)                  */
} orc_problem;

typedef struct {
  int32_t method;
  /* Step-size controller: on acceptance the next step is scaled by
   * clamp(safety * err^-beta1 * err_prev^beta2 * err_prev2^beta3, fac_min,
   * fac_max), err_prev and err_prev2 the error norms of the last two
   * accepted steps (clamped below at 1e-4, 1 before there were any).
   * beta2 = beta3 = 0 is the integral controller of the benchmarks; beta3
   * is the PID term (set after round_state_f32, below).                    */
  double beta1, beta2, safety, fac_min, fac_max;
  int32_t max_steps;     /* attempted steps per instance                     */
  int32_t n_threads;     /* OpenMP threads (<= 0: library default)           */
  /* Replay: if h_replay != NULL, instance i makes exactly n_replay[i]
   * attempts with sizes |h_replay[i, :]|, no controller deciding: a positive
   * entry is an accepted step, a negative entry a rejected attempt (computed,
   * then discarded).  The last positive entry is the step that ends on t_end.
   * This is the fixed-step mode and the replay of a recorded sequence.     */
  const double* h_replay;
  const int32_t* n_replay;
  int32_t replay_cap;
  /* Optional [B]: 0 marks a record that stopped before t_end (its last
   * accepted step is an ordinary step); NULL means every record ends there. */
  const int32_t* replay_final;
  /* Recording: if h_rec != NULL, the size of every attempted step is written
   * to h_rec[i, n] for n < rec_cap, negated when the attempt was rejected.  */
  double* h_rec;
  int32_t rec_cap;
  /* Replay diagnostics: if err_rec != NULL, the error norm of every replayed
   * attempt is written to err_rec[i, n] (n < replay_cap), computed exactly as
   * an adaptive step computes it, and if hprop_rec != NULL the step size the
   * controller would propose next, given the replayed decisions so far.    */
  double* err_rec;
  double* hprop_rec;
  /* Rounding probe for the tests (not part of the method): when nonzero the
   * state is rounded to the nearest float after every accepted step, which
   * shows how strongly the trajectory amplifies float-sized perturbations
   * made at every step; 2 also rounds every stage input and every stage
   * derivative to float, so each attempt's error norm carries the rounding
   * noise a float datapath puts into it (its distance from the plain
   * replay's norm measures how strongly that noise moves the norm).        */
  int32_t round_state_f32;
  double beta3; /* third controller exponent (PID), see beta1            */
  /* Fixed-step integration (a validation mode; the paper's section 3 names
   * only adaptive controllers): every instance steps with its own h0 (required), every
   * attempt is accepted, the step that would pass t_end ends there.        */
  int32_t fixed_step;
} orc_options;

/* Solves every instance.  Outputs:
 *   y_eval [B, E, D]   solution at t_eval (NaN where never reached)
 *   y_final [B, D]     state at the end (or where the instance stopped)
 *   stats [5, B]       attempted, accepted, rejected, f-evaluations, status
 * Returns 0, or -1 for an invalid problem description.                      */
int orc_solve(const orc_problem* P, const orc_options* O, double* y_eval,
              double* y_final, int32_t* stats);

/* One right-hand-side evaluation f(t, y) for instance i (y, out: [dim]). */
void orc_rhs(const orc_problem* P, int32_t i, double t, const double* y,
             double* out);

/* Discrete adjoint of the solve whose accepted steps are h_steps / n_steps
 * (step sizes and accept decisions frozen).  Given cotangents g_eval [B,E,D]
 * and g_final [B, D] it returns dy0 [B, D] and, for MLP / CNF right-hand
 * sides, dtheta = d/d(W1, b1, W2, b2, W3, b3) flattened in that order and
 * summed over instances (length n0*n1 + n1 + n1*n2 + n2 + n2*n3 + n3).      */
int orc_adjoint(const orc_problem* P, const orc_options* O,
                const double* h_steps, const int32_t* n_steps, int32_t cap,
                const double* g_eval, const double* g_final, double* dy0,
                double* dtheta);

/* mu = J_f(t, y)^T kap for instance i (mu, kap: [dim]); for MLP / CNF
 * right-hand sides (df/dtheta)^T kap is added into dtheta (layout as
 * orc_adjoint's; may be NULL for the analytic fields).                     */
void orc_vjp(const orc_problem* P, int32_t i, double t, const double* y,
             const double* kap, double* mu, double* dtheta);

/* Number of MLP parameters (0 without an MLP). */
long orc_n_params(const orc_problem* P);

/* Tableau export for the tests: c[7], a[7*7] (row-major), b[7], bhat[7].   */
void orc_tableau(int32_t method, double* c, double* a, double* b,
                 double* bhat);

/* Continuous-extension weights w[7] at theta: the dense output is
 * y(t_n + theta h) = y_n + h * sum_j w_j(theta) k_j.                       */
void orc_dense_weights(int32_t method, double theta, double* w);

/* Hairer's starting step for instance i (returns h, adds f-evals to *nfe). */
double orc_initial_step(const orc_problem* P, int32_t i, int32_t* nfe);

/* 1 if instance i passes the input checks of an independent solve.        */
int orc_instance_valid(const orc_problem* P, int32_t i);

/* Joint (coupled) solve of section 4.1: the members (valid instances with
 * the first valid instance's t0, t_end, t_eval and h0) form one system with
 * a single step size, error norm and accept/reject decision (joint.c).
 * Outputs as orc_solve; every member reports the joint counts.  The
 * options' replay and recording fields are not used.                        */
int orc_solve_joint(const orc_problem* P, const orc_options* O,
                    double* y_eval, double* y_final, int32_t* stats);

/* Continuous adjoint (appendix A, the adjoint-equation training of the
 * CNF): the augmented system y' = f, a' = -(df/dy)^T a, g' = -(df/dtheta)^T a
 * integrated adaptively from t_end back to t0 (cadjoint.c), per instance
 * (joint = 0: every instance its own (y, a, g), b (f + p) variables) or
 * jointly (joint = 1: the members' y and a stacked with one shared g, one
 * step size; members are the instances with fwd_status SUCCESS and the first
 * such instance's t0, t_end and t_eval).  y_final [B, D] and fwd_status [B]
 * come from the forward solve; g_eval [B, E, D] (may be NULL when E = 0) and
 * g_final [B, D] are the output cotangents.  Outputs dy0 [B, D] (NaN for
 * instances not differentiated), dtheta [p] (MLP / CNF; the sum over
 * instances) and stats [5, B] of the backward solve (attempted, accepted,
 * rejected, augmented evaluations, status; INVALID for instances not
 * differentiated).  Returns 0, or -1 for invalid arguments.                */
int orc_cadjoint(const orc_problem* P, const orc_options* O, int32_t joint,
                 const double* y_final, const int32_t* fwd_status,
                 const double* g_eval, const double* g_final, double* dy0,
                 double* dtheta, int32_t* stats);

#ifdef __cplusplus
}
#endif
#endif
