/*
 * Continuous adjoint (optimize-then-discretize) of the oracle's solve.
 * TEST INFRASTRUCTURE ONLY.
 *
 * Appendix A (the CNF benchmark) trains through the adjoint equation: after
 * the forward solve, an augmented system is integrated backwards in time from
 * t_end to t0,
 *
 *   y' = f(t, y),   a' = -(df/dy)^T a,   g' = -(df/dtheta)^T a,
 *
 * from y(t_end) (the forward solution), a(t_end) = the cotangent of
 * y(t_end) and g(t_end) = 0; then a(t0) is the gradient with respect to y0
 * and g(t0) the gradient with respect to theta.  A cotangent on the output at
 * an evaluation time t_e is added to a when the backward solve reaches t_e
 * (the solve stops exactly there).
 *
 * The appendix contrasts two ways to batch this system:
 *
 *  - per instance (the default of the paper's library): every instance i
 *    integrates its own augmented state (y_i, a_i, g_i) of size 2 n + p with
 *    its own step size, error norm and accept/reject decision, so the batch
 *    carries b (f + p) variables;
 *  - joint: the instances' y and a are stacked with one shared g into a
 *    single system of size 2 b f + p (b f + p in the appendix's count, which
 *    leaves out the re-integrated y), solved with one step size.
 *
 * Both use the forward solve's method, controller and tolerances: each
 * component is scaled by atol + rtol max(|z_n|, |z_n+1|) with its instance's
 * tolerances (the shared g of the joint system takes the first member's),
 * the error norm is the RMS over all components of the (per-instance or
 * joint) augmented state, the start step is Hairer's rule on that state over
 * the whole span, the step is clipped to land on every evaluation time and
 * on t0, and the controller continues across those stops.  The parameter
 * gradient returned is the sum of the g_i (per instance) or the shared g.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#include "oracle.h"

static double clampc(double x, double lo, double hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}

/* The augmented system of a set of members: z = [y_m, a_m for each member,
 * then g] (g shared), component scales from per-component tolerances.     */
typedef struct {
  const orc_problem* P;
  int32_t nm;           /* members */
  const int32_t* mem;   /* [nm] instance indices */
  const long* off;      /* [nm] offset of y_m in z (a_m follows at +n_m) */
  long p;               /* parameters (g length) */
  long N;               /* total length */
  double* atol;         /* [N] */
  double* rtol;         /* [N] */
  double* mu;           /* scratch [max n] */
} aug_sys;

/* F(t, z) = [f(t, y_m), -(df/dy)^T a_m for each member, -sum_m (df/dtheta)^T
 * a_m]. */
static void aug_rhs(const aug_sys* S, double t, const double* z, double* F) {
  const orc_problem* P = S->P;
  double* g = F + (S->N - S->p);
  for (long q = 0; q < S->p; ++q) g[q] = 0.0;
  for (int32_t m = 0; m < S->nm; ++m) {
    const int32_t i = S->mem[m];
    const int n = P->dim[i];
    const double* y = z + S->off[m];
    const double* a = y + n;
    orc_rhs(P, i, t, y, F + S->off[m]);
    orc_vjp(P, i, t, y, a, S->mu, S->p > 0 ? g : NULL);
    for (int q = 0; q < n; ++q) F[S->off[m] + n + q] = -S->mu[q];
  }
  for (long q = 0; q < S->p; ++q) g[q] = -g[q];
}

/* Cotangents of the evaluation times equal to t, added to the members' a. */
static void add_jumps(const aug_sys* S, double t, const double* g_eval,
                      double* z) {
  const orc_problem* P = S->P;
  for (int32_t m = 0; m < S->nm; ++m) {
    const int32_t i = S->mem[m];
    const int n = P->dim[i];
    for (int e = 0; e < P->E; ++e)
      if (P->t_eval[(long)i * P->E + e] == t)
        for (int q = 0; q < n; ++q)
          z[S->off[m] + n + q] += g_eval[((long)i * P->E + e) * P->D + q];
  }
}

/* Integrates S backwards from t_end to t0 (t_end > t0) in place.  stops:
 * the distinct evaluation times strictly inside (t0, t_end), descending.
 * stats: attempted, accepted, rejected, augmented evaluations, status.      */
static void backward_solve(const orc_options* O, const aug_sys* S, double* z,
                           double t_end, double t0, const double* stops,
                           int n_stops, const double* g_eval, int32_t* st) {
  const long N = S->N;
  double c[7], a[7][7], b[7], bh[7], e[7];
  orc_tableau(O->method, c, &a[0][0], b, bh);
  for (int j = 0; j < 7; ++j) e[j] = b[j] - bh[j];
  double* buf = malloc(sizeof(double) * 9 * N);
  double* k[7];
  for (int j = 0; j < 7; ++j) k[j] = buf + j * N;
  double* Z = buf + 7 * N;
  double* Y1 = buf + 8 * N;
  int32_t natt = 0, nacc = 0, nrej = 0, nfe = 0, status = ORC_RUNNING;
  double t = t_end;
  aug_rhs(S, t, z, k[0]);
  nfe = 1;
  /* Hairer's rule on the augmented state, backwards (h < 0) */
  double h;
  {
    const double span = t_end - t0;
    double s0 = 0.0, s1 = 0.0;
    for (long q = 0; q < N; ++q) {
      const double sc = S->atol[q] + fabs(z[q]) * S->rtol[q];
      s0 += (z[q] / sc) * (z[q] / sc);
      s1 += (k[0][q] / sc) * (k[0][q] / sc);
    }
    const double d0 = sqrt(s0 / N), d1 = sqrt(s1 / N);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    h0 = fmin(h0, span);
    for (long q = 0; q < N; ++q) Y1[q] = z[q] - h0 * k[0][q];
    aug_rhs(S, t - h0, Y1, k[1]);
    nfe += 1;
    double s2 = 0.0;
    for (long q = 0; q < N; ++q) {
      const double sc = S->atol[q] + fabs(z[q]) * S->rtol[q];
      const double d = (k[1][q] - k[0][q]) / sc;
      s2 += d * d;
    }
    const double d2 = sqrt(s2 / N) / h0;
    const double h1 = (d1 <= 1e-15 && d2 <= 1e-15)
                          ? fmax(1e-6, h0 * 1e-3)
                          : pow(0.01 / fmax(d1, d2), 1.0 / 5.0);
    h = -fmin(fmin(100.0 * h0, h1), span);
  }
  int next = 0; /* next stop */
  double err_prev = 1.0, err_prev2 = 1.0;
  int prev_rejected = 0;
  while (status == ORC_RUNNING) {
    if (natt >= O->max_steps) {
      status = ORC_MAX_STEPS;
      break;
    }
    const double target = next < n_stops ? stops[next] : t0;
    const int last = (t + h <= target);
    const double hs = last ? target - t : h;
    for (int s = 1; s < 7; ++s) {
      for (long q = 0; q < N; ++q) {
        double acc = 0.0;
        for (int j = 0; j < s; ++j) acc += a[s][j] * k[j][q];
        Z[q] = z[q] + hs * acc;
      }
      aug_rhs(S, t + c[s] * hs, Z, k[s]);
    }
    nfe += 6;
    natt += 1;
    double acc = 0.0;
    for (long q = 0; q < N; ++q) {
      double eq = 0.0;
      for (int j = 0; j < 7; ++j) eq += e[j] * k[j][q];
      eq *= hs;
      const double sc = S->atol[q] + S->rtol[q] * fmax(fabs(z[q]), fabs(Z[q]));
      acc += (eq / sc) * (eq / sc);
    }
    const double err = sqrt(acc / N);
    const int accept = err < 1.0;
    double fac;
    if (!isfinite(err))
      fac = O->fac_min;
    else if (accept) {
      if (err == 0.0)
        fac = O->fac_max;
      else
        fac = clampc(O->safety * pow(err, -O->beta1) *
                         pow(err_prev, O->beta2) * pow(err_prev2, O->beta3),
                     O->fac_min, O->fac_max);
      if (prev_rejected) fac = fmin(1.0, fac);
    } else {
      fac = fmax(O->fac_min, O->safety * pow(err, -1.0 / 5.0));
    }
    if (accept) {
      t = last ? target : t + hs;
      memcpy(z, Z, sizeof(double) * N);
      memcpy(k[0], k[6], sizeof(double) * N); /* FSAL */
      err_prev2 = err_prev;
      err_prev = fmax(err, 1e-4);
      nacc += 1;
      prev_rejected = 0;
      if (last) {
        if (next < n_stops) {
          /* an evaluation time: its cotangent enters a, which changes the
           * augmented right-hand side at t (the FSAL stage is refreshed) */
          add_jumps(S, t, g_eval, z);
          aug_rhs(S, t, z, k[0]);
          nfe += 1;
          ++next;
        } else {
          status = ORC_SUCCESS;
        }
      }
    } else {
      nrej += 1;
      prev_rejected = 1;
    }
    h = hs * fac;
    if (status == ORC_RUNNING && !(fabs(h) > 16.0 * DBL_EPSILON * fabs(t)))
      status = ORC_DT_UNDERFLOW;
  }
  st[0] = natt;
  st[1] = nacc;
  st[2] = nrej;
  st[3] = nfe;
  st[4] = status;
  free(buf);
}

/* Distinct evaluation times of instance i strictly inside (t0, t_end),
 * descending; returns their count. */
static int stop_list(const orc_problem* P, int32_t i, double* stops) {
  int n = 0;
  const double t0 = P->t0[i], te = P->t_end[i];
  for (int e = P->E - 1; e >= 0; --e) {
    const double v = P->t_eval[(long)i * P->E + e];
    if (v > t0 && v < te && (n == 0 || stops[n - 1] != v)) stops[n++] = v;
  }
  return n;
}

/* Sets up the member list's augmented state: y from y_final, a from the
 * cotangents of y(t_end) (final and evaluation times equal to t_end). */
static void init_state(const aug_sys* S, const double* y_final,
                       const double* g_eval, const double* g_final,
                       double* z) {
  const orc_problem* P = S->P;
  memset(z, 0, sizeof(double) * S->N);
  for (int32_t m = 0; m < S->nm; ++m) {
    const int32_t i = S->mem[m];
    const int n = P->dim[i];
    for (int q = 0; q < n; ++q) {
      z[S->off[m] + q] = y_final[(long)i * P->D + q];
      z[S->off[m] + n + q] = g_final[(long)i * P->D + q];
    }
  }
  const int32_t r = S->mem[0];
  add_jumps(S, P->t_end[r], g_eval, z);
}

/* dy0 for the members from their a(t0), plus the cotangents at t0. */
static void finish_state(const aug_sys* S, const double* g_eval,
                         const double* z, double* dy0) {
  const orc_problem* P = S->P;
  double* tmp = malloc(sizeof(double) * S->N);
  memcpy(tmp, z, sizeof(double) * S->N);
  const int32_t r = S->mem[0];
  if (P->t0[r] < P->t_end[r]) add_jumps(S, P->t0[r], g_eval, tmp);
  for (int32_t m = 0; m < S->nm; ++m) {
    const int32_t i = S->mem[m];
    const int n = P->dim[i];
    for (int q = 0; q < P->D; ++q)
      dy0[(long)i * P->D + q] = q < n ? tmp[S->off[m] + n + q] : 0.0;
  }
  free(tmp);
}

static int same_span(const orc_problem* P, int32_t i, int32_t r) {
  if (P->t0[i] != P->t0[r] || P->t_end[i] != P->t_end[r]) return 0;
  for (int e = 0; e < P->E; ++e)
    if (P->t_eval[(long)i * P->E + e] != P->t_eval[(long)r * P->E + e])
      return 0;
  return 1;
}

int orc_cadjoint(const orc_problem* P, const orc_options* O, int32_t joint,
                 const double* y_final, const int32_t* fwd_status,
                 const double* g_eval, const double* g_final, double* dy0,
                 double* dtheta, int32_t* stats) {
  if (!P || !O || !y_final || !fwd_status || !g_final || !dy0 || !stats)
    return -1;
  if (P->E > 0 && (!g_eval || !P->t_eval)) return -1;
  if (O->method != ORC_DOPRI5 && O->method != ORC_TSIT5) return -1;
  const long B = P->B, D = P->D, p = orc_n_params(P);
  if (p > 0 && !dtheta) return -1;
  for (long q = 0; q < B * D; ++q) dy0[q] = NAN;
  for (long q = 0; q < 5 * B; ++q) stats[q] = 0;
  for (long i = 0; i < B; ++i) stats[4 * B + i] = ORC_INVALID;
  for (long q = 0; q < p; ++q) dtheta[q] = 0.0;
  int maxn = 1;
  for (long i = 0; i < B; ++i) maxn = P->dim[i] > maxn ? P->dim[i] : maxn;

  if (joint) {
    int32_t* mem = malloc(sizeof(int32_t) * (B > 0 ? B : 1));
    long* off = malloc(sizeof(long) * (B > 0 ? B : 1));
    int32_t nm = 0;
    long N = 0;
    for (int32_t i = 0; i < B; ++i) {
      if (fwd_status[i] != ORC_SUCCESS) continue;
      if (nm > 0 && !same_span(P, i, mem[0])) continue;
      mem[nm] = i;
      off[nm++] = N;
      N += 2L * P->dim[i];
    }
    if (nm > 0) {
      aug_sys S = {P, nm, mem, off, p, N + p, NULL, NULL, NULL};
      S.atol = malloc(sizeof(double) * S.N);
      S.rtol = malloc(sizeof(double) * S.N);
      S.mu = malloc(sizeof(double) * maxn);
      for (int32_t m = 0; m < nm; ++m)
        for (long q = 0; q < 2L * P->dim[mem[m]]; ++q) {
          S.atol[off[m] + q] = P->atol[mem[m]];
          S.rtol[off[m] + q] = P->rtol[mem[m]];
        }
      for (long q = 0; q < p; ++q) {
        S.atol[N + q] = P->atol[mem[0]];
        S.rtol[N + q] = P->rtol[mem[0]];
      }
      double* z = malloc(sizeof(double) * S.N);
      double* stops = malloc(sizeof(double) * (P->E + 1));
      const int32_t r = mem[0];
      const int ns = stop_list(P, r, stops);
      init_state(&S, y_final, g_eval, g_final, z);
      int32_t st[5] = {0, 0, 0, 0, ORC_SUCCESS};
      if (P->t_end[r] > P->t0[r])
        backward_solve(O, &S, z, P->t_end[r], P->t0[r], stops, ns, g_eval,
                       st);
      finish_state(&S, g_eval, z, dy0);
      for (long q = 0; q < p; ++q) dtheta[q] = z[N + q];
      for (int32_t m = 0; m < nm; ++m)
        for (int f = 0; f < 5; ++f) stats[f * B + mem[m]] = st[f];
      free(z);
      free(stops);
      free(S.atol);
      free(S.rtol);
      free(S.mu);
    }
    free(mem);
    free(off);
    return 0;
  }

  const int nt = O->n_threads > 0 ? O->n_threads : omp_get_max_threads();
  double* part = calloc((size_t)(p > 0 ? p : 1) * nt, sizeof(double));
  /* contiguous blocks of instances per thread, partial sums added in thread
   * order: the same sum order on every run with the same thread count */
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int32_t i = 0; i < B; ++i) {
    if (fwd_status[i] != ORC_SUCCESS) continue;
    const int n = P->dim[i];
    int32_t mem[1] = {i};
    long off[1] = {0};
    aug_sys S = {P, 1, mem, off, p, 2L * n + p, NULL, NULL, NULL};
    S.atol = malloc(sizeof(double) * S.N);
    S.rtol = malloc(sizeof(double) * S.N);
    S.mu = malloc(sizeof(double) * maxn);
    for (long q = 0; q < S.N; ++q) {
      S.atol[q] = P->atol[i];
      S.rtol[q] = P->rtol[i];
    }
    double* z = malloc(sizeof(double) * S.N);
    double* stops = malloc(sizeof(double) * (P->E + 1));
    const int ns = stop_list(P, i, stops);
    init_state(&S, y_final, g_eval, g_final, z);
    int32_t st[5] = {0, 0, 0, 0, ORC_SUCCESS};
    if (P->t_end[i] > P->t0[i])
      backward_solve(O, &S, z, P->t_end[i], P->t0[i], stops, ns, g_eval, st);
    finish_state(&S, g_eval, z, dy0);
    double* acc = part + (long)omp_get_thread_num() * (p > 0 ? p : 1);
    for (long q = 0; q < p; ++q) acc[q] += z[2L * n + q];
    for (int f = 0; f < 5; ++f) stats[f * B + i] = st[f];
    free(z);
    free(stops);
    free(S.atol);
    free(S.rtol);
    free(S.mu);
  }
  for (long q = 0; q < p; ++q) {
    double acc = 0.0;
    for (int th = 0; th < nt; ++th) acc += part[(long)th * p + q];
    dtheta[q] = acc;
  }
  free(part);
  return 0;
}
