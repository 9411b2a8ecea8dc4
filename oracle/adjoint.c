/*
 * Discrete adjoint of the oracle's solve.  TEST INFRASTRUCTURE ONLY.
 *
 * The paper trains its graph model by backpropagation through the solver
 * (section 4.2, discretize-then-optimize).  The oracle differentiates the map
 * from (y0, theta) to the emitted outputs with the accepted step sizes and the
 * accept decisions held fixed: rejected steps and the controller carry no
 * gradient.  For one step of size h from y_n:
 *
 *   Y_1 = y_n,  k_s = f(t_n + c_s h, Y_s),  Y_s = y_n + h sum_{j<s} a_sj k_j,
 *   y_n+1 = Y_7,  dense output y(theta) = y_n + h sum_j w_j(theta) k_j.
 *
 * Walking the stages backwards with cotangents kappa_s on k_s and lambda on
 * y_n+1 gives mu_s = J_f(Y_s)^T kappa_s, kappa_j += h a_sj mu_s (j < s) and
 * lambda_n = lambda_n+1 + sum_s mu_s + sum_e g_e; the parameter gradient
 * collects (df/dtheta)^T kappa_s.  FSAL reuse does not change the map, so
 * stage 1 is simply recomputed.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#include "oracle.h"

typedef struct {
  double *W1, *b1, *W2, *b2, *W3, *b3;
} grads;

static grads split(const orc_problem* P, double* g) {
  grads r;
  r.W1 = g;
  r.b1 = r.W1 + (long)P->n0 * P->n1;
  r.W2 = r.b1 + P->n1;
  r.b2 = r.W2 + (long)P->n1 * P->n2;
  r.W3 = r.b2 + P->n2;
  r.b3 = r.W3 + (long)P->n2 * P->n3;
  return r;
}

static long n_params(const orc_problem* P) {
  return (long)P->n0 * P->n1 + P->n1 + (long)P->n1 * P->n2 + P->n2 +
         (long)P->n2 * P->n3 + P->n3;
}

/* mu = J^T kappa for the MLP at (t, y); accumulates dtheta into G. */
static void vjp_mlp(const orc_problem* P, double t, const double* y,
                    const double* kap, double* mu, grads G) {
  const int n0 = P->n0, n1 = P->n1, n2 = P->n2, n3 = P->n3;
  double x[n0], a1[n1], a2[n2], g1[n1], g2[n2];
  for (int c = 0; c < n3; ++c) x[c] = y[c];
  x[n3] = t;
  for (int j = 0; j < n1; ++j) {
    double acc = P->b1[j];
    for (int i = 0; i < n0; ++i) acc += x[i] * P->W1[(long)i * n1 + j];
    a1[j] = tanh(acc);
  }
  for (int j = 0; j < n2; ++j) {
    double acc = P->b2[j];
    for (int i = 0; i < n1; ++i) acc += a1[i] * P->W2[(long)i * n2 + j];
    a2[j] = tanh(acc);
  }
  /* output layer: out = a2 W3 + b3 */
  for (int i = 0; i < n2; ++i) {
    double acc = 0.0;
    for (int j = 0; j < n3; ++j) {
      G.W3[(long)i * n3 + j] += a2[i] * kap[j];
      acc += P->W3[(long)i * n3 + j] * kap[j];
    }
    g2[i] = (1.0 - a2[i] * a2[i]) * acc; /* cotangent of layer-2 preact */
  }
  for (int j = 0; j < n3; ++j) G.b3[j] += kap[j];
  for (int i = 0; i < n1; ++i) {
    double acc = 0.0;
    for (int j = 0; j < n2; ++j) {
      G.W2[(long)i * n2 + j] += a1[i] * g2[j];
      acc += P->W2[(long)i * n2 + j] * g2[j];
    }
    g1[i] = (1.0 - a1[i] * a1[i]) * acc;
  }
  for (int j = 0; j < n2; ++j) G.b2[j] += g2[j];
  for (int i = 0; i < n0; ++i) {
    double acc = 0.0;
    for (int j = 0; j < n1; ++j) {
      G.W1[(long)i * n1 + j] += x[i] * g1[j];
      acc += P->W1[(long)i * n1 + j] * g1[j];
    }
    if (i < n3) mu[i] = acc; /* the time input carries no state cotangent */
  }
  for (int j = 0; j < n1; ++j) G.b1[j] += g1[j];
}

/* VJP of the CNF field [g(z,t), -eps^T (dg/dz) eps]: reverse mode over the
 * forward-mode tangent computation, second-order tanh terms included.      */
static void vjp_cnf(const orc_problem* P, int32_t inst, double t,
                    const double* y, const double* kap, double* mu, grads G) {
  const int n0 = P->n0, n1 = P->n1, n2 = P->n2, d = P->n3;
  const double* eps = P->eps + (long)inst * P->D;
  double x[n0], a1[n1], a2[n2], da1[n1], da2[n2], dp1[n1], dp2[n2];
  double abar2[n2], dabar2[n2], dpbar2[n2], dabar1[n1], pbar2[n2], abar1[n1],
      dpbar1[n1], pbar1[n1], dgbar[d];
  for (int c = 0; c < d; ++c) x[c] = y[c];
  x[d] = t;
  /* primal and tangent */
  for (int j = 0; j < n1; ++j) {
    double acc = P->b1[j], tac = 0.0;
    for (int i = 0; i < n0; ++i) acc += x[i] * P->W1[(long)i * n1 + j];
    for (int i = 0; i < d; ++i) tac += eps[i] * P->W1[(long)i * n1 + j];
    a1[j] = tanh(acc);
    dp1[j] = tac;
    da1[j] = (1.0 - a1[j] * a1[j]) * tac;
  }
  for (int j = 0; j < n2; ++j) {
    double acc = P->b2[j], tac = 0.0;
    for (int i = 0; i < n1; ++i) {
      acc += a1[i] * P->W2[(long)i * n2 + j];
      tac += da1[i] * P->W2[(long)i * n2 + j];
    }
    a2[j] = tanh(acc);
    dp2[j] = tac;
    da2[j] = (1.0 - a2[j] * a2[j]) * tac;
  }
  /* cotangents: gbar = kappa_z, dgbar = -kappa_l eps */
  const double* gbar = kap;
  for (int j = 0; j < d; ++j) dgbar[j] = -kap[d] * eps[j];
  for (int i = 0; i < n2; ++i) {
    double s1 = 0.0, s2 = 0.0;
    for (int j = 0; j < d; ++j) {
      G.W3[(long)i * d + j] += a2[i] * gbar[j] + da2[i] * dgbar[j];
      s1 += P->W3[(long)i * d + j] * gbar[j];
      s2 += P->W3[(long)i * d + j] * dgbar[j];
    }
    abar2[i] = s1;
    dabar2[i] = s2;
  }
  for (int j = 0; j < d; ++j) G.b3[j] += gbar[j];
  for (int i = 0; i < n2; ++i) {
    const double s = 1.0 - a2[i] * a2[i];
    dpbar2[i] = s * dabar2[i];
    abar2[i] += -2.0 * a2[i] * dp2[i] * dabar2[i];
    pbar2[i] = s * abar2[i];
  }
  for (int i = 0; i < n1; ++i) {
    double s1 = 0.0, s2 = 0.0;
    for (int j = 0; j < n2; ++j) {
      G.W2[(long)i * n2 + j] += da1[i] * dpbar2[j] + a1[i] * pbar2[j];
      s1 += P->W2[(long)i * n2 + j] * dpbar2[j];
      s2 += P->W2[(long)i * n2 + j] * pbar2[j];
    }
    dabar1[i] = s1;
    abar1[i] = s2;
  }
  for (int j = 0; j < n2; ++j) G.b2[j] += pbar2[j];
  for (int i = 0; i < n1; ++i) {
    const double s = 1.0 - a1[i] * a1[i];
    dpbar1[i] = s * dabar1[i];
    abar1[i] += -2.0 * a1[i] * dp1[i] * dabar1[i];
    pbar1[i] = s * abar1[i];
  }
  for (int i = 0; i < n0; ++i) {
    double acc = 0.0;
    for (int j = 0; j < n1; ++j) {
      double gw = x[i] * pbar1[j];
      if (i < d) gw += eps[i] * dpbar1[j];
      G.W1[(long)i * n1 + j] += gw;
      acc += P->W1[(long)i * n1 + j] * pbar1[j];
    }
    if (i < d) mu[i] = acc;
  }
  for (int j = 0; j < n1; ++j) G.b1[j] += pbar1[j];
  mu[d] = 0.0; /* the field does not depend on l */
}

static void vjp(const orc_problem* P, int32_t i, double t, const double* y,
                const double* kap, double* mu, grads G);

void orc_vjp(const orc_problem* P, int32_t i, double t, const double* y,
             const double* kap, double* mu, double* dtheta) {
  double dummy[1] = {0.0};
  vjp(P, i, t, y, kap, mu, split(P, P->W1 ? dtheta : dummy));
}

long orc_n_params(const orc_problem* P) { return P->W1 ? n_params(P) : 0; }

static void vjp(const orc_problem* P, int32_t i, double t, const double* y,
                const double* kap, double* mu, grads G) {
  const int n = P->dim[i];
  switch (P->kind[i]) {
    case ORC_RHS_VDP: {
      const double m = P->mu[i], x = y[0], v = y[1];
      mu[0] = kap[1] * (-2.0 * m * x * v - 1.0);
      mu[1] = kap[0] + kap[1] * m * (1.0 - x * x);
      break;
    }
    case ORC_RHS_LINEAR: {
      const double* A = P->A + (long)i * P->D * P->D;
      for (int c = 0; c < n; ++c) {
        double acc = 0.0;
        for (int r = 0; r < n; ++r) acc += A[(long)r * P->D + c] * kap[r];
        mu[c] = acc;
      }
      break;
    }
    case ORC_RHS_MLP:
      vjp_mlp(P, t, y, kap, mu, G);
      break;
    case ORC_RHS_CNF:
      vjp_cnf(P, i, t, y, kap, mu, G);
      break;
    case ORC_RHS_CNF_DIAG: {
      const double* lam = P->lam + (long)i * P->D;
      for (int c = 0; c < n - 1; ++c) mu[c] = lam[c] * kap[c];
      mu[n - 1] = 0.0;
      break;
    }
    default:
      for (int c = 0; c < n; ++c) mu[c] = NAN;
  }
}

static void adjoint_one(const orc_problem* P, const orc_options* O, int32_t i,
                        const double* h_steps, const int32_t* n_steps,
                        int32_t cap, const double* g_eval,
                        const double* g_final, double* dy0, grads G) {
  const long D = P->D, E = P->E;
  const int n = P->dim[i], N = n_steps[i];
  const double* hs = h_steps + (long)i * cap;
  const double* teval = P->t_eval + (long)i * E;
  double c[7], a[7][7], b[7], bh[7];
  orc_tableau(O->method, c, &a[0][0], b, bh);

  /* frozen forward: t_n and y_n for n = 0..N */
  double* tn = malloc(sizeof(double) * (N + 1));
  double* yn = malloc(sizeof(double) * (long)(N + 1) * n);
  double* work = malloc(sizeof(double) * 18 * n);
  double* Y = work;
  double* k[7];
  double* Ys[7];
  for (int j = 0; j < 7; ++j) k[j] = work + (1 + j) * n;
  for (int j = 0; j < 7; ++j) Ys[j] = work + (8 + j) * n;
  double* lam = work + 15 * n;
  double* mu = work + 16 * n;
  double* lamn = work + 17 * n;
  double* kap = malloc(sizeof(double) * 7 * n);

  tn[0] = P->t0[i];
  for (int q = 0; q < n; ++q) yn[q] = P->y0[(long)i * D + q];
  for (int s = 0; s < N; ++s) {
    const double t = tn[s], h = hs[s];
    const double* y = yn + (long)s * n;
    orc_rhs(P, i, t, y, k[0]);
    for (int st = 1; st < 7; ++st) {
      for (int q = 0; q < n; ++q) {
        double acc = 0.0;
        for (int j = 0; j < st; ++j) acc += a[st][j] * k[j][q];
        Y[q] = y[q] + h * acc;
      }
      orc_rhs(P, i, t + c[st] * h, Y, k[st]);
    }
    for (int q = 0; q < n; ++q) yn[(long)(s + 1) * n + q] = Y[q];
    tn[s + 1] = (s == N - 1) ? P->t_end[i] : t + h;
  }

  /* owner step of each evaluation time (-1: answered by y0 at t0) */
  int* owner = malloc(sizeof(int) * (E > 0 ? E : 1));
  {
    int cursor = 0;
    while (cursor < E && teval[cursor] <= tn[0]) owner[cursor++] = -1;
    for (int s = 0; s < N; ++s)
      while (cursor < E && teval[cursor] <= tn[s + 1]) owner[cursor++] = s;
    while (cursor < E) owner[cursor++] = N; /* never reached */
  }

  for (int q = 0; q < n; ++q) lam[q] = g_final[(long)i * D + q];
  for (int s = N - 1; s >= 0; --s) {
    const double t = tn[s], h = hs[s];
    const double* y = yn + (long)s * n;
    /* recompute the stages of step s */
    for (int q = 0; q < n; ++q) Ys[0][q] = y[q];
    orc_rhs(P, i, t, Ys[0], k[0]);
    for (int st = 1; st < 7; ++st) {
      for (int q = 0; q < n; ++q) {
        double acc = 0.0;
        for (int j = 0; j < st; ++j) acc += a[st][j] * k[j][q];
        Ys[st][q] = y[q] + h * acc;
      }
      orc_rhs(P, i, t + c[st] * h, Ys[st], k[st]);
    }
    memset(kap, 0, sizeof(double) * 7 * n);
    for (int q = 0; q < n; ++q) lamn[q] = 0.0;
    /* dense outputs owned by this step */
    for (int e = 0; e < E; ++e) {
      if (owner[e] != s) continue;
      double w[7];
      orc_dense_weights(O->method, (teval[e] - t) / h, w);
      const double* g = g_eval + ((long)i * E + e) * D;
      for (int j = 0; j < 7; ++j)
        for (int q = 0; q < n; ++q) kap[j * n + q] += h * w[j] * g[q];
      for (int q = 0; q < n; ++q) lamn[q] += g[q];
    }
    /* stage 7 feeds only the dense output; Y_7 = y_n+1 */
    vjp(P, i, t + c[6] * h, Ys[6], kap + 6 * n, mu, G);
    for (int q = 0; q < n; ++q) lam[q] += mu[q];
    for (int j = 0; j < 6; ++j)
      for (int q = 0; q < n; ++q) kap[j * n + q] += h * a[6][j] * lam[q];
    for (int q = 0; q < n; ++q) lamn[q] += lam[q];
    for (int st = 5; st >= 0; --st) {
      vjp(P, i, t + c[st] * h, Ys[st], kap + st * n, mu, G);
      for (int j = 0; j < st; ++j)
        for (int q = 0; q < n; ++q) kap[j * n + q] += h * a[st][j] * mu[q];
      for (int q = 0; q < n; ++q) lamn[q] += mu[q];
    }
    for (int q = 0; q < n; ++q) lam[q] = lamn[q];
  }
  for (int e = 0; e < E; ++e)
    if (owner[e] == -1)
      for (int q = 0; q < n; ++q) lam[q] += g_eval[((long)i * E + e) * D + q];
  for (int q = 0; q < D; ++q) dy0[(long)i * D + q] = (q < n) ? lam[q] : 0.0;
  free(tn);
  free(yn);
  free(work);
  free(kap);
  free(owner);
}

int orc_adjoint(const orc_problem* P, const orc_options* O,
                const double* h_steps, const int32_t* n_steps, int32_t cap,
                const double* g_eval, const double* g_final, double* dy0,
                double* dtheta) {
  if (!P || !O || !h_steps || !n_steps || !g_final || !dy0) return -1;
  if (P->E > 0 && !g_eval) return -1;
  const long np = (P->W1 ? n_params(P) : 0);
  const int nt = O->n_threads > 0 ? O->n_threads : omp_get_max_threads();
  double* part = calloc((size_t)(np > 0 ? np : 1) * nt, sizeof(double));
  /* contiguous blocks of instances per thread, partial sums added in thread
   * order: the same sum order on every run with the same thread count */
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int32_t i = 0; i < P->B; ++i) {
    grads G = split(P, part + (long)omp_get_thread_num() * (np > 0 ? np : 1));
    adjoint_one(P, O, i, h_steps, n_steps, cap, g_eval, g_final, dy0, G);
  }
  if (dtheta && np > 0) {
    for (long q = 0; q < np; ++q) {
      double acc = 0.0;
      for (int th = 0; th < nt; ++th) acc += part[(long)th * np + q];
      dtheta[q] = acc;
    }
  }
  free(part);
  return 0;
}
