/*
 * Right-hand sides of the oracle, in plain FP64 loops.  TEST INFRASTRUCTURE
 * ONLY.
 *
 *  - Van der Pol (section 4.1, Eq. eq:vdp): x'' = mu (1 - x^2) x' - x, written
 *    as the first-order system x' = v, v' = mu (1 - x^2) v - x.
 *  - Linear y' = A y (the closed-form test family).
 *  - A neural right-hand side MLP([y, t]) with two tanh hidden layers and a
 *    linear output, the shape of learned dynamics the paper benchmarks
 *    (appendix A: FEN and FFJORD models are learned vector fields).
 *  - A continuous normalising flow (appendix A, FFJORD on MNIST): the state is
 *    [z, l] with z' = g(z, t) and l' = -eps^T (dg/dz) eps, the one-sample
 *    Hutchinson estimate of -trace(dg/dz).  The Jacobian-vector product is
 *    taken in forward mode, layer by layer.
 *  - CNF_DIAG (tests only): the same augmentation for g(z) = lam * z, whose
 *    log-density change has a closed form.
 */
#include <math.h>
#include <string.h>

#include "oracle.h"

/* out = [tanh](in W + b) for a layer with n_in inputs and n_out outputs. */
static void dense(const double* in, int n_in, const double* W, const double* b,
                  int n_out, int apply_tanh, double* out) {
  for (int j = 0; j < n_out; ++j) {
    double acc = b[j];
    for (int i = 0; i < n_in; ++i) acc += in[i] * W[(long)i * n_out + j];
    out[j] = apply_tanh ? tanh(acc) : acc;
  }
}

/* y' = MLP([y, t]) for the n3-dimensional state y. */
static void mlp(const orc_problem* P, double t, const double* y, double* out) {
  const int n3 = P->n3;
  double x[P->n0], a1[P->n1], a2[P->n2];
  for (int c = 0; c < n3; ++c) x[c] = y[c];
  x[n3] = t;
  dense(x, P->n0, P->W1, P->b1, P->n1, 1, a1);
  dense(a1, P->n1, P->W2, P->b2, P->n2, 1, a2);
  dense(a2, P->n2, P->W3, P->b3, n3, 0, out);
}

/* [z, l]' = [g(z, t), -eps^T J eps] with J = dg/dz, via forward mode. */
static void cnf(const orc_problem* P, int32_t i, double t, const double* y,
                double* out) {
  const int d = P->n3;
  double x[P->n0], a1[P->n1], a2[P->n2], dx[P->n0], da1[P->n1], da2[P->n2],
      dg[d];
  const double* eps = P->eps + (long)i * P->D;
  for (int c = 0; c < d; ++c) {
    x[c] = y[c];
    dx[c] = eps[c];
  }
  x[d] = t;
  dx[d] = 0.0; /* the probe does not move time */
  dense(x, P->n0, P->W1, P->b1, P->n1, 1, a1);
  /* tangent of layer 1: (1 - a1^2) * (dx W1) */
  for (int j = 0; j < P->n1; ++j) {
    double acc = 0.0;
    for (int k = 0; k < P->n0; ++k) acc += dx[k] * P->W1[(long)k * P->n1 + j];
    da1[j] = (1.0 - a1[j] * a1[j]) * acc;
  }
  dense(a1, P->n1, P->W2, P->b2, P->n2, 1, a2);
  for (int j = 0; j < P->n2; ++j) {
    double acc = 0.0;
    for (int k = 0; k < P->n1; ++k) acc += da1[k] * P->W2[(long)k * P->n2 + j];
    da2[j] = (1.0 - a2[j] * a2[j]) * acc;
  }
  dense(a2, P->n2, P->W3, P->b3, d, 0, out);
  for (int j = 0; j < d; ++j) {
    double acc = 0.0;
    for (int k = 0; k < P->n2; ++k) acc += da2[k] * P->W3[(long)k * d + j];
    dg[j] = acc;
  }
  double q = 0.0;
  for (int j = 0; j < d; ++j) q += eps[j] * dg[j];
  out[d] = -q;
}

void orc_rhs(const orc_problem* P, int32_t i, double t, const double* y,
             double* out) {
  const int kind = P->kind[i];
  const int n = P->dim[i];
  switch (kind) {
    case ORC_RHS_VDP: {
      const double mu = P->mu[i];
      const double x = y[0], v = y[1];
      out[0] = v;
      out[1] = mu * (1.0 - x * x) * v - x;
      break;
    }
    case ORC_RHS_LINEAR: {
      const double* A = P->A + (long)i * P->D * P->D;
      for (int r = 0; r < n; ++r) {
        double acc = 0.0;
        for (int c = 0; c < n; ++c) acc += A[(long)r * P->D + c] * y[c];
        out[r] = acc;
      }
      break;
    }
    case ORC_RHS_MLP:
      mlp(P, t, y, out);
      break;
    case ORC_RHS_CNF:
      cnf(P, i, t, y, out);
      break;
    case ORC_RHS_CNF_DIAG: {
      const double* lam = P->lam + (long)i * P->D;
      const double* eps = P->eps + (long)i * P->D;
      double q = 0.0;
      for (int c = 0; c < n - 1; ++c) {
        out[c] = lam[c] * y[c];
        q += eps[c] * lam[c] * eps[c];
      }
      out[n - 1] = -q;
      break;
    }
    default:
      for (int c = 0; c < n; ++c) out[c] = NAN;
  }
}
