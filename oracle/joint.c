/*
 * Joint (coupled) batch solving: the comparison mode of paper section 4.1.
 * TEST INFRASTRUCTURE ONLY.
 *
 * Section 4.1 describes how other libraries batch: the n instances of size p
 * are concatenated into one problem of size n p and solved as one system,
 * so they share the step size and the error estimate, and a step is accepted
 * or rejected for all of them at once.  The oracle does exactly that:
 *
 *  - one time t, one step size h, one controller history;
 *  - the error norm is the weighted RMS over every component of every
 *    instance in the system, each component scaled by its own instance's
 *    atol + rtol max(|y_n|, |y_n+1|) (the per-instance norm of the
 *    independent solve, extended to the stacked vector);
 *  - the start step is Hairer's rule on the stacked vector (or h0 of the
 *    first member);
 *  - the controller, the end clip and the evaluation-time ownership are
 *    those of the independent solve (solve.c).
 *
 * Members are the valid instances whose t0, t_end and evaluation times equal
 * those of the first valid instance; every other instance is INVALID.  Every
 * member reports the joint step counts; its f-evaluation count is its own
 * (1 + start-step probe + 6 per attempted step).
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static double clampj(double x, double lo, double hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}

static int same_span(const orc_problem* P, int32_t i, int32_t r) {
  if (P->t0[i] != P->t0[r] || P->t_end[i] != P->t_end[r]) return 0;
  for (int e = 0; e < P->E; ++e)
    if (P->t_eval[(long)i * P->E + e] != P->t_eval[(long)r * P->E + e])
      return 0;
  if (P->h0 && P->h0[i] != P->h0[r]) return 0;
  return 1;
}

int orc_solve_joint(const orc_problem* P, const orc_options* O,
                    double* y_eval, double* y_final, int32_t* stats) {
  if (!P || !O || P->B < 0 || P->D < 1 || P->E < 0 || !y_final || !stats)
    return -1;
  if (P->E > 0 && (!y_eval || !P->t_eval)) return -1;
  if (O->method != ORC_DOPRI5 && O->method != ORC_TSIT5) return -1;
  const long B = P->B, D = P->D, E = P->E;
  double c[7], a[7][7], b[7], bh[7], e[7];
  orc_tableau(O->method, c, &a[0][0], b, bh);
  for (int j = 0; j < 7; ++j) e[j] = b[j] - bh[j];

  /* members and their offsets in the stacked vector */
  int32_t* off = malloc(sizeof(int32_t) * (B + 1));
  int32_t ref = -1;
  long N = 0;
  for (int32_t i = 0; i < B; ++i) {
    int member = orc_instance_valid(P, i);
    if (member && ref < 0) ref = i;
    if (member && !same_span(P, i, ref)) member = 0;
    off[i] = member ? (int32_t)N : -1;
    if (member) N += P->dim[i];
  }
  for (long q = 0; q < B * E * D; ++q) y_eval[q] = NAN;
  for (long q = 0; q < B * D; ++q) y_final[q] = NAN;
  for (int32_t i = 0; i < B; ++i) {
    const int n = P->dim[i];
    for (long x = 0; x < E; ++x)
      for (long q = 0; q < D; ++q)
        if (q >= n) y_eval[(i * E + x) * D + q] = 0.0;
    for (long q = 0; q < D; ++q)
      if (q >= n) y_final[i * D + q] = 0.0;
  }
  int32_t natt = 0, nacc = 0, nrej = 0, nfe = 0, status = ORC_INVALID;
  if (ref >= 0) {
    status = ORC_RUNNING;
    double* buf = malloc(sizeof(double) * 10 * N);
    double* y = buf;
    double* Y = buf + N;
    double* k[7];
    for (int j = 0; j < 7; ++j) k[j] = buf + (2 + j) * N;
    double* ynew = buf + 9 * N;
    double t = P->t0[ref];
    const double te = P->t_end[ref];
    const double* teval = P->t_eval + (long)ref * E;
    for (int32_t i = 0; i < B; ++i)
      if (off[i] >= 0) {
        memcpy(y + off[i], P->y0 + i * D, sizeof(double) * P->dim[i]);
        orc_rhs(P, i, t, y + off[i], k[0] + off[i]);
      }
    nfe = 1;
    int cursor = 0;
    while (cursor < E && teval[cursor] <= t) {
      for (int32_t i = 0; i < B; ++i)
        if (off[i] >= 0)
          for (int q = 0; q < P->dim[i]; ++q)
            y_eval[(i * E + cursor) * D + q] = y[off[i] + q];
      ++cursor;
    }
    double h = 0.0;
    if (te == t) {
      status = ORC_SUCCESS;
    } else if (P->h0) {
      h = P->h0[ref];
    } else { /* Hairer's rule on the stacked vector */
      const double span = te - t;
      double s0 = 0.0, s1 = 0.0;
      for (int32_t i = 0; i < B; ++i)
        for (int q = 0; off[i] >= 0 && q < P->dim[i]; ++q) {
          const double sc = P->atol[i] + fabs(y[off[i] + q]) * P->rtol[i];
          s0 += (y[off[i] + q] / sc) * (y[off[i] + q] / sc);
          s1 += (k[0][off[i] + q] / sc) * (k[0][off[i] + q] / sc);
        }
      const double d0 = sqrt(s0 / N), d1 = sqrt(s1 / N);
      double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
      h0 = fmin(h0, span);
      for (long q = 0; q < N; ++q) Y[q] = y[q] + h0 * k[0][q];
      for (int32_t i = 0; i < B; ++i)
        if (off[i] >= 0) orc_rhs(P, i, t + h0, Y + off[i], k[1] + off[i]);
      nfe += 1;
      double s2 = 0.0;
      for (int32_t i = 0; i < B; ++i)
        for (int q = 0; off[i] >= 0 && q < P->dim[i]; ++q) {
          const double sc = P->atol[i] + fabs(y[off[i] + q]) * P->rtol[i];
          const double d = (k[1][off[i] + q] - k[0][off[i] + q]) / sc;
          s2 += d * d;
        }
      const double d2 = sqrt(s2 / N) / h0;
      const double h1 = (d1 <= 1e-15 && d2 <= 1e-15)
                            ? fmax(1e-6, h0 * 1e-3)
                            : pow(0.01 / fmax(d1, d2), 1.0 / 5.0);
      h = fmin(fmin(100.0 * h0, h1), span);
    }
    double err_prev = 1.0, err_prev2 = 1.0;
    int prev_rejected = 0;
    while (status == ORC_RUNNING) {
      if (natt >= O->max_steps) {
        status = ORC_MAX_STEPS;
        break;
      }
      const int last = (t + h >= te);
      const double hs = last ? te - t : h;
      for (int s = 1; s < 7; ++s)
        for (int32_t i = 0; i < B; ++i) {
          if (off[i] < 0) continue;
          const int n = P->dim[i];
          double* Yi = Y + off[i];
          for (int q = 0; q < n; ++q) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += a[s][j] * k[j][off[i] + q];
            Yi[q] = y[off[i] + q] + hs * acc;
          }
          orc_rhs(P, i, t + c[s] * hs, Yi, k[s] + off[i]);
        }
      memcpy(ynew, Y, sizeof(double) * N);
      nfe += 6;
      natt += 1;
      double acc = 0.0;
      for (int32_t i = 0; i < B; ++i)
        for (int q = 0; off[i] >= 0 && q < P->dim[i]; ++q) {
          const long x = off[i] + q;
          double eq = 0.0;
          for (int j = 0; j < 7; ++j) eq += e[j] * k[j][x];
          eq *= hs;
          const double sc =
              P->atol[i] + P->rtol[i] * fmax(fabs(y[x]), fabs(ynew[x]));
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
          fac = clampj(O->safety * pow(err, -O->beta1) *
                           pow(err_prev, O->beta2) * pow(err_prev2, O->beta3),
                       O->fac_min, O->fac_max);
        if (prev_rejected) fac = fmin(1.0, fac);
      } else {
        fac = fmax(O->fac_min, O->safety * pow(err, -1.0 / 5.0));
      }
      if (O->h_rec && natt <= O->rec_cap) /* the joint attempt, per member */
        for (int32_t i = 0; i < B; ++i)
          if (off[i] >= 0)
            O->h_rec[(long)i * O->rec_cap + natt - 1] = accept ? hs : -hs;
      if (accept) {
        const double tnew = last ? te : t + hs;
        while (cursor < E && teval[cursor] <= tnew) {
          double w[7];
          orc_dense_weights(O->method, (teval[cursor] - t) / hs, w);
          for (int32_t i = 0; i < B; ++i)
            for (int q = 0; off[i] >= 0 && q < P->dim[i]; ++q) {
              double s2 = 0.0;
              for (int j = 0; j < 7; ++j) s2 += w[j] * k[j][off[i] + q];
              y_eval[(i * E + cursor) * D + q] = y[off[i] + q] + hs * s2;
            }
          ++cursor;
        }
        t = tnew;
        memcpy(y, ynew, sizeof(double) * N);
        memcpy(k[0], k[6], sizeof(double) * N); /* FSAL */
        err_prev2 = err_prev;
        err_prev = fmax(err, 1e-4);
        nacc += 1;
        prev_rejected = 0;
        if (last) status = ORC_SUCCESS;
      } else {
        nrej += 1;
        prev_rejected = 1;
      }
      h = hs * fac;
      if (status == ORC_RUNNING && !(h > 16.0 * DBL_EPSILON * fabs(t)))
        status = ORC_DT_UNDERFLOW;
    }
    for (int32_t i = 0; i < B; ++i)
      for (int q = 0; off[i] >= 0 && q < P->dim[i]; ++q)
        y_final[i * D + q] = y[off[i] + q];
    free(buf);
  }
  const int probe = ref >= 0 && !P->h0 && P->t_end[ref] > P->t0[ref];
  for (int32_t i = 0; i < B; ++i) {
    const int member = off[i] >= 0;
    stats[0 * B + i] = member ? natt : 0;
    stats[1 * B + i] = member ? nacc : 0;
    stats[2 * B + i] = member ? nrej : 0;
    stats[3 * B + i] = member ? 1 + probe + 6 * natt : 0;
    stats[4 * B + i] = member ? status : ORC_INVALID;
  }
  free(off);
  return 0;
}
