/*
 * The oracle's adaptive solve.  TEST INFRASTRUCTURE ONLY.
 *
 * Paper section 3 (Design & Features): the batch dimension is explicit and
 * each instance has its own initial condition, integration bounds, tolerances,
 * step size and accept/reject decision, so the oracle simply solves the
 * instances one after another with a scalar loop.  Where the paper is silent
 * (error norm, controller law, start step, end clipping, evaluation-point
 * ownership) the oracle takes these readings:
 *
 *  - error norm: weighted RMS over the instance's true dimension with scale
 *    atol + rtol * max(|y_n|, |y_n+1|) (Hairer's norm, the one scipy's RK45
 *    uses); accept iff err < 1;
 *  - controller (section 3 and appendix C: PID control generalises the
 *    integral controller of the benchmarks; the PID acts on the logarithm
 *    of the error, Soderlind 2002): on acceptance
 *    fac = clamp(safety err^-beta1 err_prev^beta2 err_prev2^beta3,
 *                fac_min, fac_max),
 *    capped at 1 right after a rejection; on rejection
 *    fac = max(fac_min, safety err^-1/5); err == 0 gives fac_max and a
 *    non-finite err gives fac_min; on acceptance err_prev2 = err_prev and
 *    err_prev = max(err, 1e-4), both 1 before the first accepted step;
 *  - start step: Hairer's rule (Solving ODEs I, II.4) unless h0 is given;
 *  - the step that reaches t_end is clipped to t_end - t and ends exactly on
 *    t_end;
 *  - step n owns the evaluation times in (t_n, t_n+1]; times equal to t0 are
 *    answered with y0 before the first step;
 *  - statistics (section 3: total and accepted steps are collected by
 *    default) count only the instance's own work: f-evaluations are
 *    1 + [start-step probe] + 6 per attempted step (FSAL).
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#include "oracle.h"

static double clampd(double x, double lo, double hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}

/* Hairer's starting step given f0 = f(t0, y0); counts its one probe. */
static double hairer_start(const orc_problem* P, int32_t i, const double* f0,
                           int32_t* nfe) {
  const int n = P->dim[i];
  const double* y0 = P->y0 + (long)i * P->D;
  const double t0 = P->t0[i], span = P->t_end[i] - P->t0[i];
  const double rtol = P->rtol[i], atol = P->atol[i];
  if (span == 0.0) return 0.0;
  double* sc = malloc(sizeof(double) * 3 * n);
  double* y1 = sc + n;
  double* f1 = sc + 2 * n;
  double s0 = 0.0, s1 = 0.0;
  for (int c = 0; c < n; ++c) {
    sc[c] = atol + fabs(y0[c]) * rtol;
    s0 += (y0[c] / sc[c]) * (y0[c] / sc[c]);
    s1 += (f0[c] / sc[c]) * (f0[c] / sc[c]);
  }
  const double d0 = sqrt(s0 / n), d1 = sqrt(s1 / n);
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
  h0 = fmin(h0, span);
  for (int c = 0; c < n; ++c) y1[c] = y0[c] + h0 * f0[c];
  orc_rhs(P, i, t0 + h0, y1, f1);
  *nfe += 1;
  double s2 = 0.0;
  for (int c = 0; c < n; ++c) {
    const double q = (f1[c] - f0[c]) / sc[c];
    s2 += q * q;
  }
  const double d2 = sqrt(s2 / n) / h0;
  double h1;
  if (d1 <= 1e-15 && d2 <= 1e-15)
    h1 = fmax(1e-6, h0 * 1e-3);
  else
    h1 = pow(0.01 / fmax(d1, d2), 1.0 / 5.0);
  free(sc);
  return fmin(fmin(100.0 * h0, h1), span);
}

double orc_initial_step(const orc_problem* P, int32_t i, int32_t* nfe) {
  const int n = P->dim[i];
  double* f0 = malloc(sizeof(double) * n);
  orc_rhs(P, i, P->t0[i], P->y0 + (long)i * P->D, f0);
  *nfe += 1;
  const double h = hairer_start(P, i, f0, nfe);
  free(f0);
  return h;
}

int orc_instance_valid(const orc_problem* P, int32_t i) {
  const int n = P->dim[i];
  if (n < 1 || n > P->D) return 0;
  if (P->kind[i] < ORC_RHS_VDP || P->kind[i] > ORC_RHS_CNF_DIAG) return 0;
  if (P->kind[i] == ORC_RHS_VDP && n != 2) return 0;
  const double t0 = P->t0[i], te = P->t_end[i];
  if (!isfinite(t0) || !isfinite(te) || te < t0) return 0;
  const double rt = P->rtol[i], at = P->atol[i];
  if (!(rt >= 0.0) || !(at >= 0.0) || (rt == 0.0 && at == 0.0)) return 0;
  for (int c = 0; c < n; ++c)
    if (!isfinite(P->y0[(long)i * P->D + c])) return 0;
  const double* te_row = P->t_eval + (long)i * P->E;
  for (int e = 0; e < P->E; ++e) {
    if (!(te_row[e] >= t0 && te_row[e] <= te)) return 0;
    if (e > 0 && te_row[e] < te_row[e - 1]) return 0;
  }
  if (P->h0 && !(P->h0[i] > 0.0)) return 0;
  return 1;
}

/* out = y + h * sum_j w_j k_j over the first n components. */
static void emit(int method, double theta, double h, const double* y,
                 double* const* k, int n, double* out) {
  double w[7];
  orc_dense_weights(method, theta, w);
  for (int c = 0; c < n; ++c) {
    double acc = 0.0;
    for (int j = 0; j < 7; ++j) acc += w[j] * k[j][c];
    out[c] = y[c] + h * acc;
  }
}

static void solve_one(const orc_problem* P, const orc_options* O, int32_t i,
                      double* y_eval, double* y_final, int32_t* stats) {
  const long B = P->B, D = P->D, E = P->E;
  const int n = P->dim[i];
  double c[7], a[7][7], b[7], bh[7], e[7];
  orc_tableau(O->method, c, &a[0][0], b, bh);
  for (int j = 0; j < 7; ++j) e[j] = b[j] - bh[j];

  double* yev = y_eval + (long)i * E * D;
  double* yfin = y_final + (long)i * D;
  for (long q = 0; q < E * D; ++q) yev[q] = ((q % D) < n) ? NAN : 0.0;
  for (long q = 0; q < D; ++q) yfin[q] = (q < n) ? NAN : 0.0;

  int32_t natt = 0, nacc = 0, nrej = 0, nfe = 0, status = ORC_RUNNING;
  if (!orc_instance_valid(P, i)) {
    status = ORC_INVALID;
    goto done;
  }
  {
    double* buf = malloc(sizeof(double) * 10 * n);
    double* y = buf;
    double* Y = buf + n;
    double* k[7];
    for (int j = 0; j < 7; ++j) k[j] = buf + (2 + j) * n;
    double* ynew = buf + 9 * n;

    const double* teval = P->t_eval + (long)i * E;
    const double te = P->t_end[i], rtol = P->rtol[i], atol = P->atol[i];
    const int replay = O->h_replay != NULL;
    const double* hr = replay ? O->h_replay + (long)i * O->replay_cap : NULL;
    const int nr = replay ? O->n_replay[i] : 0;
    int last_acc = -1; /* index of the replay's final accepted step */
    for (int q = 0; q < nr && q < (replay ? O->replay_cap : 0); ++q)
      if (hr[q] > 0.0) last_acc = q;
    const int ends = !replay || !O->replay_final || O->replay_final[i];
    double t = P->t0[i];
    for (int q = 0; q < n; ++q) y[q] = P->y0[(long)i * D + q];
    orc_rhs(P, i, t, y, k[0]);
    nfe = 1;
    int cursor = 0;
    while (cursor < E && teval[cursor] <= t) {
      for (int q = 0; q < n; ++q) yev[(long)cursor * D + q] = y[q];
      ++cursor;
    }
    double h = 0.0;
    if (te == t)
      status = ORC_SUCCESS;
    else if (replay)
      status = (nr > 0 && nr <= O->replay_cap && (last_acc >= 0 || !ends))
                   ? ORC_RUNNING
                   : ORC_INVALID;
    else
      h = P->h0 ? P->h0[i] : hairer_start(P, i, k[0], &nfe);

    double err_prev = 1.0, err_prev2 = 1.0;
    int prev_rejected = 0;
    while (status == ORC_RUNNING) {
      if (natt >= O->max_steps) {
        status = ORC_MAX_STEPS;
        break;
      }
      int last;
      double hs;
      int replay_reject = 0;
      if (replay) {
        if (natt >= nr) { /* sequence exhausted before the end */
          status = ORC_MAX_STEPS;
          break;
        }
        hs = fabs(hr[natt]);
        replay_reject = hr[natt] < 0.0;
        last = ends && (natt == last_acc);
      } else {
        last = (t + h >= te);
        hs = last ? te - t : h;
      }
      /* stages 2..7: Y_s = y + h sum_{j<s} a_sj k_j, k_s = f(t + c_s h, Y_s) */
      for (int s = 1; s < 7; ++s) {
        for (int q = 0; q < n; ++q) {
          double acc = 0.0;
          for (int j = 0; j < s; ++j) acc += a[s][j] * k[j][q];
          Y[q] = y[q] + hs * acc;
        }
        if (O->round_state_f32 == 2) /* float-datapath probe, see oracle.h */
          for (int q = 0; q < n; ++q) Y[q] = (double)(float)Y[q];
        orc_rhs(P, i, t + c[s] * hs, Y, k[s]);
        if (O->round_state_f32 == 2)
          for (int q = 0; q < n; ++q) k[s][q] = (double)(float)k[s][q];
      }
      memcpy(ynew, Y, sizeof(double) * n); /* SSAL: stage 7 input is y_n+1 */
      nfe += 6;
      natt += 1;

      double acc = 0.0;
      for (int q = 0; q < n; ++q) {
        double eq = 0.0;
        for (int j = 0; j < 7; ++j) eq += e[j] * k[j][q];
        eq *= hs;
        const double sc = atol + rtol * fmax(fabs(y[q]), fabs(ynew[q]));
        acc += (eq / sc) * (eq / sc);
      }
      const double err = sqrt(acc / n);
      int accept = O->fixed_step || (replay ? !replay_reject : err < 1.0);
      double fac = 1.0;
      if (!O->fixed_step) {
        if (!isfinite(err))
          fac = O->fac_min;
        else if (accept) {
          if (err == 0.0)
            fac = O->fac_max;
          else
            fac = clampd(O->safety * pow(err, -O->beta1) *
                             pow(err_prev, O->beta2) *
                             pow(err_prev2, O->beta3),
                         O->fac_min, O->fac_max);
          if (prev_rejected) fac = fmin(1.0, fac);
        } else {
          fac = fmax(O->fac_min, O->safety * pow(err, -1.0 / 5.0));
        }
      }
      if (O->h_rec && natt <= O->rec_cap)
        O->h_rec[(long)i * O->rec_cap + natt - 1] = accept ? hs : -hs;
      if (replay && O->err_rec)
        O->err_rec[(long)i * O->replay_cap + natt - 1] = err;
      if (replay && O->hprop_rec)
        O->hprop_rec[(long)i * O->replay_cap + natt - 1] = hs * fac;
      if (accept) {
        const double tnew = last ? te : t + hs;
        while (cursor < E && teval[cursor] <= tnew) {
          const double theta = (teval[cursor] - t) / hs;
          emit(O->method, theta, hs, y, k, n, yev + (long)cursor * D);
          ++cursor;
        }
        t = tnew;
        memcpy(y, ynew, sizeof(double) * n);
        if (O->round_state_f32)
          for (int c = 0; c < n; ++c) y[c] = (double)(float)y[c];
        memcpy(k[0], k[6], sizeof(double) * n); /* FSAL */
        err_prev2 = err_prev;
        err_prev = fmax(err, 1e-4);
        nacc += 1;
        prev_rejected = 0;
        if (last) status = ORC_SUCCESS;
      } else {
        nrej += 1;
        prev_rejected = 1;
      }
      if (!replay) {
        h = hs * fac;
        if (status == ORC_RUNNING && !(h > 16.0 * DBL_EPSILON * fabs(t)))
          status = ORC_DT_UNDERFLOW;
      }
    }
    for (int q = 0; q < n; ++q) yfin[q] = y[q];
    free(buf);
  }
done:
  stats[0 * B + i] = natt;
  stats[1 * B + i] = nacc;
  stats[2 * B + i] = nrej;
  stats[3 * B + i] = nfe;
  stats[4 * B + i] = status;
}

int orc_solve(const orc_problem* P, const orc_options* O, double* y_eval,
              double* y_final, int32_t* stats) {
  if (!P || !O || P->B < 0 || P->D < 1 || P->E < 0 || !y_final || !stats)
    return -1;
  if (P->E > 0 && (!y_eval || !P->t_eval)) return -1;
  if (O->method != ORC_DOPRI5 && O->method != ORC_TSIT5) return -1;
  if (O->fixed_step && (!P->h0 || O->h_replay)) return -1;
  const int nt = O->n_threads > 0 ? O->n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int32_t i = 0; i < P->B; ++i) solve_one(P, O, i, y_eval, y_final, stats);
  return 0;
}
