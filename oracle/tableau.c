/*
 * Butcher tableaux and continuous extensions of the two methods the paper
 * names (appendix A: "dopri5", used in every experiment, and "tsit5", which
 * the solver also provides).  TEST INFRASTRUCTURE ONLY.
 *
 * Dopri5: Dormand & Prince (1980), "A family of embedded Runge-Kutta
 * formulae", J. Comp. Appl. Math. 6, written as exact rationals.  Its
 * continuous extension is the fourth-order Hermite-plus-correction form of
 * Hairer, Norsett & Wanner, Solving ODEs I, section II.6 (dense output of
 * DOPRI5), whose correction weights d_j are given below.
 *
 * Tsit5: Tsitouras (2011), "Runge-Kutta pairs of order 5(4) satisfying only
 * the first column simplifying assumption", Comput. Math. Appl. 62, with its
 * degree-4 interpolant in factored form.
 *
 * The paper relies on FSAL and SSAL (section 3, "What makes torchode fast?"):
 * both methods have a_7j = b_j and c_7 = 1, so stage 7 is evaluated at the new
 * solution and becomes stage 1 of the next step.
 */
#include <string.h>

#include "oracle.h"

static void dopri5(double* c, double a[7][7], double* b, double* bh) {
  static const double C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0,
                              8.0 / 9.0, 1.0, 1.0};
  memcpy(c, C, sizeof C);
  memset(a, 0, sizeof(double) * 49);
  a[1][0] = 1.0 / 5.0;
  a[2][0] = 3.0 / 40.0;
  a[2][1] = 9.0 / 40.0;
  a[3][0] = 44.0 / 45.0;
  a[3][1] = -56.0 / 15.0;
  a[3][2] = 32.0 / 9.0;
  a[4][0] = 19372.0 / 6561.0;
  a[4][1] = -25360.0 / 2187.0;
  a[4][2] = 64448.0 / 6561.0;
  a[4][3] = -212.0 / 729.0;
  a[5][0] = 9017.0 / 3168.0;
  a[5][1] = -355.0 / 33.0;
  a[5][2] = 46732.0 / 5247.0;
  a[5][3] = 49.0 / 176.0;
  a[5][4] = -5103.0 / 18656.0;
  static const double B[7] = {35.0 / 384.0,     0.0, 500.0 / 1113.0,
                              125.0 / 192.0,    -2187.0 / 6784.0,
                              11.0 / 84.0,      0.0};
  static const double BH[7] = {5179.0 / 57600.0,    0.0,
                               7571.0 / 16695.0,    393.0 / 640.0,
                               -92097.0 / 339200.0, 187.0 / 2100.0,
                               1.0 / 40.0};
  memcpy(b, B, sizeof B);
  memcpy(bh, BH, sizeof BH);
  for (int j = 0; j < 7; ++j) a[6][j] = B[j]; /* FSAL / SSAL row */
}

static void tsit5(double* c, double a[7][7], double* b, double* bh) {
  static const double C[7] = {0.0, 0.161, 0.327, 0.9, 0.9800255409045097,
                              1.0, 1.0};
  memcpy(c, C, sizeof C);
  memset(a, 0, sizeof(double) * 49);
  a[1][0] = 0.161;
  a[2][0] = -0.008480655492356989;
  a[2][1] = 0.335480655492357;
  a[3][0] = 2.897153057105493;
  a[3][1] = -6.359448489975075;
  a[3][2] = 4.3622954328695815;
  a[4][0] = 5.325864828439257;
  a[4][1] = -11.748883564062828;
  a[4][2] = 7.4955393428898365;
  a[4][3] = -0.09249506636175525;
  a[5][0] = 5.86145544294642;
  a[5][1] = -12.92096931784711;
  a[5][2] = 8.159367898576159;
  a[5][3] = -0.071584973281401;
  a[5][4] = -0.028269050394068383;
  static const double B[7] = {0.09646076681806523, 0.01,
                              0.4798896504144996,  1.379008574103742,
                              -3.290069515436081,  2.324710524099774,
                              0.0};
  /* Tsitouras gives the error weights e = b - bhat; bhat follows. */
  static const double E[7] = {-0.00178001105222577714, -0.0008164344596567469,
                              0.007880878010261995,    -0.1447110071732629,
                              0.5823571654525552,      -0.45808210592918697,
                              1.0 / 66.0};
  memcpy(b, B, sizeof B);
  for (int j = 0; j < 7; ++j) {
    a[6][j] = B[j];
    bh[j] = B[j] - E[j];
  }
}

void orc_tableau(int32_t method, double* c, double* a, double* b,
                 double* bhat) {
  double A[7][7];
  if (method == ORC_TSIT5)
    tsit5(c, A, b, bhat);
  else
    dopri5(c, A, b, bhat);
  memcpy(a, A, sizeof A);
}

/* Dense-output weights w_j(theta) with y(t + theta h) = y_n + h sum w_j k_j. */
void orc_dense_weights(int32_t method, double theta, double* w) {
  const double th = theta;
  if (method == ORC_TSIT5) {
    /* Tsitouras' interpolant b_j(theta), as published in factored form. */
    w[0] = -1.0530884977290216 * th * (th - 1.3299890189751412) *
           (th * th - 1.4364028541716351 * th + 0.7139816917074209);
    w[1] = 0.1017 * th * th *
           (th * th - 2.1966568338249754 * th + 1.2949852507374631);
    w[2] = 2.490627285651252793 * th * th *
           (th * th - 2.38535645472061657 * th + 1.57803468208092486);
    w[3] = -16.54810288924490272 * (th - 1.21712927295533244) *
           (th - 0.61620406037800089) * th * th;
    w[4] = 47.37952196281928122 * (th - 1.203071208372362603) *
           (th - 0.658047292653547382) * th * th;
    w[5] = -34.87065786149660974 * (th - 1.2) * (th - 0.666666666666666667) *
           th * th;
    w[6] = 2.5 * (th - 1.0) * (th - 0.6) * th * th;
    return;
  }
  /* DOPRI5 continuous extension (Hairer-Norsett-Wanner II.6):
   *   y(theta) = y_n + theta (D + (1-theta) (h k1 - D
   *              + theta (2 D - h (k1 + k7) + (1-theta) h sum_j d_j k_j)))
   * with D = y_{n+1} - y_n = h sum_j b_j k_j.  Collecting the coefficient of
   * h k_j term by term gives the weights below.                            */
  static const double d[7] = {-12715105075.0 / 11282082432.0,
                              0.0,
                              87487479700.0 / 32700410799.0,
                              -10690763975.0 / 1880347072.0,
                              701980252875.0 / 199316789632.0,
                              -1453857185.0 / 822651844.0,
                              69997945.0 / 29380423.0};
  double c[7], a[49], b[7], bh[7];
  orc_tableau(ORC_DOPRI5, c, a, b, bh);
  const double u = 1.0 - th;
  for (int j = 0; j < 7; ++j) {
    const double first = (j == 0) ? 1.0 : 0.0;
    const double last = (j == 6) ? 1.0 : 0.0;
    w[j] = th * b[j] + th * u * (first - b[j]) +
           th * th * u * (2.0 * b[j] - first - last) + th * th * u * u * d[j];
  }
}
