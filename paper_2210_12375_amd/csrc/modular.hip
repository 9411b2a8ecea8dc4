// Batched ("modular") solver for neural right-hand sides (MLP and CNF fields).
//
// The paper's learned dynamics (section 4.2, appendix A: the FEN graph model
// trained through the solver and the FFJORD continuous normalising flow) are
// batched networks, so the state lives in HBM as [B, D] arrays and one
// attempted step of every running instance is a short sequence of kernels:
//
//   stage s = 2..7   field_kernel: Y_s = y + h sum_{j<s} a_sj k_j formed in
//                    the prologue (per-instance h), then k_s = f(t + c_s h, Y_s)
//   commit_kernel    one wavefront per instance: embedded error, weighted RMS
//                    norm (wavefront reduction), controller, accept / reject,
//                    dense output at the instance's own times, commit
//
// Instances keep their own t, h, controller state and decision (section 3);
// finished instances are skipped by the commit kernel and whole tiles of them
// by the field kernels.  The host drives attempt rounds and reads the running
// count once per kRoundsPerSync rounds.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>
#include <new>

#include "analytic.hpp"
#include "common.hpp"
#include "modular.hpp"
#include "mlp_mfma.hpp"
#include "tableau.hpp"

namespace bode {

namespace {
constexpr int kRoundsPerSync = 8;
}

// ---- device-side description ------------------------------------------------

template <typename R>
struct Mod {
  int32_t B, D, E, H, cnf, d_in;  // d_in: state features fed to the field
  const R* y0;
  const double *t0, *t_end, *rtol, *atol, *t_eval, *h0;
  const R *W1, *b1, *W2, *b2, *W3, *b3, *eps;
  R* y_eval;
  R* y_final;
  State<R> st;     // t, h, err_prev^beta2, counters, status, cursor, y, k1
  R* K;            // [7, B, D] stages (K[0] = k1 = st.k1)
  R* Y7;           // [B, D] stage-7 input = candidate solution
  R* hs;           // [B] size of the current attempt
  int32_t* last;   // [B] the current attempt ends on t_end
  R* aux;          // [B] start-step scratch
  double* h_rec;   // [B, rec_cap] attempt record (rejected < 0)
  int32_t rec_cap;
  int32_t* n_running;
  DenseKeep<R> dk;
  int32_t keep;
  Ctrl ctrl;
};

// Stage input Y = y + hs * sum_j coef_j K[kidx_j]; field time t + c hs.
struct StageSpec {
  int n;
  int kidx[6];
  double coef[6];
  double c;
  int write_y7;
};

template <class M>
StageSpec stage_spec(int s) {  // s = 1..6 (stage s+1)
  StageSpec sp{};
  sp.n = 0;
  for (int j = 0; j < s; ++j)
    if (M::A[s][j] != 0.0) {
      sp.kidx[sp.n] = j;
      sp.coef[sp.n] = M::A[s][j];
      ++sp.n;
    }
  sp.c = M::C[s];
  sp.write_y7 = (s == 6);
  return sp;
}

// ---- field kernel (FMA path: FP64 validation mode and FP32 mode) -------------
//
// ROWS instances per workgroup; thread j owns output column j of every layer
// for those rows (coalesced weight reads, broadcast activation reads from
// LDS).  Each layer accumulates b_j + sum_i in_i W[i][j] in input order.  For
// the CNF the tangent (Jacobian-vector product with the Rademacher probe)
// runs alongside the primal pass.

template <typename R>
__device__ __forceinline__ R rtanh(R x) {
  return tanh(x);
}

template <typename R, int ROWS>
__global__ __launch_bounds__(256) void field_fma_kernel(Mod<R> m, StageSpec sp,
                                                        R* out, int out_stage) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* smem = reinterpret_cast<R*>(smem_raw);
  const int B = m.B, D = m.D, H = m.H, din = m.d_in, n0 = din + 1;
  const int cnf = m.cnf;
  R* X = smem;                       // [ROWS][n0]
  R* A1 = X + ROWS * n0;             // [ROWS][H]
  R* A2 = A1 + ROWS * H;             // [ROWS][H]
  R* dX = A2 + ROWS * H;             // CNF tangents
  R* dA1 = dX + ROWS * n0;
  R* dA2 = dA1 + ROWS * H;
  R* red = cnf ? dA2 + ROWS * H : A2 + ROWS * H;  // [ROWS][din]
  __shared__ int any_running;
  const int r0 = blockIdx.x * ROWS;
  if (threadIdx.x == 0) any_running = 0;
  __syncthreads();
  if (threadIdx.x < ROWS && r0 + threadIdx.x < B &&
      m.st.status[r0 + threadIdx.x] == kRunning)
    any_running = 1;
  __syncthreads();
  if (!any_running) return;

  for (int idx = threadIdx.x; idx < ROWS * D; idx += blockDim.x) {
    const int r = idx / D, c = idx % D, row = r0 + r;
    R Yv = R(0);
    if (row < B) {
      R acc = R(0);
      for (int j = 0; j < sp.n; ++j)
        acc += R(sp.coef[j]) * m.K[((long)sp.kidx[j] * B + row) * D + c];
      Yv = m.st.y[(long)row * D + c] + m.hs[row] * acc;
      if (sp.write_y7) m.Y7[(long)row * D + c] = Yv;
    }
    if (c < din) {
      X[r * n0 + c] = Yv;
      if (cnf) dX[r * n0 + c] = row < B ? m.eps[(long)row * D + c] : R(0);
    }
  }
  for (int r = threadIdx.x; r < ROWS; r += blockDim.x) {
    const int row = r0 + r;
    X[r * n0 + din] =
        row < B ? R(m.st.t[row] + sp.c * double(m.hs[row])) : R(0);
    if (cnf) dX[r * n0 + din] = R(0);  // the probe does not move time
  }
  __syncthreads();

  // layer 1
  for (int j = threadIdx.x; j < H; j += blockDim.x) {
    R acc[ROWS], tac[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) acc[r] = m.b1[j], tac[r] = R(0);
    for (int i = 0; i < n0; ++i) {
      const R w = m.W1[(long)i * H + j];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        acc[r] += X[r * n0 + i] * w;
        if (cnf) tac[r] += dX[r * n0 + i] * w;
      }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const R a = rtanh(acc[r]);
      A1[r * H + j] = a;
      if (cnf) dA1[r * H + j] = (R(1) - a * a) * tac[r];
    }
  }
  __syncthreads();
  // layer 2
  for (int j = threadIdx.x; j < H; j += blockDim.x) {
    R acc[ROWS], tac[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) acc[r] = m.b2[j], tac[r] = R(0);
    for (int i = 0; i < H; ++i) {
      const R w = m.W2[(long)i * H + j];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        acc[r] += A1[r * H + i] * w;
        if (cnf) tac[r] += dA1[r * H + i] * w;
      }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const R a = rtanh(acc[r]);
      A2[r * H + j] = a;
      if (cnf) dA2[r * H + j] = (R(1) - a * a) * tac[r];
    }
  }
  __syncthreads();
  // layer 3 (linear output)
  for (int j = threadIdx.x; j < din; j += blockDim.x) {
    R acc[ROWS], tac[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) acc[r] = m.b3[j], tac[r] = R(0);
    for (int i = 0; i < H; ++i) {
      const R w = m.W3[(long)i * din + j];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        acc[r] += A2[r * H + i] * w;
        if (cnf) tac[r] += dA2[r * H + i] * w;
      }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const int row = r0 + r;
      if (row < B) out[(long)row * D + j] = acc[r];
      if (cnf) red[r * din + j] = m.eps[(long)(row < B ? row : 0) * D + j] *
                                  tac[r];
    }
  }
  if (cnf) {
    __syncthreads();
    // l' = -eps^T (dg/dz) eps, summed in output order
    for (int r = threadIdx.x; r < ROWS; r += blockDim.x) {
      const int row = r0 + r;
      R q = R(0);
      for (int j = 0; j < din; ++j) q += red[r * din + j];
      if (row < B) out[(long)row * D + din] = -q;
    }
  }
  (void)out_stage;
}

template <typename R>
size_t field_smem(int rows, int n0, int H, int din, int cnf) {
  const size_t per = (size_t)n0 + 2 * (size_t)H;
  return sizeof(R) * rows * (per * (cnf ? 2 : 1) + din);
}

template <typename R>
hipError_t launch_field_fma(const Mod<R>& m, const StageSpec& sp, R* out,
                            hipStream_t s) {
  const int n0 = m.d_in + 1;
  int rows = 16;
  while (rows > 1 && field_smem<R>(rows, n0, m.H, m.d_in, m.cnf) > 65536)
    rows /= 2;
  const size_t sm = field_smem<R>(rows, n0, m.H, m.d_in, m.cnf);
  if (sm > 65536) return hipErrorInvalidValue;
  const dim3 g((m.B + rows - 1) / rows), b(256);
  switch (rows) {
    case 16:
      hipLaunchKernelGGL((field_fma_kernel<R, 16>), g, b, sm, s, m, sp, out, 0);
      break;
    case 8:
      hipLaunchKernelGGL((field_fma_kernel<R, 8>), g, b, sm, s, m, sp, out, 0);
      break;
    case 4:
      hipLaunchKernelGGL((field_fma_kernel<R, 4>), g, b, sm, s, m, sp, out, 0);
      break;
    case 2:
      hipLaunchKernelGGL((field_fma_kernel<R, 2>), g, b, sm, s, m, sp, out, 0);
      break;
    default:
      hipLaunchKernelGGL((field_fma_kernel<R, 1>), g, b, sm, s, m, sp, out, 0);
  }
  return hipGetLastError();
}

// ---- row kernels (one wavefront per instance) -----------------------------------

template <typename R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename R>
__device__ __forceinline__ void finish_row(const Mod<R>& m, int row, int lane,
                                           int status, int cursor) {
  const int D = m.D;
  for (int c = lane; c < D; c += 64)
    m.y_final[(long)row * D + c] = m.st.y[(long)row * D + c];
  if (status != kSuccess)
    for (int e = cursor; e < m.E; ++e)
      for (int c = lane; c < D; c += 64)
        m.y_eval[((long)row * m.E + e) * D + c] = quiet_nan<R>();
}

// Initialisation of every instance: input checks, y = y0, answers at t0.
template <typename R>
__global__ void mod_init_rows(Mod<R> m) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= m.B) return;
  const int D = m.D, E = m.E;
  const double t0 = m.t0[row], te = m.t_end[row];
  bool ok = __builtin_isfinite(t0) && __builtin_isfinite(te) && te >= t0;
  const double rt = m.rtol[row], at = m.atol[row];
  ok = ok && rt >= 0.0 && at >= 0.0 && !(rt == 0.0 && at == 0.0);
  if (m.h0 != nullptr) ok = ok && m.h0[row] > 0.0;
  bool fin = true;
  for (int c = lane; c < D; c += 64)
    fin = fin && __builtin_isfinite(double(m.y0[(long)row * D + c]));
  ok = ok && __all(fin);
  bool sorted = true;
  for (int e = lane; e < E; e += 64) {
    const double v = m.t_eval[(long)row * E + e];
    const double prev = e == 0 ? t0 : m.t_eval[(long)row * E + e - 1];
    sorted = sorted && v >= prev && v <= te;
  }
  ok = ok && __all(sorted);
  State<R> st = m.st;
  if (lane == 0) {
    st.n_att[row] = st.n_acc[row] = st.n_rej[row] = 0;
    st.n_fe[row] = ok ? 1 : 0;
    st.prev_rej[row] = 0;
    st.err_prev[row] = R(1);
    st.t[row] = t0;
    st.h[row] = R(0);
    m.hs[row] = R(0);
    m.last[row] = 0;
  }
  if (!ok) {
    if (lane == 0) {
      st.status[row] = kInvalid;
      st.cursor[row] = 0;
    }
    for (int c = lane; c < D; c += 64) {
      m.y_final[(long)row * D + c] = quiet_nan<R>();
      st.y[(long)row * D + c] = quiet_nan<R>();
    }
    for (long e = lane; e < (long)E * D; e += 64)
      m.y_eval[(long)row * E * D + e] = quiet_nan<R>();
    return;
  }
  for (int c = lane; c < D; c += 64)
    st.y[(long)row * D + c] = m.y0[(long)row * D + c];
  int cursor = 0;
  while (cursor < E && m.t_eval[(long)row * E + cursor] <= t0) {
    for (int c = lane; c < D; c += 64)
      m.y_eval[((long)row * E + cursor) * D + c] = m.y0[(long)row * D + c];
    ++cursor;
  }
  if (lane == 0) {
    st.cursor[row] = cursor;
    st.status[row] = te == t0 ? kSuccess : kRunning;
  }
  if (te == t0)
    for (int c = lane; c < D; c += 64)
      m.y_final[(long)row * D + c] = m.y0[(long)row * D + c];
}

// Start step, part 1: d0, d1 and the probe h0' (Hairer, Solving ODEs I,
// II.4), or the user's h0.  The probe evaluation then runs as a stage with
// Y = y0 + h0' k1 at t0 + h0'.
template <typename R>
__global__ void mod_start_a(Mod<R> m) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= m.B || m.st.status[row] != kRunning) return;
  const int D = m.D;
  const R rt = R(m.rtol[row]), at = R(m.atol[row]);
  R s0 = R(0), s1 = R(0);
  for (int c = lane; c < D; c += 64) {
    const R y = m.st.y[(long)row * D + c], k = m.K[(long)row * D + c];
    const R sc = at + rabs(y) * rt;
    const R u = ctl_div(y, sc), v = ctl_div(k, sc);
    s0 += u * u;
    s1 += v * v;
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (lane != 0) return;
  const double span = m.t_end[row] - m.t0[row];
  if (m.h0 != nullptr) {
    m.st.h[row] = R(m.h0[row]);
    return;
  }
  const R d0 = ctl_sqrt(ctl_div(s0, R(D))), d1 = ctl_sqrt(ctl_div(s1, R(D)));
  R h0 = (d0 < R(1e-5) || d1 < R(1e-5)) ? R(1e-6) : R(0.01) * ctl_div(d0, d1);
  h0 = rmin(h0, R(span));
  m.hs[row] = h0;
  m.aux[row] = d1;
  m.st.n_fe[row] += 1;
}

// Start step, part 2 (d2 from the probe f1 in K[1]) and the first attempt's
// size; with a user h0 only the latter.
template <typename R>
__global__ void mod_start_b(Mod<R> m, int probe) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= m.B || m.st.status[row] != kRunning) return;
  const int D = m.D, B = m.B;
  R s2 = R(0);
  if (probe) {
    const R rt = R(m.rtol[row]), at = R(m.atol[row]);
    for (int c = lane; c < D; c += 64) {
      const R y = m.st.y[(long)row * D + c];
      const R k = m.K[(long)row * D + c], f1 = m.K[((long)B + row) * D + c];
      const R sc = at + rabs(y) * rt;
      const R u = ctl_div(f1 - k, sc);
      s2 += u * u;
    }
    s2 = wave_sum(s2);
  }
  if (lane != 0) return;
  const double t = m.st.t[row], te = m.t_end[row];
  R h = m.st.h[row];
  if (probe) {
    const R h0 = m.hs[row], d1 = m.aux[row];
    const R d2 = ctl_div(ctl_sqrt(ctl_div(s2, R(D))), h0);
    R h1;
    if (d1 <= R(1e-15) && d2 <= R(1e-15))
      h1 = rmax(R(1e-6), h0 * R(1e-3));
    else
      h1 = ctl_pow(ctl_div(R(0.01), rmax(d1, d2)), R(0.2));
    h = rmin(rmin(R(100) * h0, h1), R(te - t));
    m.st.h[row] = h;
  }
  const bool last = t + double(h) >= te;
  m.last[row] = last;
  m.hs[row] = last ? R(te - t) : h;
}

// Error norm, controller, accept / reject, dense output, commit.
template <typename R, class M, bool KEEP>
__global__ __launch_bounds__(256) void commit_kernel(Mod<R> m) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= m.B || m.st.status[row] != kRunning) return;
  const int D = m.D, B = m.B;
  const R hs = m.hs[row];
  const R rt = R(m.rtol[row]), at = R(m.atol[row]);
  R acc = R(0);
  for (int c = lane; c < D; c += 64) {
    R eq = R(0);
#pragma unroll
    for (int j = 0; j < 7; ++j)
      if (M::E[j] != 0.0) eq += R(M::E[j]) * m.K[((long)j * B + row) * D + c];
    eq *= hs;
    const R y = m.st.y[(long)row * D + c], yn = m.Y7[(long)row * D + c];
    const R sc = at + rt * rmax(rabs(y), rabs(yn));
    const R r = ctl_div(eq, sc);
    acc += r * r;
  }
  acc = wave_sum(acc);
  const R err = ctl_sqrt(ctl_div(acc, R(D)));
  const bool accept = err < R(1);
  const int n_att = m.st.n_att[row] + 1;
  if (lane == 0 && m.h_rec != nullptr && n_att <= m.rec_cap)
    m.h_rec[(long)row * m.rec_cap + n_att - 1] =
        accept ? double(hs) : -double(hs);
  const Ctrl& c = m.ctrl;
  const R pw = ctl_pow(err, accept ? R(-c.beta1) : R(-0.2));
  R fac = R(c.safety) * pw;
  fac = accept ? fac * m.st.err_prev[row] : fac;
  fac = rmax(R(c.fac_min), accept ? rmin(R(c.fac_max), fac) : fac);
  fac = (accept && m.st.prev_rej[row]) ? rmin(R(1), fac) : fac;
  fac = __builtin_isfinite(err) ? fac : R(c.fac_min);

  double t = m.st.t[row];
  const double te = m.t_end[row];
  const bool last = m.last[row];
  int status = kRunning;
  int cursor = m.st.cursor[row];
  if (accept) {
    const double tnew = last ? te : t + double(hs);
    while (cursor < m.E) {
      const double tv = m.t_eval[(long)row * m.E + cursor];
      if (!(tv <= tnew)) break;
      const R th = R((tv - t) / double(hs));
      R w[7];
#pragma unroll
      for (int j = 0; j < 7; ++j)
        w[j] = th * (R(M::P[j][0]) +
                     th * (R(M::P[j][1]) +
                           th * (R(M::P[j][2]) + th * R(M::P[j][3]))));
      for (int cc = lane; cc < D; cc += 64) {
        R s2 = R(0);
#pragma unroll
        for (int j = 0; j < 7; ++j)
          if (M::P[j][0] != 0.0 || M::P[j][1] != 0.0 || M::P[j][2] != 0.0 ||
              M::P[j][3] != 0.0)
            s2 += w[j] * m.K[((long)j * B + row) * D + cc];
        m.y_eval[((long)row * m.E + cursor) * D + cc] =
            m.st.y[(long)row * D + cc] + hs * s2;
      }
      ++cursor;
    }
    if (KEEP) {
      if (lane == 0) {
        m.dk.t_prev[row] = t;
        m.dk.h_last[row] = hs;
      }
      for (int cc = lane; cc < D; cc += 64) {
        m.dk.y_prev[(long)row * D + cc] = m.st.y[(long)row * D + cc];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          R s2 = R(0);
#pragma unroll
          for (int j = 0; j < 7; ++j)
            if (M::P[j][q] != 0.0)
              s2 += R(M::P[j][q]) * m.K[((long)j * B + row) * D + cc];
          m.dk.q[((long)q * B + row) * D + cc] = hs * s2;
        }
      }
    }
    for (int cc = lane; cc < D; cc += 64) {
      m.st.y[(long)row * D + cc] = m.Y7[(long)row * D + cc];
      m.K[(long)row * D + cc] = m.K[((long)6 * B + row) * D + cc];  // FSAL
    }
    t = tnew;
    if (last) status = kSuccess;
    if (lane == 0) {
      m.st.cursor[row] = cursor;
      m.st.err_prev[row] =
          c.beta2 != 0.0 ? ctl_pow(rmax(err, R(1e-4)), R(c.beta2)) : R(1);
      m.st.n_acc[row] += 1;
    }
  }
  const R h = hs * fac;
  if (status == kRunning && !(double(h) > 16.0 * DBL_EPSILON * fabs(t)))
    status = kDtUnderflow;
  if (status == kRunning && n_att >= c.max_steps) status = kMaxSteps;
  if (lane == 0) {
    m.st.n_att[row] = n_att;
    m.st.n_fe[row] += 6;
    if (!accept) m.st.n_rej[row] += 1;
    m.st.prev_rej[row] = accept ? 0 : 1;
    m.st.t[row] = t;
    m.st.h[row] = h;
    m.st.status[row] = status;
    if (status == kRunning) {
      const bool nl = t + double(h) >= te;
      m.last[row] = nl;
      m.hs[row] = nl ? R(te - t) : h;
      atomicAdd(m.n_running, 1);
    }
  }
  if (status != kRunning) finish_row(m, row, lane, status, cursor);
}

__global__ void count_equal_kernel(const int32_t* a, int n, int32_t v,
                                   int32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool hit = i < n && a[i] == v;
  const unsigned long long msk = __ballot(hit);
  if ((threadIdx.x & 63) == 0 && msk) atomicAdd(out, (int)__popcll(msk));
}

hipError_t launch_count_equal(const int32_t* a, int n, int32_t v, int32_t* out,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(count_equal_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     s, a, n, v, out);
  return hipGetLastError();
}

// ---- host side ----------------------------------------------------------------

struct ModImpl {
  bode_config cfg{};
  bode_problem p{};
  Mod<double> md{};
  Mod<float> mf{};
  MfmaWeights mw{};  // BF16 packed weights (BF16 precision)
  bool is64 = false;
  int32_t* host_running = nullptr;  // pinned
};

namespace {

struct Lay {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) / 256 * 256;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

template <typename R>
size_t lay_mod(const bode_config& c, void* base, Mod<R>* m, MfmaWeights* mw) {
  Lay L{static_cast<char*>(base)};
  const size_t B = c.B, D = c.D;
  State<R> st{};
  st.t = L.take<double>(B);
  st.h = L.take<R>(B);
  st.err_prev = L.take<R>(B);
  st.n_att = L.take<int32_t>(B);
  st.n_acc = L.take<int32_t>(B);
  st.n_rej = L.take<int32_t>(B);
  st.n_fe = L.take<int32_t>(B);
  st.status = L.take<int32_t>(B);
  st.cursor = L.take<int32_t>(B);
  st.prev_rej = L.take<int32_t>(B);
  st.y = L.take<R>(B * D);
  R* K = L.take<R>(7 * B * D);
  st.k1 = K;
  R* Y7 = L.take<R>(B * D);
  R* hs = L.take<R>(B);
  int32_t* last = L.take<int32_t>(B);
  R* aux = L.take<R>(B);
  int32_t* nrun = L.take<int32_t>(64);
  double* h_rec = c.record_cap > 0 ? L.take<double>(B * c.record_cap) : nullptr;
  DenseKeep<R> dk{};
  if (c.keep_dense) {
    dk.t_prev = L.take<double>(B);
    dk.h_last = L.take<R>(B);
    dk.y_prev = L.take<R>(B * D);
    dk.q = L.take<R>(4 * B * D);
  }
  const int din = c.rhs == BODE_RHS_CNF ? c.D - 1 : c.D;
  MfmaWeights w{};
  if (c.precision == BODE_BF16) {
    const size_t n = mfma_packed_elems(din, c.mlp_hidden);
    w.packed = L.take<uint16_t>(n);
    w.fvec = L.take<float>(mfma_fvec_elems(din, c.mlp_hidden));
  }
  if (m) {
    m->st = st;
    m->K = K;
    m->Y7 = Y7;
    m->hs = hs;
    m->last = last;
    m->aux = aux;
    m->n_running = nrun;
    m->h_rec = h_rec;
    m->rec_cap = c.record_cap;
    m->dk = dk;
    m->keep = c.keep_dense;
  }
  if (mw) *mw = w;
  return L.off + 256;
}

template <typename R>
void fill_mod(Mod<R>* m, const bode_config& c, const bode_problem& p) {
  m->B = c.B;
  m->D = c.D;
  m->E = c.E;
  m->H = c.mlp_hidden;
  m->cnf = c.rhs == BODE_RHS_CNF;
  m->d_in = m->cnf ? c.D - 1 : c.D;
  m->y0 = static_cast<const R*>(p.y0);
  m->t0 = p.t0;
  m->t_end = p.t_end;
  m->rtol = p.rtol;
  m->atol = p.atol;
  m->t_eval = p.t_eval;
  m->h0 = p.h0;
  m->W1 = static_cast<const R*>(p.W1);
  m->b1 = static_cast<const R*>(p.b1);
  m->W2 = static_cast<const R*>(p.W2);
  m->b2 = static_cast<const R*>(p.b2);
  m->W3 = static_cast<const R*>(p.W3);
  m->b3 = static_cast<const R*>(p.b3);
  m->eps = static_cast<const R*>(p.eps);
  m->y_eval = static_cast<R*>(p.y_eval);
  m->y_final = static_cast<R*>(p.y_final);
  m->ctrl = Ctrl{c.beta1, c.beta2, c.safety, c.fac_min, c.fac_max,
                 c.max_steps};
}

template <typename R>
hipError_t field(ModImpl& im, const Mod<R>& m, const StageSpec& sp, R* out,
                 hipStream_t s);

template <>
hipError_t field<double>(ModImpl&, const Mod<double>& m, const StageSpec& sp,
                         double* out, hipStream_t s) {
  return launch_field_fma<double>(m, sp, out, s);
}

template <>
hipError_t field<float>(ModImpl& im, const Mod<float>& m, const StageSpec& sp,
                        float* out, hipStream_t s) {
  if (im.cfg.precision == BODE_BF16) {
    MfmaArgs a = mfma_args(m.B, m.D, m.d_in, m.H, m.cnf, m.st.status, m.st.y,
                           m.K, m.Y7, m.hs, m.st.t, m.eps, im.mw);
    a.n = sp.n;
    for (int j = 0; j < 6; ++j) {
      a.kidx[j] = sp.kidx[j];
      a.coef[j] = float(sp.coef[j]);
    }
    a.c = sp.c;
    a.write_y7 = sp.write_y7;
    a.out = out;
    return launch_field_mfma(a, get_row_tile(im.cfg), s);
  }
  return launch_field_fma<float>(m, sp, out, s);
}

template <typename R>
dim3 row_grid(int B) {
  return dim3((B + 3) / 4);
}

template <typename R, class M>
hipError_t round_launch(ModImpl& im, Mod<R>& m, hipStream_t s) {
  hipError_t e = launch_fill_i32(m.n_running, 1, 0, s);
  for (int st = 1; st < 7 && e == hipSuccess; ++st)
    e = field<R>(im, m, stage_spec<M>(st), m.K + (size_t)st * m.B * m.D, s);
  if (e != hipSuccess) return e;
  if (m.keep)
    hipLaunchKernelGGL((commit_kernel<R, M, true>), row_grid<R>(m.B),
                       dim3(256), 0, s, m);
  else
    hipLaunchKernelGGL((commit_kernel<R, M, false>), row_grid<R>(m.B),
                       dim3(256), 0, s, m);
  return hipGetLastError();
}

template <typename R>
hipError_t init_launch(ModImpl& im, Mod<R>& m, hipStream_t s) {
  hipLaunchKernelGGL(mod_init_rows<R>, row_grid<R>(m.B), dim3(256), 0, s, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  StageSpec sp0{};  // Y = y0 at t0
  e = field<R>(im, m, sp0, m.K, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mod_start_a<R>, row_grid<R>(m.B), dim3(256), 0, s, m);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int probe = m.h0 == nullptr;
  if (probe) {
    StageSpec sp{};
    sp.n = 1;
    sp.kidx[0] = 0;
    sp.coef[0] = 1.0;
    sp.c = 1.0;
    e = field<R>(im, m, sp, m.K + (size_t)m.B * m.D, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(mod_start_b<R>, row_grid<R>(m.B), dim3(256), 0, s, m,
                     probe);
  return hipGetLastError();
}

template <typename R>
hipError_t run_rounds(ModImpl& im, Mod<R>& m, int budget, hipStream_t s) {
  int done = 0;
  while (done < budget) {
    const int chunk = budget - done < kRoundsPerSync ? budget - done
                                                     : kRoundsPerSync;
    for (int r = 0; r < chunk; ++r) {
      hipError_t e = im.cfg.method == BODE_TSIT5
                         ? round_launch<R, Tsit5>(im, m, s)
                         : round_launch<R, Dopri5>(im, m, s);
      if (e != hipSuccess) return e;
    }
    done += chunk;
    hipError_t e = hipMemcpyAsync(im.host_running, m.n_running,
                                  sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (*im.host_running == 0) break;
  }
  return hipSuccess;
}

}  // namespace

std::string modular_supported(const bode_config& c) {
  if (c.rhs != BODE_RHS_MLP && c.rhs != BODE_RHS_CNF)
    return "not a neural right-hand side";
  const int din = c.rhs == BODE_RHS_CNF ? c.D - 1 : c.D;
  if (c.precision == BODE_BF16) return mfma_supported(din, c.mlp_hidden);
  if (c.mlp_hidden > 2048 || din > 1024)
    return "MLP width above 2048 or state above 1024 is not built";
  return "";
}

size_t modular_layout(const bode_config& c, void* base, ModularPlan* mp) {
  if (c.precision == BODE_FP64) {
    Mod<double> m{};
    const size_t n = lay_mod<double>(c, base, mp ? &m : nullptr, nullptr);
    if (mp) {
      ModImpl* im = new ModImpl();
      im->md = m;
      im->is64 = true;
      mp->impl = im;
    }
    return n;
  }
  Mod<float> m{};
  MfmaWeights w{};
  const size_t n = lay_mod<float>(c, base, mp ? &m : nullptr, &w);
  if (mp) {
    ModImpl* im = new ModImpl();
    im->mf = m;
    im->mw = w;
    mp->impl = im;
  }
  return n;
}

hipError_t modular_init(ModularPlan& mp, const bode_config& c,
                        const bode_problem& p, hipStream_t s) {
  ModImpl* im = static_cast<ModImpl*>(mp.impl);
  if (!im) return hipErrorInvalidValue;
  im->cfg = c;
  im->p = p;
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&im->host_running),
                               sizeof(int32_t), hipHostMallocDefault);
  if (e != hipSuccess) return e;
  auto publish = [&](auto& m) {
    mp.t = m.st.t;
    mp.n_att = m.st.n_att;
    mp.n_acc = m.st.n_acc;
    mp.n_rej = m.st.n_rej;
    mp.n_fe = m.st.n_fe;
    mp.status = m.st.status;
    mp.cursor = m.st.cursor;
    mp.prev_rej = m.st.prev_rej;
    mp.h_rec = m.h_rec;
  };
  if (im->is64) {
    fill_mod<double>(&im->md, c, p);
    publish(im->md);
    return init_launch<double>(*im, im->md, s);
  }
  fill_mod<float>(&im->mf, c, p);
  publish(im->mf);
  if (c.precision == BODE_BF16) {
    e = mfma_pack_weights(im->mw, im->mf.d_in, c.mlp_hidden,
                          static_cast<const float*>(p.W1),
                          static_cast<const float*>(p.b1),
                          static_cast<const float*>(p.W2),
                          static_cast<const float*>(p.b2),
                          static_cast<const float*>(p.W3),
                          static_cast<const float*>(p.b3), s);
    if (e != hipSuccess) return e;
  }
  return init_launch<float>(*im, im->mf, s);
}

hipError_t modular_run(ModularPlan& mp, int budget, hipStream_t s) {
  ModImpl* im = static_cast<ModImpl*>(mp.impl);
  if (!im) return hipErrorInvalidValue;
  return im->is64 ? run_rounds<double>(*im, im->md, budget, s)
                  : run_rounds<float>(*im, im->mf, budget, s);
}

hipError_t modular_eval(ModularPlan& mp, const double* t_query, void* y_out,
                        int32_t* qstatus, hipStream_t s) {
  ModImpl* im = static_cast<ModImpl*>(mp.impl);
  if (!im) return hipErrorInvalidValue;
  if (im->is64)
    return launch_dense_eval<double>(im->md.dk, im->md.st, im->cfg.B,
                                     im->cfg.D, t_query,
                                     static_cast<double*>(y_out), qstatus, s);
  return launch_dense_eval<float>(im->mf.dk, im->mf.st, im->cfg.B, im->cfg.D,
                                  t_query, static_cast<float*>(y_out), qstatus,
                                  s);
}

hipError_t modular_backward(ModularPlan& mp, const void* g_y_eval,
                            const void* g_y_final, void* dy0, void* dtheta,
                            hipStream_t s);

void modular_release(ModularPlan& mp) {
  ModImpl* im = static_cast<ModImpl*>(mp.impl);
  if (!im) return;
  if (im->host_running) (void)hipHostFree(im->host_running);
  delete im;
  mp.impl = nullptr;
}

}  // namespace bode
