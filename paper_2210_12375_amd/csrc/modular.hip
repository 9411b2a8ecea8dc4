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

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "analytic.hpp"
#include "common.hpp"
#include "modular.hpp"
#include "mlp_mfma.hpp"
#include "mlp_mfma_tile.hpp"
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
  State<R> st;     // t, h, error history, counters, status, cursor, y, k1
  R* K;            // [7, B, D] stages (K[0] = k1 = st.k1)
  R* Y7;           // [B, D] stage-7 input = candidate solution
  R* hs;           // [B] size of the current attempt
  int32_t* last;   // [B] the current attempt ends on t_end
  R* aux;          // [B] start-step scratch
  double* h_rec;   // [B, rec_cap] attempt record (rejected < 0)
  double* e_rec;   // [B, rec_cap] the attempts' error norms
  int32_t rec_cap;
  int32_t* n_running;
  DenseKeep<R> dk;
  int32_t keep;
  Ctrl ctrl;
  R* ckpt;          // [B, ck_cap, D] y_n for n = 0, k, 2k, ... (or nullptr)
  int32_t ck_every, ck_cap;
};

// Stage input Y = y + hs * sum_j coef_j K[kidx_j]; field time t + c hs.
struct StageSpec {
  int n;
  int kidx[6];
  double coef[6];
  double c;
  void* yout;  // if not null, the stage input Y is written here ([B, D])
  void* act_out;  // matrix-core fields: the hidden layers' values (MfmaArgs)
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
  sp.yout = nullptr;
  return sp;
}

// Buffers of the discrete-adjoint backward (workspace views).
template <typename R>
struct Back {
  double* hacc;    // [B, cap] accepted step sizes, in order
  double* tn;      // [B, cap + 1] step start times
  int32_t* nacc;   // [B] accepted steps in the record
  int32_t* owner;  // [B, E] step answering each evaluation time (-1: t0)
  int32_t* act;    // [B] status view: running iff step n exists
  R* bh;           // [B] h_n of the step being processed
  double* bt;      // [B] t_n
  R* lam;          // [B, D] cotangent of y_n+1 / y_n
  R* lamn;         // [B, D] cotangent of y_n being accumulated
  R* kap;          // [7, B, D] stage cotangents
  R* Ys;           // [7, B, D] stage inputs of step n
  R* Ks;           // [7, B, D] stage values
  R* yseg;         // [k + 1, B, D] states of the current segment
  R* slots;        // [G, P] split-K partials of the parameter gradient
  int32_t* flags;  // [0]: max accepted steps, [1]: record overflow
  // Tape of C steps, sample-major ([k][feature], k = (slot * 7 + stage) *
  // Bs + row, Bs = B, or 2B for the CNF whose tangent rows follow the
  // primal ones; slot = the step's place in its chunk of C):
  // layer inputs with a trailing constant feature (1 on primal rows, 0 on
  // tangent rows: the bias gradient) and the layer-output cotangents.  Row
  // widths: T1in din + 2, T2in and T3in H + 1, T1g and T2g H, T3g din.
  R *T1in, *T1g, *T2in, *T2g, *T3in, *T3g;
  long K;  // 7 * Bs * C
  int32_t cap, k, G, C;
  // Segment store (matrix-core fields, when it fits): the stage inputs
  // [k][7][B][D] and hidden-layer values [k][7][Bs][2][H] of every step of
  // the current checkpoint segment, kept from its one recomputation so the
  // vector-Jacobian products neither recompute stages nor the forward layers
  // (null: recompute per step).
  // Two such stores (half 1 at Yst + yst_half, Ast + ast_half): the next
  // segment's recomputation runs on a second stream while this segment's
  // vector-Jacobian products run, with its own step view act2, bh2, bt2.
  R* Yst;
  float* Ast;
  size_t yst_half, ast_half;
  int32_t* act2;
  R* bh2;
  double* bt2;
  long P;
};

constexpr int kSlots = 128;  // most k-splits of a parameter-gradient GEMM

// Steps the discrete adjoint's gradient tape holds: the parameter gradient
// is one GEMM per layer over a chunk of steps, so a small batch's GEMMs run
// on enough tape rows to fill the chip (one step of a 1024-instance MLP is
// 7168 rows, 0.9 GFLOP); the tape is two halves whose chunks alternate, so
// at most 4 steps (chunks of two: the last chunk's GEMMs, which follow the
// last VJP, stay short) and at most 512 MiB, but two steps where one fits
// in 1 GiB (a 8192-instance CNF step is 0.96 GB).
inline int tape_steps(const bode_config& c, long B, int din, int H,
                      size_t elem) {
  const long rows = 7L * B * (c.rhs == BODE_RHS_CNF ? 2 : 1);
  const size_t per_step =
      (size_t)rows * (size_t)((din + 2) + H + 2 * (H + 1) + H + din) * elem;
  const size_t budget = size_t(512) << 20;
  int steps = per_step > 0 ? (int)(budget / per_step) : 1;
  // two steps at least while a step's tape is at most 1 GiB, so that one
  // step's parameter-gradient GEMMs can run beside the next one's VJPs
  if (steps < 2 && per_step <= (size_t(1) << 30)) steps = 2;
  if (steps > 4) steps = 4;
  if (steps > c.record_cap) steps = c.record_cap;
  return steps < 1 ? 1 : steps;
}

inline long n_params(int din, int H) {
  const long n0 = din + 1;
  return n0 * H + H + (long)H * H + H + (long)H * din + din;
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
      if (sp.yout) static_cast<R*>(sp.yout)[(long)row * D + c] = Yv;
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

// Sum over the W lanes (32 or 64) that share a row.
template <int W, typename R>
__device__ __forceinline__ R group_sum(R v) {
#pragma unroll
  for (int o = W / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename R, int W = 64>
__device__ __forceinline__ void finish_row(const Mod<R>& m, int row, int lane,
                                           int status, int cursor) {
  const int D = m.D;
  for (int c = lane; c < D; c += W)
    m.y_final[(long)row * D + c] = m.st.y[(long)row * D + c];
  if (status != kSuccess)
    for (int e = cursor; e < m.E; ++e)
      for (int c = lane; c < D; c += W)
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
    st.err_prev2[row] = R(1);
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
  for (int c = lane; c < D; c += 64) {
    st.y[(long)row * D + c] = m.y0[(long)row * D + c];
    if (m.ckpt) m.ckpt[(long)row * m.ck_cap * D + c] = m.y0[(long)row * D + c];
  }
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

// Where a row's seven stage values are: stage j, column c at
// base[j * sj + rr * D + c] — the [7, B, D] arrays in HBM (base = m.K,
// sj = B D, rr = the row), or in the fused solve a tile's [7, rows, D]
// block in LDS (KL: rr = the row's place in the tile).
template <typename R>
struct KView {
  R* base;
  long sj;
  int rr;
};

// Error norm, controller, accept / reject, dense output, commit.
// One row per W lanes (W = 64: a wavefront; W = 32: half of one, two rows
// at a time); lane is the row's own lane index in [0, W).
template <typename R, class M, bool KEEP, int W = 64, bool KL = false>
__device__ __forceinline__ void commit_row(const Mod<R>& m, int row, int lane,
                                           KView<R> kw = KView<R>{}) {
  if (row >= m.B || m.st.status[row] != kRunning) return;
  const int D = m.D, B = m.B;
  if (!KL) kw = KView<R>{m.K, (long)B * D, row};
  R* const kr = kw.base + (long)kw.rr * D;  // stage 0 of the row
  const long sj = kw.sj;
  const R hs = m.hs[row];
  const R rt = R(m.rtol[row]), at = R(m.atol[row]);
  R acc = R(0);
  // FP32 rows of at most 4 W columns, a multiple of 4: each lane owns four
  // consecutive columns, loads every array it needs as one 16-byte vector
  // (all loads in flight together) and keeps the candidate and the last
  // stage in registers for the commit below
  constexpr bool kF = std::is_same<R, float>::value;
  const bool vec = kF && (D & 3) == 0 && D <= 4 * W;
  const bool own = vec && lane * 4 < D;
  f32x4 ynv{}, k6v{};
  if (vec) {
    if (own) {
      const long o = (long)row * D + lane * 4;
      // the stages are read once here (the next attempt rewrites them):
      // non-temporal loads
      f32x4 kv[7];
#pragma unroll
      for (int j = 0; j < 7; ++j)
        if (M::E[j] != 0.0 || j == 6) {
          const f32x4* q = reinterpret_cast<const f32x4*>(
              reinterpret_cast<const float*>(kr) + j * sj + lane * 4);
          kv[j] = KL ? *q : __builtin_nontemporal_load(q);
        }
      const f32x4 yv = __builtin_nontemporal_load(
          reinterpret_cast<const f32x4*>(
              reinterpret_cast<const float*>(m.st.y) + o));
      ynv = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(
          reinterpret_cast<const float*>(m.Y7) + o));
      k6v = kv[6];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float eq = 0.f;
#pragma unroll
        for (int j = 0; j < 7; ++j)
          if (M::E[j] != 0.0) eq += float(M::E[j]) * kv[j][q];
        eq *= float(hs);
        const float sc = float(at) + float(rt) * rmax(rabs(yv[q]),
                                                      rabs(ynv[q]));
        const float r = ctl_div(eq, sc);
        acc += R(r * r);
      }
    }
  } else {
    for (int c = lane; c < D; c += W) {
      R eq = R(0);
#pragma unroll
      for (int j = 0; j < 7; ++j)
        if (M::E[j] != 0.0)
          eq += R(M::E[j]) * kr[j * sj + c];
      eq *= hs;
      const R y = m.st.y[(long)row * D + c], yn = m.Y7[(long)row * D + c];
      const R sc = at + rt * rmax(rabs(y), rabs(yn));
      const R r = ctl_div(eq, sc);
      acc += r * r;
    }
  }
  acc = group_sum<W>(acc);
  const R err = ctl_sqrt(ctl_div(acc, R(D)));
  const bool accept = m.ctrl.fixed || err < R(1);
  const int n_att = m.st.n_att[row] + 1;
  if (lane == 0 && m.h_rec != nullptr && n_att <= m.rec_cap) {
    m.h_rec[(long)row * m.rec_cap + n_att - 1] =
        accept ? double(hs) : -double(hs);
    m.e_rec[(long)row * m.rec_cap + n_att - 1] = double(err);
  }
  const Ctrl& c = m.ctrl;
  const R pw = ctl_pow(err, accept ? R(-c.beta1) : R(-0.2));
  R fac = R(c.safety) * pw;
  if (accept) {  // PI and PID terms of the two previous accepted steps
    if (c.beta2 != 0.0) fac = fac * ctl_pow(m.st.err_prev[row], R(c.beta2));
    if (c.beta3 != 0.0) fac = fac * ctl_pow(m.st.err_prev2[row], R(c.beta3));
  }
  fac = (accept && err == R(0)) ? R(c.fac_max) : fac;
  fac = rmax(R(c.fac_min), accept ? rmin(R(c.fac_max), fac) : fac);
  fac = (accept && m.st.prev_rej[row]) ? rmin(R(1), fac) : fac;
  fac = __builtin_isfinite(err) ? fac : R(c.fac_min);
  fac = c.fixed ? R(1) : fac;  // fixed step: h stays

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
      for (int cc = lane; cc < D; cc += W) {
        R s2 = R(0);
#pragma unroll
        for (int j = 0; j < 7; ++j)
          if (M::P[j][0] != 0.0 || M::P[j][1] != 0.0 || M::P[j][2] != 0.0 ||
              M::P[j][3] != 0.0)
            s2 += w[j] * kr[j * sj + cc];
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
      for (int cc = lane; cc < D; cc += W) {
        m.dk.y_prev[(long)row * D + cc] = m.st.y[(long)row * D + cc];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          R s2 = R(0);
#pragma unroll
          for (int j = 0; j < 7; ++j)
            if (M::P[j][q] != 0.0)
              s2 += R(M::P[j][q]) * kr[j * sj + cc];
          m.dk.q[((long)q * B + row) * D + cc] = hs * s2;
        }
      }
    }
    const int nacc = m.st.n_acc[row] + 1;
    const bool ck = m.ckpt != nullptr && nacc % m.ck_every == 0 &&
                    nacc / m.ck_every < m.ck_cap;
    if (vec) {
      if (own) {
        const long o = (long)row * D + lane * 4;
        *reinterpret_cast<f32x4*>(reinterpret_cast<float*>(m.st.y) + o) = ynv;
        *reinterpret_cast<f32x4*>(reinterpret_cast<float*>(kr) + lane * 4) =
            k6v;  // FSAL
        if (ck)
          *reinterpret_cast<f32x4*>(
              reinterpret_cast<float*>(m.ckpt) +
              ((long)row * m.ck_cap + nacc / m.ck_every) * D + lane * 4) = ynv;
      }
    } else {
      for (int cc = lane; cc < D; cc += W) {
        const R yn = m.Y7[(long)row * D + cc];
        m.st.y[(long)row * D + cc] = yn;
        kr[cc] = kr[6 * sj + cc];  // FSAL
        if (ck)
          m.ckpt[((long)row * m.ck_cap + nacc / m.ck_every) * D + cc] = yn;
      }
    }
    t = tnew;
    if (last) status = kSuccess;
    if (lane == 0) {
      m.st.cursor[row] = cursor;
      m.st.err_prev2[row] = m.st.err_prev[row];
      m.st.err_prev[row] = rmax(err, R(1e-4));
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
    }
  }
  if (status != kRunning) finish_row<R, W>(m, row, lane, status, cursor);
}

// One workgroup per group of 256 / W rows (a grid-stride form over 2048
// workgroups measured slower on 2^20 rows: 608 against 573 us).
template <typename R, class M, bool KEEP, int W>
__global__ __launch_bounds__(256) void commit_kernel(Mod<R> m) {
  commit_row<R, M, KEEP, W>(m, blockIdx.x * (blockDim.x / W) + threadIdx.x / W,
                            threadIdx.x % W);
}

inline dim3 commit_grid(int B, int per) { return dim3((B + per - 1) / per); }

// ---- fused persistent solve (matrix-core fields) ------------------------------
//
// One launch per solve: a workgroup owns one 16-row tile of the field kernel
// (16 instances, or 8 CNF instances with their tangent rows) and runs its
// instances' attempts to the end: the six new stage evaluations of an
// attempt, then each row's commit by one wavefront.  Instances are
// independent (each has its own step, section 3), so no workgroup waits on
// another and there is no per-round launch or host round trip.  Stage
// outputs pass between the waves of the tile through memory; the barrier
// between stages orders them (all waves share the compute unit's cache).
struct FusedArgs {
  MfmaArgs st[6];  // stages 2..7: combination, node, output
  int budget;      // attempts per instance
  int kl_off;      // KL: byte offset of the tile's stage block in LDS
};

// KL: the tile's seven stage values stay in LDS ([7][rows][D] after the
// field's own LDS): stage inputs, outputs, error estimate, dense outputs and
// FSAL never go through HBM; the FSAL stage is loaded at entry and stored
// back at exit (a later launch, or a step slice, continues from it).
template <class Op, int NTW, bool CNF, int WV, class M, bool KL>
__global__ __launch_bounds__(64 * WV) void solve_fused_kernel(Mod<float> m,
                                                              FusedArgs f) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int PR = CNF ? 8 : 16;
  const int r0 = blockIdx.x * PR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int D = m.D;
  float* kl = KL ? reinterpret_cast<float*>(smem_raw + f.kl_off) : nullptr;
  if (KL) {
    for (int i = threadIdx.x; i < PR * D; i += blockDim.x) {
      const int row = r0 + i / D;
      kl[i] = row < m.B ? m.K[(long)row * D + i % D] : 0.f;
    }
  }
  __shared__ int active;
  for (int round = 0; round < f.budget; ++round) {
    __syncthreads();
    if (threadIdx.x == 0) active = 0;
    __syncthreads();
    if (threadIdx.x < PR && r0 + (int)threadIdx.x < m.B &&
        m.st.status[r0 + threadIdx.x] == kRunning)
      active = 1;
    __syncthreads();
    if (!active) break;
    for (int s = 0; s < 6; ++s) {
      mtile::field_tile<Op, NTW, CNF, WV, false, KL>(f.st[s], r0, smem_raw,
                                                      kl);
      __syncthreads();
    }
    // MLP: two rows per wavefront (32 lanes each) while D fits two columns
    // a lane (364 vs 404 us for 4096 instances); the CNF keeps one row per
    // wavefront, whose tile kernel is already at the register limit of two
    // wavefronts per SIMD
    if (!CNF && m.D <= 64) {
      for (int r = 2 * wave + (lane >> 5); r < PR; r += 2 * WV)
        commit_row<float, M, false, 32, KL>(m, r0 + r, lane & 31,
                                            KView<float>{kl, PR * D, r});
    } else {
      for (int r = wave; r < PR; r += WV)
        commit_row<float, M, false, 64, KL>(m, r0 + r, lane,
                                            KView<float>{kl, PR * D, r});
    }
  }
  if (KL) {  // the FSAL stage back to HBM
    __syncthreads();
    for (int i = threadIdx.x; i < PR * D; i += blockDim.x) {
      const int row = r0 + i / D;
      if (row < m.B) m.K[(long)row * D + i % D] = kl[i];
    }
  }
}

template <class Op, int NTW, bool CNF, int WV, class M>
hipError_t fused_t(const Mod<float>& m, FusedArgs f, hipStream_t s) {
  constexpr int PR = CNF ? 8 : 16;
  const size_t sm = mtile::mfma_smem<Op, NTW, CNF, WV>(m.d_in);
  if (sm > 65536) return hipErrorInvalidValue;
  // the stage block in LDS while it fits beside the field's LDS
  f.kl_off = (int)((sm + 15) / 16 * 16);
  const size_t smk = f.kl_off + sizeof(float) * 7 * PR * (size_t)m.D;
  if (smk <= 65536)
    hipLaunchKernelGGL((solve_fused_kernel<Op, NTW, CNF, WV, M, true>),
                       dim3((m.B + PR - 1) / PR), dim3(64 * WV), smk, s, m,
                       f);
  else
    hipLaunchKernelGGL((solve_fused_kernel<Op, NTW, CNF, WV, M, false>),
                       dim3((m.B + PR - 1) / PR), dim3(64 * WV), sm, s, m, f);
  return hipGetLastError();
}

// Wavefronts per tile as for the per-stage field kernel (4 for the CNF at
// H = 512: 2.89 vs 3.35 ms per solve of 8192 instances).
template <class Op, bool CNF, class M>
hipError_t fused_h(const Mod<float>& m, const FusedArgs& f, hipStream_t s) {
  const int wv = mfma_waves(m.H, CNF, m.B, f.st[0].waves);
  switch (m.H) {
    case 512:
      return wv == 4 ? fused_t<Op, 8, CNF, 4, M>(m, f, s)
                     : fused_t<Op, 4, CNF, 8, M>(m, f, s);
    case 256:
      return wv == 4 ? fused_t<Op, 4, CNF, 4, M>(m, f, s)
                     : fused_t<Op, 2, CNF, 8, M>(m, f, s);
    case 128:
      return wv == 4 ? fused_t<Op, 2, CNF, 4, M>(m, f, s)
                     : fused_t<Op, 1, CNF, 8, M>(m, f, s);
    default: return fused_t<Op, 1, CNF, 4, M>(m, f, s);
  }
}

template <class M>
hipError_t fused_launch(const Mod<float>& m, const FusedArgs& f, int f32,
                        int plain, hipStream_t s) {
  if (f32)
    return m.cnf ? fused_h<mtile::F32, true, M>(m, f, s)
                 : fused_h<mtile::F32, false, M>(m, f, s);
  if (plain)
    return m.cnf ? fused_h<mtile::Bf1, true, M>(m, f, s)
                 : fused_h<mtile::Bf1, false, M>(m, f, s);
  return m.cnf ? fused_h<mtile::Bf3, true, M>(m, f, s)
               : fused_h<mtile::Bf3, false, M>(m, f, s);
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
  Back<double> bd{};
  Back<float> bf{};
  MfmaWeights mw{};  // packed weights of the matrix-core kernels
  bool is64 = false;
  int32_t* host_running = nullptr;  // pinned
  // rounds_per_sync rounds of the per-stage loop, captured once per handle
  hipGraphExec_t rounds_exec = nullptr;
  int rounds_per_sync = 0;
  // private stream for captures (the caller's may be the null stream,
  // which cannot be captured; graphs are replayed on the caller's)
  hipStream_t cap_stream = nullptr;
  // the discrete adjoint's events for its second stream (segment
  // recomputation): start, ready[2], free[2], done; and for its third
  // (tape GEMMs): chunk written, GEMMs of tape half 0 / 1 done, all done
  hipEvent_t ev[10] = {};
};

// Captures what enqueue(q) launches on the handle's capture stream q into an
// executable graph (no memset nodes: every fill here is a kernel).
template <class F>
hipError_t capture(ModImpl& im, F enqueue, hipGraphExec_t* out) {
  hipError_t e = hipSuccess;
  if (im.cap_stream == nullptr)
    e = hipStreamCreateWithFlags(&im.cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  hipStream_t q = im.cap_stream;
  e = hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t ee = enqueue(q);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(q, &g);
  if (ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return ee;
  }
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

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

// BF16 always runs on the matrix cores; FP32 does where the shape is built
// (else the FMA kernels); FP64 uses the FMA kernels.
inline bool uses_mfma(const bode_config& c, int din) {
  if (c.precision == BODE_BF16) return true;
  return c.precision == BODE_FP32 && mfma_supported(din, c.mlp_hidden).empty();
}

template <typename R>
size_t lay_mod(const bode_config& c, void* base, Mod<R>* m, MfmaWeights* mw,
               Back<R>* bkout) {
  Lay L{static_cast<char*>(base)};
  const size_t B = c.B, D = c.D;
  State<R> st{};
  st.t = L.take<double>(B);
  st.h = L.take<R>(B);
  st.err_prev = L.take<R>(B);
  st.err_prev2 = L.take<R>(B);
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
  double* e_rec = c.record_cap > 0 ? L.take<double>(B * c.record_cap) : nullptr;
  DenseKeep<R> dk{};
  if (c.keep_dense) {
    dk.t_prev = L.take<double>(B);
    dk.h_last = L.take<R>(B);
    dk.y_prev = L.take<R>(B * D);
    dk.q = L.take<R>(4 * B * D);
  }
  const int din = c.rhs == BODE_RHS_CNF ? c.D - 1 : c.D;
  R* ckpt = nullptr;
  int ck_cap = 0;
  if (c.ckpt_every > 0) {
    ck_cap = c.record_cap / c.ckpt_every + 2;
    ckpt = L.take<R>(B * (size_t)ck_cap * D);
  }
  Back<R> bk{};
  if (c.record_cap > 0) {
    const size_t cap = c.record_cap;
    const int k = c.ckpt_every > 0 ? c.ckpt_every : c.record_cap;
    bk.cap = c.record_cap;
    bk.k = k;
    bk.P = n_params(din, c.mlp_hidden);
    bk.G = kSlots;
    bk.hacc = L.take<double>(B * cap);
    bk.tn = L.take<double>(B * (cap + 1));
    bk.nacc = L.take<int32_t>(B);
    bk.owner = L.take<int32_t>(B * (size_t)(c.E > 0 ? c.E : 1));
    bk.act = L.take<int32_t>(B);
    bk.bh = L.take<R>(B);
    bk.bt = L.take<double>(B);
    bk.lam = L.take<R>(B * D);
    bk.lamn = L.take<R>(B * D);
    bk.kap = L.take<R>(7 * B * D);
    bk.Ys = L.take<R>(7 * B * D);
    bk.Ks = L.take<R>(7 * B * D);
    bk.yseg = L.take<R>((size_t)(k + 1) * B * D);
    bk.slots = L.take<R>((size_t)bk.G * bk.P);
    bk.flags = L.take<int32_t>(64);
    const int H = c.mlp_hidden, n0 = din + 1;
    bk.C = tape_steps(c, B, din, H, sizeof(R));
    bk.K = 7L * (long)B * (c.rhs == BODE_RHS_CNF ? 2 : 1) * bk.C;
    bk.T1in = L.take<R>((size_t)(n0 + 1) * bk.K);
    bk.T1g = L.take<R>((size_t)H * bk.K);
    bk.T2in = L.take<R>((size_t)(H + 1) * bk.K);
    bk.T2g = L.take<R>((size_t)H * bk.K);
    bk.T3in = L.take<R>((size_t)(H + 1) * bk.K);
    bk.T3g = L.take<R>((size_t)din * bk.K);
    const size_t Bs = B * (c.rhs == BODE_RHS_CNF ? 2 : 1);
    const size_t store = (size_t)k * 7 * (B * D * sizeof(R) + Bs * 2 * H * 4);
    if (std::is_same<R, float>::value && uses_mfma(c, din) &&
        store <= (size_t(2) << 30)) {
      bk.yst_half = (size_t)k * 7 * B * D;
      bk.ast_half = (size_t)k * 7 * Bs * 2 * H;
      bk.Yst = L.take<R>(2 * bk.yst_half);
      bk.Ast = L.take<float>(2 * bk.ast_half);
      bk.act2 = L.take<int32_t>(B);
      bk.bh2 = L.take<R>(B);
      bk.bt2 = L.take<double>(B);
    }
  }
  MfmaWeights w{};
  if (uses_mfma(c, din)) {
    w.f32 = c.precision == BODE_FP32;
    w.plain = c.precision == BODE_BF16 && c.plain_bf16;
    w.packed = L.take<unsigned char>(mfma_packed_bytes(din, c.mlp_hidden, w.f32));
    w.fvec = L.take<float>(mfma_fvec_elems(din, c.mlp_hidden));
    // transposed layers for the VJP kernels (discrete and continuous adjoint)
    w.packedT =
        L.take<unsigned char>(mfma_packedT_bytes(din, c.mlp_hidden, w.f32));
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
    m->e_rec = e_rec;
    m->rec_cap = c.record_cap;
    m->dk = dk;
    m->keep = c.keep_dense;
    m->ckpt = ckpt;
    m->ck_every = c.ckpt_every;
    m->ck_cap = ck_cap;
  }
  if (bkout) *bkout = bk;
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
                 c.max_steps, c.beta3, c.fixed_step};
}

template <typename R>
hipError_t field(ModImpl& im, const Mod<R>& m, const StageSpec& sp, R* out,
                 hipStream_t s);

template <>
hipError_t field<double>(ModImpl&, const Mod<double>& m, const StageSpec& sp,
                         double* out, hipStream_t s) {
  return launch_field_fma<double>(m, sp, out, s);
}

MfmaArgs stage_args(const ModImpl& im, const Mod<float>& m,
                    const StageSpec& sp, float* out) {
  MfmaArgs a = mfma_args(m.B, m.D, m.d_in, m.H, m.cnf, m.st.status, m.st.y,
                         m.K, m.Y7, m.hs, m.st.t, m.eps, im.mw);
  a.n = sp.n;
  for (int j = 0; j < 6; ++j) {
    a.kidx[j] = sp.kidx[j];
    a.coef[j] = float(sp.coef[j]);
  }
  a.c = sp.c;
  a.write_y7 = sp.yout != nullptr;
  a.Y7 = static_cast<float*>(sp.yout);
  a.out = out;
  a.act_out = static_cast<float*>(sp.act_out);
  a.waves = get_tune(im.cfg).waves;
  return a;
}

template <>
hipError_t field<float>(ModImpl& im, const Mod<float>& m, const StageSpec& sp,
                        float* out, hipStream_t s) {
  if (im.mw.packed != nullptr)
    return launch_field_mfma(stage_args(im, m, sp, out), 0, s);
  return launch_field_fma<float>(m, sp, out, s);
}

// The whole solve (up to budget attempts per instance) in one launch of the
// fused kernel.
template <class M>
hipError_t run_fused(const ModImpl& im, const Mod<float>& m, int budget,
                     hipStream_t s) {
  FusedArgs f{};
  for (int st = 1; st < 7; ++st) {
    StageSpec sp = stage_spec<M>(st);
    if (st == 6) sp.yout = m.Y7;
    f.st[st - 1] = stage_args(im, m, sp, m.K + (size_t)st * m.B * m.D);
    f.st[st - 1].kslot = st;
  }
  f.budget = budget;
  return fused_launch<M>(m, f, im.mw.f32, im.mw.plain, s);
}

template <typename R>
dim3 row_grid(int B) {
  return dim3((B + 3) / 4);
}

template <typename R, class M>
hipError_t round_launch(ModImpl& im, Mod<R>& m, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int st = 1; st < 7 && e == hipSuccess; ++st) {
    StageSpec sp = stage_spec<M>(st);
    if (st == 6) sp.yout = m.Y7;
    e = field<R>(im, m, sp, m.K + (size_t)st * m.B * m.D, s);
  }
  if (e != hipSuccess) return e;
  // several rows per wavefront while each lane keeps a few columns: more
  // rows' loads in flight per wavefront and a shorter cross-lane sum (2^20
  // instances, D = 64: 16 lanes a row 0.73 ms, 8 lanes 0.80, 32 lanes 1.05,
  // 64 lanes 1.60 per launch)
  if (m.D <= 64) {
    const dim3 g = commit_grid(m.B, 16);
    if (m.keep)
      hipLaunchKernelGGL((commit_kernel<R, M, true, 16>), g, dim3(256), 0, s,
                         m);
    else
      hipLaunchKernelGGL((commit_kernel<R, M, false, 16>), g, dim3(256), 0, s,
                         m);
  } else if (m.D <= 128) {
    const dim3 g = commit_grid(m.B, 8);
    if (m.keep)
      hipLaunchKernelGGL((commit_kernel<R, M, true, 32>), g, dim3(256), 0, s,
                         m);
    else
      hipLaunchKernelGGL((commit_kernel<R, M, false, 32>), g, dim3(256), 0, s,
                         m);
  } else if (m.keep) {
    hipLaunchKernelGGL((commit_kernel<R, M, true, 64>), commit_grid(m.B, 4),
                       dim3(256), 0, s, m);
  } else {
    hipLaunchKernelGGL((commit_kernel<R, M, false, 64>), commit_grid(m.B, 4),
                       dim3(256), 0, s, m);
  }
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
  if constexpr (std::is_same<R, float>::value) {
    if (im.mw.packed != nullptr && !m.keep)
      return im.cfg.method == BODE_TSIT5 ? run_fused<Tsit5>(im, m, budget, s)
                                         : run_fused<Dopri5>(im, m, budget, s);
  }
  auto rounds = [&](int n, hipStream_t q) -> hipError_t {
    for (int r = 0; r < n; ++r) {
      hipError_t e = im.cfg.method == BODE_TSIT5
                         ? round_launch<R, Tsit5>(im, m, q)
                         : round_launch<R, Dopri5>(im, m, q);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  // rounds per running-count read-back (and per captured graph): tuned,
  // else kRoundsPerSync; fixed for the handle once its graph is captured
  if (im.rounds_per_sync == 0) {
    const int t = get_tune(im.cfg).rounds;
    im.rounds_per_sync = t > 0 ? t : kRoundsPerSync;
  }
  const int K = im.rounds_per_sync;
  int done = 0;
  while (done < budget) {
    const int chunk = budget - done < K ? budget - done : K;
    hipError_t e;
    if (chunk == K && !im.cfg.eager) {
      // a full block of rounds: one graph launch (captured on first use)
      e = im.rounds_exec != nullptr
              ? hipSuccess
              : capture(im, [&](hipStream_t q) { return rounds(K, q); },
                        &im.rounds_exec);
      if (e == hipSuccess) e = hipGraphLaunch(im.rounds_exec, s);
    } else {
      e = rounds(chunk, s);
    }
    if (e != hipSuccess) return e;
    done += chunk;
    // instances still running: one ballot count per wavefront (a count per
    // row in the commit would serialise B atomics on one counter)
    e = launch_fill_i32(m.n_running, 1, 0, s);
    if (e == hipSuccess)
      e = launch_count_equal(m.st.status, m.B, kRunning, m.n_running, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(im.host_running, m.n_running,
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
    Back<double> bk{};
    const size_t n = lay_mod<double>(c, base, mp ? &m : nullptr, nullptr, &bk);
    if (mp) {
      ModImpl* im = new ModImpl();
      im->md = m;
      im->bd = bk;
      im->is64 = true;
      mp->impl = im;
    }
    return n;
  }
  Mod<float> m{};
  MfmaWeights w{};
  Back<float> bk{};
  const size_t n = lay_mod<float>(c, base, mp ? &m : nullptr, &w, &bk);
  if (mp) {
    ModImpl* im = new ModImpl();
    im->mf = m;
    im->bf = bk;
    im->mw = w;
    mp->impl = im;
  }
  return n;
}

// Pinned host words for the running-count read-backs, two per handle, kept
// in a process-wide free list (pinned allocations are slow; handles come
// and go every training step).
namespace {
std::mutex g_pin_mu;
std::vector<int32_t*> g_pin_free;

hipError_t pinned_take(int32_t** out) {
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (!g_pin_free.empty()) {
      *out = g_pin_free.back();
      g_pin_free.pop_back();
      return hipSuccess;
    }
  }
  return hipHostMalloc(reinterpret_cast<void**>(out), 64,
                       hipHostMallocDefault);
}

void pinned_give(int32_t* p) {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.push_back(p);
}
}  // namespace

hipError_t modular_init(ModularPlan& mp, const bode_config& c,
                        const bode_problem& p, hipStream_t s) {
  ModImpl* im = static_cast<ModImpl*>(mp.impl);
  if (!im) return hipErrorInvalidValue;
  im->cfg = c;
  im->p = p;
  hipError_t e = pinned_take(&im->host_running);
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
    mp.e_rec = m.e_rec;
    mp.n_running = m.n_running;
  };
  if (im->is64) {
    fill_mod<double>(&im->md, c, p);
    publish(im->md);
    return init_launch<double>(*im, im->md, s);
  }
  fill_mod<float>(&im->mf, c, p);
  publish(im->mf);
  if (im->mw.packed != nullptr) {
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

// ---- discrete adjoint ----------------------------------------------------------
//
// Paper section 4.2 trains its graph model by backpropagating through the
// solver.  This is the discrete adjoint of the accepted steps with their sizes
// and decisions frozen (rejected attempts and the controller carry no
// gradient).  For step n (sizes h_n, start t_n, state y_n):
//   Y_1 = y_n, k_s = f(t_n + c_s h, Y_s), Y_s = y_n + h sum_{j<s} a_sj k_j,
//   y_n+1 = Y_7, dense output y(theta) = y_n + h sum_j w_j(theta) k_j.
// Walking the stages backwards: kappa_j collects h w_j(theta_e) g_e from the
// step's evaluation times; stage 7 only feeds the interpolant, so
// Lambda = lambda + J_7^T kappa_7 and kappa_j += h a_7j Lambda; then for
// s = 6..1: mu_s = J_s^T kappa_s, kappa_j += h a_sj mu_s (j < s); finally
// lambda_n = Lambda + sum_s mu_s + sum_e g_e.  Parameter gradients collect
// (df/dtheta)^T kappa_s at every stage.  y_n comes from a checkpoint every k
// accepted steps and is recomputed in between (the field kernel of the
// forward replays the recorded steps).

struct VjpSpec {
  int s;  // stage 1..7
  int n;
  int kidx[6];
  double coef[6];
  double c;
  // Continuous adjoint: mu_s = J^T kappa_s is stored here ([B, D]) and the
  // discrete adjoint's row updates are skipped.
  void* mu_out;
  // First tape row of this step (the tape holds several steps, 7 Bs rows
  // each; stage s starts at kbase + (s - 1) Bs).
  long kbase;
  // Matrix-core fields with the segment store: the stage input and the
  // stored hidden-layer values of this stage (null: Ys and recomputation).
  const void* Y;
  const float* act_in;
};

template <typename R>
__global__ void adj_prep(Mod<R> m, Back<R> b) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= m.B) return;
  const int status = m.st.status[row];
  const int natt = m.st.n_att[row];
  int N = 0;
  if (status != kInvalid) {
    if (natt > b.cap) {
      atomicOr(&b.flags[1], 1);
    } else {
      for (int q = 0; q < natt; ++q) {
        const double h = m.h_rec[(long)row * m.rec_cap + q];
        if (h > 0.0) b.hacc[(long)row * b.cap + N++] = h;
      }
    }
  }
  double* tn = b.tn + (long)row * (b.cap + 1);
  tn[0] = m.t0[row];
  for (int q = 0; q < N; ++q)
    tn[q + 1] = (q == N - 1 && status == kSuccess) ? m.t_end[row]
                                                    : tn[q] + b.hacc[(long)row * b.cap + q];
  int cursor = 0;
  const double* te = m.t_eval + (long)row * m.E;
  int32_t* own = b.owner + (long)row * (m.E > 0 ? m.E : 1);
  while (cursor < m.E && te[cursor] <= tn[0]) own[cursor++] = -1;
  for (int q = 0; q < N; ++q)
    while (cursor < m.E && te[cursor] <= tn[q + 1]) own[cursor++] = q;
  while (cursor < m.E) own[cursor++] = -2;  // never reached
  b.nacc[row] = N;
  atomicMax(&b.flags[0], N);
}

// Step n of every instance that has one: status view, h_n, t_n; optionally
// y_n -> Y_1 (the differentiated step keeps its stage inputs).
template <typename R>
__global__ void adj_setup(Mod<R> m, Back<R> b, int n, const R* yn, R* y1) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= m.B) return;
  const bool on = n < b.nacc[row];
  if (lane == 0) {
    b.act[row] = on ? kRunning : kSuccess;
    b.bh[row] = on ? R(b.hacc[(long)row * b.cap + n]) : R(0);
    b.bt[row] = on ? b.tn[(long)row * (b.cap + 1) + n] : 0.0;
  }
  if (y1 != nullptr && on)
    for (int c = lane; c < m.D; c += 64)
      y1[(long)row * m.D + c] = yn[(long)row * m.D + c];
}

// Segment start: y_{seg k} from the checkpoints (or y0).
template <typename R>
__global__ void adj_load_ckpt(Mod<R> m, Back<R> b, int seg, R* dst) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long total = (long)m.B * m.D;
  if (i >= total) return;
  const long row = i / m.D, c = i % m.D;
  dst[i] = m.ckpt != nullptr ? m.ckpt[(row * m.ck_cap + seg) * m.D + c]
                             : m.y0[i];
}

// Cotangents injected by the dense outputs of step n; with setup, also
// the step view of step n (adj_setup without the state copy).
template <typename R, class M>
__global__ void adj_dense(Mod<R> m, Back<R> b, int n, const R* g_eval,
                          int setup) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= m.B) return;
  const int D = m.D, B = m.B;
  if (setup && lane == 0) {
    const bool on = n < b.nacc[row];
    b.act[row] = on ? kRunning : kSuccess;
    b.bh[row] = on ? R(b.hacc[(long)row * b.cap + n]) : R(0);
    b.bt[row] = on ? b.tn[(long)row * (b.cap + 1) + n] : 0.0;
  }
  for (int c = lane; c < D; c += 64) {
    b.lamn[(long)row * D + c] = R(0);
    for (int j = 0; j < 7; ++j) b.kap[((long)j * B + row) * D + c] = R(0);
  }
  if (!(n < b.nacc[row]) || m.E == 0) return;
  const double h = b.hacc[(long)row * b.cap + n];
  const double t = b.tn[(long)row * (b.cap + 1) + n];
  const int32_t* own = b.owner + (long)row * m.E;
  for (int e = 0; e < m.E; ++e) {
    if (own[e] != n) continue;
    const R th = R((m.t_eval[(long)row * m.E + e] - t) / h);
    R w[7];
#pragma unroll
    for (int j = 0; j < 7; ++j)
      w[j] = th * (R(M::P[j][0]) +
                   th * (R(M::P[j][1]) + th * (R(M::P[j][2]) + th * R(M::P[j][3]))));
    for (int c = lane; c < D; c += 64) {
      const R g = g_eval[((long)row * m.E + e) * D + c];
      for (int j = 0; j < 7; ++j)
        b.kap[((long)j * B + row) * D + c] += R(h) * w[j] * g;
      b.lamn[(long)row * D + c] += g;
    }
  }
}

// mu_s = J_f(Y_s)^T kappa_s for a tile of instances (the field's layers are
// recomputed in LDS), the stage's tape entries for the parameter gradient,
// and the row updates of kappa, lambda.
template <typename R, int ROWS>
__global__ __launch_bounds__(256) void vjp_kernel(Mod<R> m, Back<R> b,
                                                  VjpSpec sp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* sm = reinterpret_cast<R*>(smem_raw);
  const int B = m.B, D = m.D, H = m.H, din = m.d_in, n0 = din + 1;
  const int cnf = m.cnf;
  R* X = sm;                  // [ROWS][n0]
  R* Kp = X + ROWS * n0;      // [ROWS][D]  kappa_s
  R* A1 = Kp + ROWS * D;      // [ROWS][H]
  R* A2 = A1 + ROWS * H;
  R* G1 = A2 + ROWS * H;      // pbar1
  R* G2 = G1 + ROWS * H;      // pbar2
  R* MU = G2 + ROWS * H;      // [ROWS][din]
  R* dX = MU + ROWS * din;    // CNF: probe, tangents and their cotangents
  R* DP1 = dX + ROWS * n0;
  R* DA1 = DP1 + ROWS * H;
  R* DP2 = DA1 + ROWS * H;
  R* DA2 = DP2 + ROWS * H;
  R* DG1 = DA2 + ROWS * H;    // dpbar1
  R* DG2 = DG1 + ROWS * H;    // dpbar2
  __shared__ int any;
  const int s = sp.s;
  const R* Yin = b.Ys + (long)(s - 1) * B * D;
  const R* Kin = b.kap + (long)(s - 1) * B * D;
  const int ntiles = (B + ROWS - 1) / ROWS;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int r0 = tile * ROWS;
    __syncthreads();
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    if (threadIdx.x < ROWS && r0 + threadIdx.x < B &&
        b.act[r0 + threadIdx.x] == kRunning)
      any = 1;
    __syncthreads();
    if (!any) continue;
    for (int idx = threadIdx.x; idx < ROWS * D; idx += blockDim.x) {
      const int r = idx / D, c = idx % D, row = r0 + r;
      const bool on = row < B && b.act[row] == kRunning;
      Kp[idx] = on ? Kin[(long)row * D + c] : R(0);
      if (c < din) {
        X[r * n0 + c] = on ? Yin[(long)row * D + c] : R(0);
        if (cnf) dX[r * n0 + c] = on ? m.eps[(long)row * D + c] : R(0);
      }
    }
    for (int r = threadIdx.x; r < ROWS; r += blockDim.x) {
      const int row = r0 + r;
      const bool on = row < B && b.act[row] == kRunning;
      X[r * n0 + din] = on ? R(b.bt[row] + sp.c * double(b.bh[row])) : R(0);
      if (cnf) dX[r * n0 + din] = R(0);
    }
    __syncthreads();
    // forward: a1, a2 (and the tangents for the CNF)
    for (int j = threadIdx.x; j < H; j += blockDim.x) {
      for (int r = 0; r < ROWS; ++r) {
        R acc = m.b1[j], tac = R(0);
        for (int i = 0; i < n0; ++i) {
          acc += X[r * n0 + i] * m.W1[(long)i * H + j];
          if (cnf && i < din) tac += dX[r * n0 + i] * m.W1[(long)i * H + j];
        }
        const R a = tanh(acc);
        A1[r * H + j] = a;
        if (cnf) {
          DP1[r * H + j] = tac;
          DA1[r * H + j] = (R(1) - a * a) * tac;
        }
      }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < H; j += blockDim.x) {
      for (int r = 0; r < ROWS; ++r) {
        R acc = m.b2[j], tac = R(0);
        for (int i = 0; i < H; ++i) {
          acc += A1[r * H + i] * m.W2[(long)i * H + j];
          if (cnf) tac += DA1[r * H + i] * m.W2[(long)i * H + j];
        }
        const R a = tanh(acc);
        A2[r * H + j] = a;
        if (cnf) {
          DP2[r * H + j] = tac;
          DA2[r * H + j] = (R(1) - a * a) * tac;
        }
      }
    }
    __syncthreads();
    // output layer backwards: gbar = kappa_z, dgbar = -kappa_l eps
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
      for (int r = 0; r < ROWS; ++r) {
        R s1 = R(0), s2 = R(0);
        for (int j = 0; j < din; ++j) {
          const R w = m.W3[(long)i * din + j];
          s1 += w * Kp[r * D + j];
          if (cnf) s2 += w * (-Kp[r * D + din] * dX[r * n0 + j]);
        }
        const R a = A2[r * H + i], g = R(1) - a * a;
        if (cnf) {
          const R dpb = g * s2;
          DG2[r * H + i] = dpb;
          s1 += R(-2) * a * DP2[r * H + i] * s2;
        }
        G2[r * H + i] = g * s1;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
      for (int r = 0; r < ROWS; ++r) {
        R s1 = R(0), s2 = R(0);
        for (int j = 0; j < H; ++j) {
          const R w = m.W2[(long)i * H + j];
          s1 += w * G2[r * H + j];
          if (cnf) s2 += w * DG2[r * H + j];
        }
        const R a = A1[r * H + i], g = R(1) - a * a;
        if (cnf) {
          DG1[r * H + i] = g * s2;
          s1 += R(-2) * a * DP1[r * H + i] * s2;
        }
        G1[r * H + i] = g * s1;
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < ROWS * din; idx += blockDim.x) {
      const int r = idx / din, c = idx % din;
      R acc = R(0);
      for (int j = 0; j < H; ++j) acc += m.W1[(long)c * H + j] * G1[r * H + j];
      MU[idx] = acc;
    }
    // tape of this stage: layer inputs (+ bias feature) and cotangents
    {
      const long Bs = cnf ? 2L * B : (long)B;
      const long kb = sp.kbase + (long)(s - 1) * Bs;
      const int l1 = n0 + 1, lh = H + 1;
      for (int idx = threadIdx.x; idx < ROWS * l1; idx += blockDim.x) {
        const int r = idx / l1, f = idx % l1, row = r0 + r;
        if (row >= B) continue;
        const long k = kb + row;
        b.T1in[k * l1 + f] = f < n0 ? X[r * n0 + f] : R(1);
        if (cnf) b.T1in[(k + B) * l1 + f] = f < din ? dX[r * n0 + f] : R(0);
      }
      for (int idx = threadIdx.x; idx < ROWS * lh; idx += blockDim.x) {
        const int r = idx / lh, f = idx % lh, row = r0 + r;
        if (row >= B) continue;
        const long k = kb + row;
        b.T2in[k * lh + f] = f < H ? A1[r * H + f] : R(1);
        b.T3in[k * lh + f] = f < H ? A2[r * H + f] : R(1);
        if (f < H) {
          b.T1g[k * H + f] = G1[r * H + f];
          b.T2g[k * H + f] = G2[r * H + f];
        }
        if (cnf) {
          b.T2in[(k + B) * lh + f] = f < H ? DA1[r * H + f] : R(0);
          b.T3in[(k + B) * lh + f] = f < H ? DA2[r * H + f] : R(0);
          if (f < H) {
            b.T1g[(k + B) * H + f] = DG1[r * H + f];
            b.T2g[(k + B) * H + f] = DG2[r * H + f];
          }
        }
      }
      for (int idx = threadIdx.x; idx < ROWS * din; idx += blockDim.x) {
        const int r = idx / din, f = idx % din, row = r0 + r;
        if (row >= B) continue;
        const long k = kb + row;
        b.T3g[k * din + f] = Kp[r * D + f];
        if (cnf) b.T3g[(k + B) * din + f] = -Kp[r * D + din] * dX[r * n0 + f];
      }
    }
    __syncthreads();
    // row updates: kappa_j += h a_sj mu (Lambda at stage 7), lambda sums
    for (int idx = threadIdx.x; idx < ROWS * D; idx += blockDim.x) {
      const int r = idx / D, c = idx % D, row = r0 + r;
      if (row >= B || b.act[row] != kRunning) continue;
      if (sp.mu_out != nullptr) {
        static_cast<R*>(sp.mu_out)[(long)row * D + c] =
            c < din ? MU[r * din + c] : R(0);
        continue;
      }
      const R h = b.bh[row];
      R mu = c < din ? MU[r * din + c] : R(0);
      const long o = (long)row * D + c;
      if (s == 7) {
        mu = b.lam[o] + mu;  // Lambda
        b.lam[o] = mu;
      }
      b.lamn[o] += mu;
      for (int j = 0; j < sp.n; ++j)
        b.kap[((long)sp.kidx[j] * B + row) * D + c] += h * R(sp.coef[j]) * mu;
      if (s == 1) b.lam[o] = b.lamn[o];
    }
  }
}

template <typename R>
size_t vjp_smem(int rows, int n0, int D, int H, int din, int cnf) {
  size_t per = (size_t)n0 + D + 4 * (size_t)H + din;
  if (cnf) per += (size_t)n0 + 6 * (size_t)H;
  return sizeof(R) * rows * per;
}

template <typename R>
hipError_t launch_vjp(const Mod<R>& m, const Back<R>& b, const VjpSpec& sp,
                      hipStream_t s) {
  const int n0 = m.d_in + 1;
  int rows = 8;
  while (rows > 1 && vjp_smem<R>(rows, n0, m.D, m.H, m.d_in, m.cnf) > 65536)
    rows /= 2;
  const size_t sm = vjp_smem<R>(rows, n0, m.D, m.H, m.d_in, m.cnf);
  if (sm > 65536) return hipErrorInvalidValue;
  const int ntiles = (m.B + rows - 1) / rows;
  const dim3 g(ntiles), blk(256);
  switch (rows) {
    case 8:
      hipLaunchKernelGGL((vjp_kernel<R, 8>), g, blk, sm, s, m, b, sp);
      break;
    case 4:
      hipLaunchKernelGGL((vjp_kernel<R, 4>), g, blk, sm, s, m, b, sp);
      break;
    case 2:
      hipLaunchKernelGGL((vjp_kernel<R, 2>), g, blk, sm, s, m, b, sp);
      break;
    default:
      hipLaunchKernelGGL((vjp_kernel<R, 1>), g, blk, sm, s, m, b, sp);
  }
  return hipGetLastError();
}

// The matrix-core VJP kernel's arguments for stage sp.s of the step.
MfmaVjpArgs vjp_args(const ModImpl& im, const Mod<float>& m,
                     const Back<float>& b, const VjpSpec& sp) {
  MfmaVjpArgs a{};
  a.B = m.B;
  a.D = m.D;
  a.din = m.d_in;
  a.H = m.H;
  a.cnf = m.cnf;
  a.act = b.act;
  a.Y = sp.Y != nullptr ? static_cast<const float*>(sp.Y)
                        : b.Ys + (long)(sp.s - 1) * m.B * m.D;
  a.act_in = sp.act_in;
  a.kap_s = b.kap + (long)(sp.s - 1) * m.B * m.D;
  a.eps = m.eps;
  a.bh = b.bh;
  a.bt = b.bt;
  a.c = sp.c;
  a.w = im.mw;
  a.T1in = b.T1in;
  a.T1g = b.T1g;
  a.T2in = b.T2in;
  a.T2g = b.T2g;
  a.T3in = b.T3in;
  a.T3g = b.T3g;
  a.K = b.K;
  a.kb = sp.kbase + (long)(sp.s - 1) * (m.cnf ? 2L * m.B : (long)m.B);
  a.s = sp.s;
  a.n = sp.n;
  for (int j = 0; j < sp.n; ++j) {
    a.kidx[j] = sp.kidx[j];
    a.coef[j] = float(sp.coef[j]);
  }
  a.lam = b.lam;
  a.lamn = b.lamn;
  a.kap = b.kap;
  a.mu_out = static_cast<float*>(sp.mu_out);
  return a;
}

// Matrix-core modes: the stage's VJP on MFMA (BF16: BF16 weights, three-way
// split activations and cotangents; FP32: FP32 operands; both accumulate in
// FP32); else the FMA kernel.
template <typename R>
hipError_t vjp(const ModImpl& im, const Mod<R>& m, const Back<R>& b,
               const VjpSpec& sp, hipStream_t s) {
  if constexpr (std::is_same<R, float>::value) {
    if (im.mw.packedT != nullptr)
      return launch_vjp_mfma(vjp_args(im, m, b, sp), s);
  }
  return launch_vjp<R>(m, b, sp, s);
}


template <typename R>
__global__ void fill_r(R* p, long n, R v) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename R>
__global__ void copy_r(R* dst, const R* src, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Parameter gradient of one step from its tape: for each layer,
// C[m][n] += sum_k Tin[k][m] Tg[k][n] over the k range of this split, added
// into slot[split] (one owner per entry, so the sum is deterministic).  The
// augmented C = [W; b] of the three layers, concatenated, is dtheta.  Tape
// rows are M (inputs) and N (cotangents) wide.  blockIdx.y selects one of
// several independent products of the same shape (the stages of an attempt):
// its tapes and slots start sin, sg and sslot elements further on.
template <typename R>
__global__ __launch_bounds__(256) void grad_gemm(const R* Tin, const R* Tg,
                                                 long K, int M, int N, int S,
                                                 R* slots, long P, long off,
                                                 long sin, long sg,
                                                 long sslot) {
  constexpr int TM = 64, TN = 64, TK = 16;
  Tin += blockIdx.y * sin;
  Tg += blockIdx.y * sg;
  slots += blockIdx.y * sslot;
  __shared__ R As[TK][TM + 4];
  __shared__ R Bs[TK][TN + 4];
  const int tiles_n = (N + TN - 1) / TN;
  const int tile = blockIdx.x / S, split = blockIdx.x % S;
  const int m0 = (tile / tiles_n) * TM, n0 = (tile % tiles_n) * TN;
  const long kc = ((K + S - 1) / S + TK - 1) / TK * TK;
  const long k0 = split * kc, k1 = k0 + kc < K ? k0 + kc : K;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  R acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = R(0);
  for (long kk = k0; kk < k1; kk += TK) {
    for (int e = threadIdx.x; e < TK * TM; e += 256) {
      const int kl = e / TM, c = e % TM;
      const long k = kk + kl;
      const int m = m0 + c, n = n0 + c;
      As[kl][c] = (m < M && k < k1) ? Tin[k * M + m] : R(0);
      Bs[kl][c] = (n < N && k < k1) ? Tg[k * N + n] : R(0);
    }
    __syncthreads();
#pragma unroll
    for (int kl = 0; kl < TK; ++kl) {
      R a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[kl][ty * 4 + i];
        bb[i] = Bs[kl][tx * 4 + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * bb[j];
    }
    __syncthreads();
  }
  R* slot = slots + (long)split * P + off;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
      if (m < M && n < N) slot[(long)m * N + n] += acc[i][j];
    }
}

// FP32 tapes: the same product on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32: exact FP32 products, FP32 accumulation).  Four
// wavefronts in a 2 x 2 grid, each WM x WN 16x16 tiles, so a workgroup
// covers (32 WM) x (32 WN) of C: 128 x 128 for the square layers, 32 x 128
// or 128 x 32 where the layer has few inputs or outputs.  Both operands
// pass through LDS 16 tape rows at a time (contiguous runs of features).
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Workgroup bx of the product (tile bx / S, k-split bx % S); As, Bs: LDS of
// at least 16 (32 WM + 16) and 16 (32 WN + 16) floats.
template <int WM, int WN>
__device__ __forceinline__ void grad_gemm_tile(int bx, const float* Tin,
                                               const float* Tg, long K, int M,
                                               int N, int S, float* slots,
                                               long P, long off, float* As,
                                               float* Bs) {
  constexpr int TM = 32 * WM, TN = 32 * WN, TK = 16;
  // row pitch 16 floats past the tile: the four lane groups of an operand
  // read land 16 banks apart
  constexpr int LA = TM + 16, LB = TN + 16;
  constexpr int NA = TK * TM / 256, NB = TK * TN / 256;  // loads per thread
  const int tiles_n = (N + TN - 1) / TN;
  const int tile = bx / S, split = bx % S;
  const int m0 = (tile / tiles_n) * TM, n0 = (tile % tiles_n) * TN;
  const long kc = ((K + S - 1) / S + TK - 1) / TK * TK;
  const long k0 = split * kc, k1 = k0 + kc < K ? k0 + kc : K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 16 * WM, wn = (wave & 1) * 16 * WN;
  const int lr = lane & 15, lk = lane >> 4;
  f32x4_t acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  // the next 16 tape rows are loaded into registers while the current ones
  // are multiplied
  float ra[NA], rb[NB];
  auto fetch = [&](long kk) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q, kl = e / TM, c = e % TM;
      const long k = kk + kl;
      const int m = m0 + c;
      ra[q] = (m < M && k < k1) ? Tin[k * M + m] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q, kl = e / TN, c = e % TN;
      const long k = kk + kl;
      const int n = n0 + c;
      rb[q] = (n < N && k < k1) ? Tg[k * N + n] : 0.f;
    }
  };
  if (k0 < k1) fetch(k0);
  for (long kk = k0; kk < k1; kk += TK) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      As[(e / TM) * LA + e % TM] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      Bs[(e / TN) * LB + e % TN] = rb[q];
    }
    __syncthreads();
    if (kk + TK < k1) fetch(kk + TK);
#pragma unroll
    for (int k4 = 0; k4 < TK; k4 += 4) {
      float a[WM], b[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) a[i] = As[(k4 + lk) * LA + wm + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < WN; ++j) b[j] = Bs[(k4 + lk) * LB + wn + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
          acc[i][j] =
              __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  float* slot = slots + (long)split * P + off;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + i * 16 + lk * 4 + v;
        const int n = n0 + wn + j * 16 + lr;
        if (m < M && n < N) slot[(long)m * N + n] += acc[i][j][v];
      }
}

template <int WM, int WN>
__global__ __launch_bounds__(256) void grad_gemm_mfma(
    const float* Tin, const float* Tg, long K, int M, int N, int S,
    float* slots, long P, long off, long sin, long sg, long sslot) {
  __shared__ float As[16 * (32 * WM + 16)];
  __shared__ float Bs[16 * (32 * WN + 16)];
  grad_gemm_tile<WM, WN>(blockIdx.x, Tin + blockIdx.y * sin,
                         Tg + blockIdx.y * sg, K, M, N, S,
                         slots + blockIdx.y * sslot, P, off, As, Bs);
}

// Tile shapes of the FP32 matrix-core gradient products.
enum GemmShape { kG14, kG41, kG42, kG34, kG44 };

// The products of one chunk (one per layer, different shapes) in one
// launch: workgroups [0, nblk[0]) are product 0's, and so on, each
// product's workgroups exactly those of its own launch.
struct GemmGroup {
  const float* Tin[3];
  const float* Tg[3];
  int M[3], N[3], S[3], shape[3], nblk[3];
  long off[3];
  long K, P;
  float* slots;
};

__global__ __launch_bounds__(256) void grad_gemm_group(GemmGroup g) {
  __shared__ float As[16 * (128 + 16)];
  __shared__ float Bs[16 * (128 + 16)];
  int b = blockIdx.x, j = 0;
  while (j < 2 && b >= g.nblk[j]) b -= g.nblk[j++];
  const float *Tin = g.Tin[j], *Tg = g.Tg[j];
  const int M = g.M[j], N = g.N[j], S = g.S[j];
  switch (g.shape[j]) {
    case kG14:
      grad_gemm_tile<1, 4>(b, Tin, Tg, g.K, M, N, S, g.slots, g.P, g.off[j], As, Bs);
      break;
    case kG41:
      grad_gemm_tile<4, 1>(b, Tin, Tg, g.K, M, N, S, g.slots, g.P, g.off[j], As, Bs);
      break;
    case kG42:
      grad_gemm_tile<4, 2>(b, Tin, Tg, g.K, M, N, S, g.slots, g.P, g.off[j], As, Bs);
      break;
    case kG34:
      grad_gemm_tile<3, 4>(b, Tin, Tg, g.K, M, N, S, g.slots, g.P, g.off[j], As, Bs);
      break;
    default:
      grad_gemm_tile<4, 4>(b, Tin, Tg, g.K, M, N, S, g.slots, g.P, g.off[j], As, Bs);
  }
}

// Large layers (both sides >= 256, long tapes): 256 x 256 tiles of C over
// 8 wavefronts (4 x 2, each 64 x 128 = 4 x 8 MFMA tiles), so each tape row
// is read by only M/256 + N/256 workgroups.  C rows [0, M) are the weight
// rows of the layer; its bias row (input feature M, the last of the ldin
// columns) is summed by the first row of tiles from the same staged
// cotangent block, on plain FMAs.
__global__ __launch_bounds__(512) void grad_gemm_big(
    const float* Tin, int ldin, const float* Tg, long K, int M, int N, int S,
    float* slots, long P, long off, long sin, long sg, long sslot) {
  constexpr int TT = 256, TK = 16, LA = TT + 16;
  Tin += blockIdx.y * sin;
  Tg += blockIdx.y * sg;
  slots += blockIdx.y * sslot;
  constexpr int NL = TK * TT / 512;  // loads per thread per operand
  __shared__ float As[TK * LA];
  __shared__ float Bs[TK * LA];
  __shared__ float Bias[TK];
  const int tiles_n = (N + TT - 1) / TT;
  const int tile = blockIdx.x / S, split = blockIdx.x % S;
  const int m0 = (tile / tiles_n) * TT, n0 = (tile % tiles_n) * TT;
  const bool brow = m0 == 0;
  const long kc = ((K + S - 1) / S + TK - 1) / TK * TK;
  const long k0 = split * kc, k1 = k0 + kc < K ? k0 + kc : K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 128;
  const int lr = lane & 15, lk = lane >> 4;
  f32x4_t acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  float ra[NL], rb[NL], rbias = 0.f;
  auto fetch = [&](long kk) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + 512 * q, kl = e / TT, c = e % TT;
      const long k = kk + kl;
      ra[q] = (m0 + c < M && k < k1) ? Tin[k * ldin + m0 + c] : 0.f;
      rb[q] = (n0 + c < N && k < k1) ? Tg[k * N + n0 + c] : 0.f;
    }
    if (brow && tid < TK)
      rbias = kk + tid < k1 ? Tin[(kk + tid) * ldin + M] : 0.f;
  };
  if (k0 < k1) fetch(k0);
  for (long kk = k0; kk < k1; kk += TK) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + 512 * q;
      As[(e / TT) * LA + e % TT] = ra[q];
      Bs[(e / TT) * LA + e % TT] = rb[q];
    }
    if (brow && tid < TK) Bias[tid] = rbias;
    __syncthreads();
    if (kk + TK < k1) fetch(kk + TK);
#pragma unroll
    for (int k4 = 0; k4 < TK; k4 += 4) {
      float a[4], b[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[(k4 + lk) * LA + wm + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < 8; ++j) b[j] = Bs[(k4 + lk) * LA + wn + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          acc[i][j] =
              __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (brow && tid < TT) {
#pragma unroll
      for (int kl = 0; kl < TK; ++kl) bacc += Bias[kl] * Bs[kl * LA + tid];
    }
    __syncthreads();
  }
  float* slot = slots + (long)split * P + off;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + i * 16 + lk * 4 + v;
        const int n = n0 + wn + j * 16 + lr;
        if (m < M && n < N) slot[(long)m * N + n] += acc[i][j][v];
      }
  if (brow && tid < TT && n0 + tid < N) slot[(long)M * N + n0 + tid] += bacc;
}

// BF16 mode's large tape products on the BF16 matrix cores.  Each FP32
// tape value x is split into two BF16 terms, hi (x's top 16 bits) and lo
// (the top 16 bits of the exact residual x - hi), and C += Ah Bh + Ah Bl +
// Al Bh (v_mfma_f32_16x16x32_bf16, FP32 accumulation): the dropped Al Bl
// and the truncated residuals leave about 2^-16 of each product, far below
// the BF16 weights' own rounding.  Tiles of 128 (m) x 256 (n) of C over 8
// wavefronts (2 x 4, each 64 x 64 = 4 x 4 MFMA tiles); 32 tape rows a
// stage, both operands stored in LDS k-contiguous ([m][k] and [n][k], row
// pitch 40 halves) so that a lane's eight k values are one 16-byte read;
// each thread loads eight rows of one feature (coalesced over features)
// and writes its eight k values as one 16-byte store per term; the next
// stage's rows are loaded during the products.  C rows are all M input
// features (the bias feature included), as in grad_gemm_mfma.
constexpr int kBgM = 128, kBgN = 256, kBgK = 32, kBgP = kBgK + 8;

__device__ __forceinline__ void split_store8(uint16_t* hi, uint16_t* lo,
                                             const float (&v)[8]) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t w[2], r[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint32_t u = __float_as_uint(v[2 * j + q]);
      const float res = v[2 * j + q] - __uint_as_float(u & 0xffff0000u);
      w[q] = u >> 16;
      r[q] = __float_as_uint(res) >> 16;
    }
    h[j] = w[0] | (w[1] << 16);
    l[j] = r[0] | (r[1] << 16);
  }
  *reinterpret_cast<uint4*>(hi) = make_uint4(h[0], h[1], h[2], h[3]);
  *reinterpret_cast<uint4*>(lo) = make_uint4(l[0], l[1], l[2], l[3]);
}

__global__ __launch_bounds__(512) void grad_gemm_bf16(
    const float* Tin, const float* Tg, long K, int M, int N, int S,
    float* slots, long P, long off) {
  __shared__ __align__(16) uint16_t Ah[kBgM * kBgP];
  __shared__ __align__(16) uint16_t Al[kBgM * kBgP];
  __shared__ __align__(16) uint16_t Bh[kBgN * kBgP];
  __shared__ __align__(16) uint16_t Bl[kBgN * kBgP];
  const int tiles_n = (N + kBgN - 1) / kBgN;
  const int tile = blockIdx.x / S, split = blockIdx.x % S;
  const int m0 = (tile / tiles_n) * kBgM, n0 = (tile % tiles_n) * kBgN;
  const long kc = ((K + S - 1) / S + kBgK - 1) / kBgK * kBgK;
  const long k0 = split * kc, k1 = k0 + kc < K ? k0 + kc : K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 2) * 64, wn = (wave & 3) * 64;
  const int r = lane & 15, kq = (lane >> 4) * 8;
  // staging: A feature tid % 128, k group tid / 128 (eight rows); B features
  // tid % 256 and the k groups tid / 256 and tid / 256 + 2
  const int am = tid % kBgM, ag = tid / kBgM;
  const int bn = tid % kBgN, bg = tid / kBgN;
  float ra[8], rb[2][8];
  auto fetch = [&](long kk) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const long k = kk + ag * 8 + j;
      const int m = m0 + am;
      ra[j] = (m < M && k < k1) ? Tin[k * M + m] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const long k = kk + (bg + 2 * q) * 8 + j;
        const int n = n0 + bn;
        rb[q][j] = (n < N && k < k1) ? Tg[k * N + n] : 0.f;
      }
  };
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (k0 < k1) fetch(k0);
  for (long kk = k0; kk < k1; kk += kBgK) {
    split_store8(Ah + am * kBgP + ag * 8, Al + am * kBgP + ag * 8, ra);
#pragma unroll
    for (int q = 0; q < 2; ++q)
      split_store8(Bh + bn * kBgP + (bg + 2 * q) * 8,
                   Bl + bn * kBgP + (bg + 2 * q) * 8, rb[q]);
    __syncthreads();
    if (kk + kBgK < k1) fetch(kk + kBgK);
    bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = (wm + i * 16 + r) * kBgP + kq;
      ah[i] = mtile::lds8(Ah + o);
      al[i] = mtile::lds8(Al + o);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = (wn + j * 16 + r) * kBgP + kq;
      bh[j] = mtile::lds8(Bh + o);
      bl[j] = mtile::lds8(Bl + o);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = mtile::mfma(ah[i], bh[j], acc[i][j]);
        acc[i][j] = mtile::mfma(ah[i], bl[j], acc[i][j]);
        acc[i][j] = mtile::mfma(al[i], bh[j], acc[i][j]);
      }
    __syncthreads();
  }
  float* slot = slots + (long)split * P + off;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + v;
        const int n = n0 + wn + j * 16 + r;
        if (m < M && n < N) slot[(long)m * N + n] += acc[i][j][v];
      }
}

// Launch shape of a parameter-gradient product C[M, N] = sum over K tape
// rows: tile shape (FP32 matrix cores: 32 WM x 32 WN), narrow where the
// layer has few inputs or outputs, so little of a tile is padding (a
// 257 x 64 layer on 128 x 64 tiles, 66 x 256 on 96 x 128); k-splits: a few
// rounds of workgroups over the chip (about 2048 over all nb products, so
// the last round's tail is short), each split at least 256 tape rows long,
// at most the S slots there are.  big: 256 x 256 tiles (layers with at
// least 256 weight rows and columns and long tapes).
struct GemmPlan {
  int shape, tiles, splits;
  bool big;
  int tb, sb;
};

inline GemmPlan plan_grad_gemm(bool f32, long K, int M, int N, int S,
                               int nb) {
  GemmPlan p{};
  int wm = 4, wn = 4;
  p.shape = kG44;
  if (M <= 32) wm = 1, p.shape = kG14;
  else if (N <= 32) wn = 1, p.shape = kG41;
  else if (N <= 64 && M > 64) wn = 2, p.shape = kG42;
  else if (M <= 96 && N > 64) wm = 3, p.shape = kG34;
  const int tm = !f32 ? 64 : 32 * wm, tn = !f32 ? 64 : 32 * wn;
  p.tiles = ((M + tm - 1) / tm) * ((N + tn - 1) / tn);
  int splits = (2048 + p.tiles * nb - 1) / (p.tiles * nb);
  const long by_k = K / 256 > 0 ? K / 256 : 1;
  if (splits > by_k) splits = (int)by_k;
  if (splits > S) splits = S;
  p.splits = splits;
  p.big = f32 && M - 1 >= 256 && N >= 256 && K * nb >= 65536;
  if (p.big) {
    // weight rows on 256 x 256 tiles; the bias row is the last input
    // feature and rides with the first row of tiles
    p.tb = ((M - 1 + 255) / 256) * ((N + 255) / 256);
    int sb = (1024 + p.tb * nb - 1) / (p.tb * nb);
    if (sb > by_k) sb = (int)by_k;
    if (sb > S) sb = S;
    p.sb = sb;
  }
  return p;
}

// nb > 1: nb products of the same shape in one launch (grid y), product j
// reading Tin + j sin and Tg + j sg and adding into its own S slots at
// slots + j sslot (sslot >= S P).  bf16: BF16 mode, whose products with
// at least 256 weight rows and columns go to the split-BF16 matrix cores.
template <typename R>
hipError_t launch_grad_gemm(const R* Tin, const R* Tg, long K, int M, int N,
                            int S, R* slots, long P, long off, hipStream_t s,
                            int nb = 1, long sin = 0, long sg = 0,
                            long sslot = 0, bool bf16 = false) {
  if (nb < 1 || (nb > 1 && sslot < (long)S * P)) return hipErrorInvalidValue;
  const bool f32 = std::is_same<R, float>::value;
  const GemmPlan pl = plan_grad_gemm(f32, K, M, N, S, nb);
  const dim3 g(pl.tiles * pl.splits, nb), blk(256);
  const int splits = pl.splits;
  if constexpr (std::is_same<R, float>::value) {
    if (bf16 && nb == 1 && M - 1 >= 256 && N >= 256) {
      // 128 x 256 tiles over all M features, about 1024 workgroups
      const int tb = ((M + kBgM - 1) / kBgM) * ((N + kBgN - 1) / kBgN);
      const long by_k = K / 256 > 0 ? K / 256 : 1;
      int sb = (1024 + tb - 1) / tb;
      if (sb > by_k) sb = (int)by_k;
      if (sb > S) sb = S;
      hipLaunchKernelGGL(grad_gemm_bf16, dim3(tb * sb), dim3(512), 0, s, Tin,
                         Tg, K, M, N, sb, slots, P, off);
      return hipGetLastError();
    }
    if (pl.big) {
      hipLaunchKernelGGL(grad_gemm_big, dim3(pl.tb * pl.sb, nb), dim3(512), 0,
                         s, Tin, M, Tg, K, M - 1, N, pl.sb, slots, P, off, sin,
                         sg, sslot);
      return hipGetLastError();
    }
    switch (pl.shape) {
      case kG14:
        hipLaunchKernelGGL((grad_gemm_mfma<1, 4>), g, blk, 0, s, Tin, Tg, K,
                           M, N, splits, slots, P, off, sin, sg, sslot);
        break;
      case kG41:
        hipLaunchKernelGGL((grad_gemm_mfma<4, 1>), g, blk, 0, s, Tin, Tg, K,
                           M, N, splits, slots, P, off, sin, sg, sslot);
        break;
      case kG42:
        hipLaunchKernelGGL((grad_gemm_mfma<4, 2>), g, blk, 0, s, Tin, Tg, K,
                           M, N, splits, slots, P, off, sin, sg, sslot);
        break;
      case kG34:
        hipLaunchKernelGGL((grad_gemm_mfma<3, 4>), g, blk, 0, s, Tin, Tg, K,
                           M, N, splits, slots, P, off, sin, sg, sslot);
        break;
      default:
        hipLaunchKernelGGL((grad_gemm_mfma<4, 4>), g, blk, 0, s, Tin, Tg, K,
                           M, N, splits, slots, P, off, sin, sg, sslot);
    }
  } else {
    hipLaunchKernelGGL(grad_gemm<R>, g, blk, 0, s, Tin, Tg, K, M, N, splits,
                       slots, P, off, sin, sg, sslot);
  }
  return hipGetLastError();
}

// The three layers' products of one chunk (tape rows K): grouped, one
// launch of grad_gemm_group where none takes the 256 x 256 tiles (each product with
// exactly the workgroups and k-splits of its own launch, so the slots hold
// the same sums), else one launch each.
template <typename R>
hipError_t launch_grad_gemm3(const R* const Tin[3], const R* const Tg[3],
                             long K, const int M[3], const int N[3], int S,
                             R* slots, long P, const long off[3],
                             hipStream_t s, bool grouped, bool bf16) {
  if constexpr (std::is_same<R, float>::value) {
    GemmGroup g{};
    bool ok = true;
    long nblk = 0;
    for (int j = 0; j < 3; ++j) {
      const GemmPlan pl = plan_grad_gemm(true, K, M[j], N[j], S, 1);
      ok = ok && !pl.big;
      g.Tin[j] = Tin[j];
      g.Tg[j] = Tg[j];
      g.M[j] = M[j];
      g.N[j] = N[j];
      g.S[j] = pl.splits;
      g.shape[j] = pl.shape;
      g.nblk[j] = pl.tiles * pl.splits;
      g.off[j] = off[j];
      nblk += g.nblk[j];
    }
    if (ok && grouped) {
      g.K = K;
      g.P = P;
      g.slots = slots;
      hipLaunchKernelGGL(grad_gemm_group, dim3((unsigned)nblk), dim3(256), 0,
                         s, g);
      return hipGetLastError();
    }
  }
  hipError_t e = hipSuccess;
  for (int j = 0; j < 3 && e == hipSuccess; ++j)
    e = launch_grad_gemm<R>(Tin[j], Tg[j], K, M[j], N[j], S, slots, P, off[j],
                            s, 1, 0, 0, 0, bf16);
  return e;
}

// dtheta = sum of the slots in slot order (deterministic).
template <typename R>
__global__ void reduce_slots(const R* slots, int G, long P, R* out) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p >= P) return;
  // grid y: independent sums, G slots each, into consecutive outputs
  slots += blockIdx.y * (long)G * P;
  out += blockIdx.y * P;
  R acc = R(0);
  for (int g = 0; g < G; ++g) acc += slots[(long)g * P + p];
  out[p] = acc;
}

// dy0 = lambda_0 + cotangents of evaluation times at t0; NaN for invalid.
template <typename R>
__global__ void adj_finish(Mod<R> m, Back<R> b, const R* g_eval, R* dy0) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)m.B * m.D) return;
  const long row = i / m.D, c = i % m.D;
  if (m.st.status[row] == kInvalid) {
    dy0[i] = quiet_nan<R>();
    return;
  }
  R v = b.lam[i];
  for (int e = 0; e < m.E; ++e)
    if (b.owner[row * m.E + e] == -1) v += g_eval[(row * m.E + e) * m.D + c];
  dy0[i] = v;
}

namespace {

inline dim3 lin_grid(long n) { return dim3((unsigned)((n + 255) / 256)); }

// At most two 16-row tiles (CNF: 8 instances) per compute unit.
template <typename R>
bool few_tiles(const Mod<R>& m) {
  return (m.B + (m.cnf ? 7 : 15)) / (m.cnf ? 8 : 16) <= 512;
}

template <typename R, class M>
hipError_t stages(ModImpl& im, Mod<R> v, Back<R>& b, R* y7dst, bool keep_y,
                  hipStream_t s) {
  // v.st.y = y_n, v.hs = h_n, v.st.t = t_n, v.st.status = act, v.K = Ks
  StageSpec sp0{};
  hipError_t e = field<R>(im, v, sp0, b.Ks, s);
  for (int st = 1; st < 7 && e == hipSuccess; ++st) {
    StageSpec sp = stage_spec<M>(st);
    if (keep_y)
      sp.yout = b.Ys + (size_t)st * v.B * v.D;
    else if (st == 6)
      sp.yout = y7dst;
    e = field<R>(im, v, sp, b.Ks + (size_t)st * v.B * v.D, s);
  }
  return e;
}

// One step's seven stages for the segment store: stage inputs into
// Yst[j][s] (stage 1's, y_n itself, is copied there by adj_setup) and the
// hidden-layer values into Ast[j][s]; stage 7's input is y_{n+1}.
template <typename R, class M>
hipError_t stages_store(ModImpl& im, Mod<R> v, Back<R>& b, int j,
                        hipStream_t s) {
  const size_t BD = (size_t)v.B * v.D;
  const size_t AH = (size_t)v.B * (v.cnf ? 2 : 1) * 2 * v.H;
  hipError_t e = hipSuccess;
  [[maybe_unused]] MfmaSteps fs{};
  for (int st = 0; st < 7 && e == hipSuccess; ++st) {
    StageSpec sp = st == 0 ? StageSpec{} : stage_spec<M>(st);
    sp.yout = st == 0 ? nullptr : b.Yst + ((size_t)j * 7 + st) * BD;
    sp.act_out = b.Ast + ((size_t)j * 7 + st) * AH;
    if constexpr (std::is_same<R, float>::value) {
      if (im.mw.packed != nullptr && few_tiles(v)) {  // the seven in one
        fs.st[fs.n] = stage_args(im, v, sp, b.Ks + (size_t)st * BD);
        fs.st[fs.n++].kslot = st;
        fs.kl = 1;  // the stage values are read only by the later stages
        continue;
      }
    }
    e = field<R>(im, v, sp, b.Ks + (size_t)st * BD, s);
  }
  if constexpr (std::is_same<R, float>::value) {
    if (e == hipSuccess && fs.n > 0) e = launch_field_steps_mfma(fs, s);
  }
  return e;
}

template <typename R, class M>
hipError_t backward_t(ModImpl& im, Mod<R>& m, Back<R>& b, const R* g_eval,
                      const R* g_final, R* dy0, R* dtheta, hipStream_t s) {
  const long BD = (long)m.B * m.D;
  const dim3 rows_g((m.B + 3) / 4), blk(256);
  if (im.mw.packedT == nullptr) {
    // tape inputs of tiles no step writes must be finite (they meet 0); the
    // matrix-core VJP kernels write zeros into those rows themselves
    const long n1 = (long)(m.d_in + 2) * b.K, n2 = (long)(m.H + 1) * b.K;
    hipLaunchKernelGGL(fill_r<R>, lin_grid(n1), blk, 0, s, b.T1in, n1, R(0));
    hipLaunchKernelGGL(fill_r<R>, lin_grid(n2), blk, 0, s, b.T2in, n2, R(0));
    hipLaunchKernelGGL(fill_r<R>, lin_grid(n2), blk, 0, s, b.T3in, n2, R(0));
  }
  hipLaunchKernelGGL(copy_r<R>, lin_grid(BD), blk, 0, s, b.lam, g_final, BD);
  hipError_t e = launch_fill_i32(b.flags, 2, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adj_prep<R>, dim3((m.B + 255) / 256), blk, 0, s, m, b);
  e = hipMemcpyAsync(im.host_running, b.flags, sizeof(int32_t) * 2,
                     hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const int nmax = im.host_running[0];
  if (im.host_running[1] != 0) return hipErrorInvalidValue;  // record overflow
  Mod<R> v = m;  // view of the forward's field inputs onto the backward buffers
  v.hs = b.bh;
  v.st.t = b.bt;
  v.st.status = b.act;
  v.K = b.Ks;
  const int k = b.k;
  // Step n's cotangent chain: dense-output cotangents, the seven stage
  // VJPs (on the stored stage inputs Yh and layers Ah of segment step j,
  // or recomputing), and the chunk's parameter-gradient GEMMs.
  // Tape GEMMs beside the cotangent chain: with room for two chunks of
  // steps (matrix-core path), the tape's two halves alternate and each
  // chunk's GEMMs run on a third stream while the next chunk's VJPs write
  // the other half; a half is rewritten only after its GEMMs are done.
  // Every GEMM adds into the slots on that one stream, in chunk order.
  const bool ovl = im.mw.packedT != nullptr && b.C >= 2 && nmax > 1;
  const int Cc = ovl ? b.C / 2 : b.C;
  // k-split slots: a GEMM over K tape rows uses at most K / 256 of them, so
  // only those of the largest chunk are cleared and summed
  const long Bs7 = 7L * (m.cnf ? 2 : 1) * m.B;
  const int G = (int)std::min<long>(b.G, std::max<long>(1, Cc * Bs7 / 256));
  hipLaunchKernelGGL(fill_r<R>, lin_grid((long)G * b.P), blk, 0, s, b.slots,
                     (long)G * b.P, R(0));
  hipStream_t s3 = nullptr;
  if (ovl) {
    if (im.ev[0] == nullptr)
      for (hipEvent_t& ev : im.ev)
        if (e == hipSuccess && ev == nullptr)
          e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = shared_aux_stream2(&s3);
    if (e != hipSuccess) return e;
  }
  auto back_step = [&](int n, const R* Yh, const float* Ah, int j,
                       int setup) -> hipError_t {
    // this step's place in its tape chunk (steps are taken in reverse)
    const int idx = nmax - 1 - n, chunk = idx / Cc, slot_c = idx % Cc;
    const int half = ovl ? (chunk & 1) : 0;
    const int slot = half * Cc + slot_c;
    const long Bs = m.cnf ? 2L * m.B : (long)m.B;
    const long kbase = (long)slot * 7 * Bs;
    if (ovl && slot_c == 0 && chunk >= 2) {
      const hipError_t r = hipStreamWaitEvent(s, im.ev[7 + half], 0);
      if (r != hipSuccess) return r;
    }
    // the seven stages in one launch on the matrix cores while the batch
    // has few tiles (launches, not the tiles' work, set its pace; the
    // dense-output part then runs in the same launch), else one launch
    // each (a CNF step of 8192 instances: 16.9 ms one each, 18.9 in one)
    [[maybe_unused]] MfmaVjpSteps vs{};
    const bool steps = std::is_same<R, float>::value && im.mw.packedT &&
                       few_tiles(m);
    if (steps) {
      if constexpr (std::is_same<R, float>::value) {
        VjpDense& d = vs.dense;
        d.on = 1;
        d.setup = setup;
        d.step = n;
        d.cap = b.cap;
        d.E = m.E;
        d.nacc = b.nacc;
        d.hacc = b.hacc;
        d.tn = b.tn;
        d.owner = b.owner;
        d.t_eval = m.t_eval;
        d.g_eval = g_eval;
        for (int jj = 0; jj < 7; ++jj)
          for (int q = 0; q < 4; ++q) d.P[jj][q] = float(M::P[jj][q]);
        d.act = b.act;
        d.bh = b.bh;
        d.bt = b.bt;
      }
    } else {
      hipLaunchKernelGGL((adj_dense<R, M>), rows_g, blk, 0, s, m, b, n,
                         g_eval, setup);
    }
    if (im.mw.packedT == nullptr) {
      // FMA kernels skip tiles without a step n: their cotangent rows must
      // read as zero (the matrix-core kernels write those zeros themselves)
      const long H = m.H, rows = 7 * Bs;
      hipLaunchKernelGGL(fill_r<R>, lin_grid(H * rows), blk, 0, s,
                         b.T1g + kbase * H, H * rows, R(0));
      hipLaunchKernelGGL(fill_r<R>, lin_grid(H * rows), blk, 0, s,
                         b.T2g + kbase * H, H * rows, R(0));
      hipLaunchKernelGGL(fill_r<R>, lin_grid((long)m.d_in * rows), blk, 0, s,
                         b.T3g + kbase * m.d_in, (long)m.d_in * rows, R(0));
    }
    for (int st = 7; st >= 1; --st) {
      VjpSpec sp{};
      sp.s = st;
      sp.c = M::C[st - 1];
      sp.kbase = kbase;
      if (Yh != nullptr) {
        sp.Y = Yh + ((size_t)j * 7 + st - 1) * BD;
        sp.act_in = Ah + ((size_t)j * 7 + st - 1) *
                             ((size_t)m.B * (m.cnf ? 2 : 1) * 2 * m.H);
      }
      // kappa_j receives h a_{s j} mu_s for the stages j < s
      const StageSpec ss = stage_spec<M>(st - 1 > 0 ? st - 1 : 0);
      sp.n = st - 1 > 0 ? ss.n : 0;
      for (int q = 0; q < sp.n; ++q) {
        sp.kidx[q] = ss.kidx[q];
        sp.coef[q] = ss.coef[q];
      }
      if constexpr (std::is_same<R, float>::value) {
        if (steps) {
          vs.st[vs.n++] = vjp_args(im, m, b, sp);
          continue;
        }
      }
      const hipError_t r = vjp<R>(im, m, b, sp, s);
      if (r != hipSuccess) return r;
    }
    if (steps) {
      const hipError_t r = launch_vjp_steps_mfma(vs, s);
      if (r != hipSuccess) return r;
    }
    if (slot_c == Cc - 1 || n == 0) {
      // parameter gradient of the chunk's steps: one GEMM per layer over
      // its (slot_c + 1) * 7 * Bs tape rows, from the half's first row
      const long Kc = (long)(slot_c + 1) * 7 * Bs;
      const long r0 = (long)half * Cc * 7 * Bs;
      const int H = m.H, din = m.d_in, n0 = din + 1;
      const long o2 = (long)(n0 + 1) * H, o3 = o2 + (long)(H + 1) * H;
      hipStream_t sg = s;
      hipError_t r = hipSuccess;
      if (ovl) {
        sg = s3;
        r = hipEventRecord(im.ev[6], s);
        if (r == hipSuccess) r = hipStreamWaitEvent(s3, im.ev[6], 0);
      }
      if (r == hipSuccess) {
        const R* const ti[3] = {b.T1in + r0 * (n0 + 1), b.T2in + r0 * (H + 1),
                                b.T3in + r0 * (H + 1)};
        const R* const tg[3] = {b.T1g + r0 * H, b.T2g + r0 * H,
                                b.T3g + r0 * din};
        const int gm[3] = {n0 + 1, H + 1, H + 1}, gn[3] = {H, H, din};
        const long go[3] = {0, o2, o3};
        // (the last chunk's products, which nothing runs beside, in one
        // launch; the others one layer at a time, beside the VJPs)
        r = launch_grad_gemm3<R>(ti, tg, Kc, gm, gn, G, b.slots, b.P, go, sg,
                                 n == 0, im.mw.packed != nullptr && !im.mw.f32);
      }
      if (r == hipSuccess && ovl) r = hipEventRecord(im.ev[7 + half], s3);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  };
  if (b.Yst != nullptr) {
    // Segment store, pipelined over two streams: segment q - 1 is
    // recomputed on the second stream (its stage inputs and layers into
    // store half (q - 1) & 1) while the caller's stream runs segment q's
    // cotangent chain on half q & 1.  Both chains are sequences of short
    // launches on a fraction of the compute units, so they overlap.
    if (im.ev[0] == nullptr) {
      for (hipEvent_t& ev : im.ev)
        if (e == hipSuccess && ev == nullptr)
          e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    hipStream_t s2 = nullptr;
    e = shared_aux_stream(&s2);
    if (e != hipSuccess) return e;
    hipEvent_t *ready = im.ev + 1, *freed = im.ev + 3;
    e = hipEventRecord(im.ev[0], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(s2, im.ev[0], 0);
    if (e != hipSuccess) return e;
    Back<R> br = b;  // the recomputation's own step view
    br.act = b.act2;
    br.bh = b.bh2;
    br.bt = b.bt2;
    Mod<R> vr = m;
    vr.hs = br.bh;
    vr.st.t = br.bt;
    vr.st.status = br.act;
    vr.K = b.Ks;
    const int nseg = (nmax + k - 1) / k;
    const size_t BD7 = 7 * (size_t)BD;
    auto seg_top = [&](int q) { return std::min(q * k + k, nmax) - 1; };
    auto recompute = [&](int q) -> hipError_t {
      const int half = q & 1;
      hipError_t r = hipSuccess;
      // the half was last read by segment q + 2's cotangent chain
      if (q + 2 < nseg) r = hipStreamWaitEvent(s2, freed[half], 0);
      if (r != hipSuccess) return r;
      Back<R> bq = br;
      bq.Yst = b.Yst + half * b.yst_half;
      bq.Ast = b.Ast + half * b.ast_half;
      hipLaunchKernelGGL(adj_load_ckpt<R>, lin_grid(BD), blk, 0, s2, m, bq, q,
                         b.yseg);
      for (int mm = q * k; mm <= seg_top(q) && r == hipSuccess; ++mm) {
        const int j = mm - q * k;
        // y_mm: the checkpoint, else stage 7's input of step mm - 1
        R* ym = j == 0 ? b.yseg : bq.Yst + (size_t)(j - 1) * BD7 + 6 * BD;
        hipLaunchKernelGGL(adj_setup<R>, rows_g, blk, 0, s2, m, bq, mm,
                           (const R*)ym, bq.Yst + (size_t)j * BD7);
        vr.st.y = ym;
        r = stages_store<R, M>(im, vr, bq, j, s2);
      }
      if (r == hipSuccess) r = hipEventRecord(ready[half], s2);
      return r;
    };
    if (nseg > 0) e = recompute(nseg - 1);
    for (int q = nseg - 1; q >= 0 && e == hipSuccess; --q) {
      if (q > 0) e = recompute(q - 1);  // enqueued ahead of q's chain
      if (e == hipSuccess) e = hipStreamWaitEvent(s, ready[q & 1], 0);
      const R* Yh = b.Yst + (q & 1) * b.yst_half;
      const float* Ah = b.Ast + (q & 1) * b.ast_half;
      for (int n = seg_top(q); n >= q * k && e == hipSuccess; --n)
        e = back_step(n, Yh, Ah, n - q * k, 1);
      if (e == hipSuccess) e = hipEventRecord(freed[q & 1], s);
    }
    if (e == hipSuccess) e = hipEventRecord(im.ev[5], s2);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, im.ev[5], 0);
    if (e != hipSuccess) return e;
  } else {
    for (int n = nmax - 1; n >= 0; --n) {
      const int seg = n / k, base = seg * k;
      if (n == nmax - 1 || n == base + k - 1) {
        // entering a segment from above: states y_base .. y_n by
        // recomputation
        hipLaunchKernelGGL(adj_load_ckpt<R>, lin_grid(BD), blk, 0, s, m, b,
                           seg, b.yseg);
        for (int mm = base; mm < n; ++mm) {
          R* ym = b.yseg + (size_t)(mm - base) * BD;
          hipLaunchKernelGGL(adj_setup<R>, rows_g, blk, 0, s, m, b, mm,
                             (const R*)nullptr, (R*)nullptr);
          v.st.y = ym;
          e = stages<R, M>(im, v, b, ym + BD, false, s);
          if (e != hipSuccess) return e;
        }
      }
      R* yn = b.yseg + (size_t)(n - base) * BD;
      hipLaunchKernelGGL(adj_setup<R>, rows_g, blk, 0, s, m, b, n,
                         (const R*)yn, b.Ys);
      v.st.y = yn;
      e = stages<R, M>(im, v, b, nullptr, true, s);
      if (e == hipSuccess) e = back_step(n, nullptr, nullptr, 0, 0);
      if (e != hipSuccess) return e;
    }
  }
  if (ovl) {  // the last chunk's GEMMs before the slots are summed
    e = hipEventRecord(im.ev[9], s3);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, im.ev[9], 0);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(adj_finish<R>, lin_grid(BD), blk, 0, s, m, b, g_eval,
                     dy0);
  hipLaunchKernelGGL(reduce_slots<R>, lin_grid(b.P), blk, 0, s, b.slots, G,
                     b.P, dtheta);
  return hipGetLastError();
}

template <typename R>
hipError_t backward_m(ModImpl& im, Mod<R>& m, Back<R>& b, const void* ge,
                      const void* gf, void* dy0, void* dth, hipStream_t s) {
  const R* g_eval = static_cast<const R*>(ge);
  if (im.cfg.method == BODE_TSIT5)
    return backward_t<R, Tsit5>(im, m, b, g_eval, static_cast<const R*>(gf),
                                static_cast<R*>(dy0), static_cast<R*>(dth), s);
  return backward_t<R, Dopri5>(im, m, b, g_eval, static_cast<const R*>(gf),
                               static_cast<R*>(dy0), static_cast<R*>(dth), s);
}

#include "cadjoint.inc"

}  // namespace

hipError_t modular_backward(ModularPlan& mp, const void* g_y_eval,
                            const void* g_y_final, void* dy0, void* dtheta,
                            hipStream_t s) {
  ModImpl* im = static_cast<ModImpl*>(mp.impl);
  if (!im || im->cfg.record_cap < 1) return hipErrorInvalidValue;
  if (im->is64)
    return backward_m<double>(*im, im->md, im->bd, g_y_eval, g_y_final, dy0,
                              dtheta, s);
  return backward_m<float>(*im, im->mf, im->bf, g_y_eval, g_y_final, dy0,
                           dtheta, s);
}

size_t modular_cadjoint_bytes(const ModularPlan& mp, int joint) {
  const ModImpl* im = static_cast<const ModImpl*>(mp.impl);
  if (!im) return 0;
  return im->is64 ? ca_layout<double>(im->cfg, joint, nullptr, nullptr)
                  : ca_layout<float>(im->cfg, joint, nullptr, nullptr);
}

namespace {
template <typename R>
hipError_t cadjoint_m(ModImpl& im, Mod<R>& m, int joint, const void* ge,
                      const void* gf, void* ws, void* dy0, void* dth,
                      int32_t* stats, hipStream_t s) {
  CA<R> c{};
  ca_layout<R>(im.cfg, joint, ws, &c);
  c.t0 = m.t0;
  c.t_end = m.t_end;
  c.rtol = m.rtol;
  c.atol = m.atol;
  c.t_eval = m.t_eval;
  c.fwd = m.st.status;
  c.yfin = m.y_final;
  c.g_eval = static_cast<const R*>(ge);
  c.g_final = static_cast<const R*>(gf);
  c.ctrl = m.ctrl;
  if (im.cfg.method == BODE_TSIT5)
    return cadjoint_t<R, Tsit5>(im, m, c, static_cast<R*>(dy0),
                                static_cast<R*>(dth), stats, s);
  return cadjoint_t<R, Dopri5>(im, m, c, static_cast<R*>(dy0),
                               static_cast<R*>(dth), stats, s);
}
}  // namespace

hipError_t modular_cadjoint(ModularPlan& mp, int joint, const void* g_y_eval,
                            const void* g_y_final, void* workspace,
                            void* dy0, void* dtheta, int32_t* stats,
                            hipStream_t s) {
  ModImpl* im = static_cast<ModImpl*>(mp.impl);
  if (!im) return hipErrorInvalidValue;
  if (im->is64)
    return cadjoint_m<double>(*im, im->md, joint, g_y_eval, g_y_final,
                              workspace, dy0, dtheta, stats, s);
  return cadjoint_m<float>(*im, im->mf, joint, g_y_eval, g_y_final, workspace,
                           dy0, dtheta, stats, s);
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

void modular_release(ModularPlan& mp) {
  ModImpl* im = static_cast<ModImpl*>(mp.impl);
  if (!im) return;
  if (im->host_running) pinned_give(im->host_running);
  if (im->rounds_exec) (void)hipGraphExecDestroy(im->rounds_exec);
  if (im->cap_stream) (void)hipStreamDestroy(im->cap_stream);
  for (hipEvent_t& e : im->ev)
    if (e) (void)hipEventDestroy(e);
  delete im;
  mp.impl = nullptr;
}

}  // namespace bode
