// BF16 MFMA evaluation of the neural fields (MLP and CNF), gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace bode {

// Packed weights: every layer as 16x32 MFMA B-fragments (64 lanes x 8
// elements, contiguous per fragment), plus FP32 vectors b1, w1t (the time
// row of W1), b2, b3.  Elements are BF16 (BF16 mode) or FP32 (FP32 mode,
// f32 != 0).
struct MfmaWeights {
  void* packed = nullptr;
  float* fvec = nullptr;
  // Transposed layers for the vector-Jacobian products of the adjoint:
  // W3^T, W2^T and W1^T without its time row (null when not needed).
  void* packedT = nullptr;
  int f32 = 0;
  // BF16 mode: 1 rounds every activation to one BF16 term (plain BF16);
  // 0 splits it into three (hi + mid + lo, FP32's precision).
  int plain = 0;
};

size_t mfma_packed_bytes(int din, int H, int f32);
size_t mfma_packedT_bytes(int din, int H, int f32);
size_t mfma_fvec_elems(int din, int H);
std::string mfma_supported(int din, int H);
// Wavefronts per 16-row tile the field kernels use: `requested` (4 or 8)
// where the width allows it, else the default for the shape.
int mfma_waves(int H, bool cnf, int B, int requested);

hipError_t mfma_pack_weights(const MfmaWeights& w, int din, int H,
                             const float* W1, const float* b1, const float* W2,
                             const float* b2, const float* W3, const float* b3,
                             hipStream_t s);

struct MfmaArgs {
  int B, D, din, H, cnf;
  const int32_t* status;
  const float* y;
  const float* K;  // [7, B, D]
  float* Y7;
  const float* hs;
  const double* t;
  const float* eps;
  MfmaWeights w;
  int n;
  int kidx[6];
  float coef[6];
  double c;
  int write_y7;
  float* out;
  // If not null, the hidden layers' values of every row are stored here for
  // a later vector-Jacobian product: [Bs][2][H] (Bs = B, or 2B for the CNF
  // whose tangent rows follow), layer 1 then layer 2 of each row; the
  // activation on primal rows, the pre-activation tangent on tangent rows.
  float* act_out;
  // wavefronts per 16-row tile: 4 or 8 (0: the default for the width)
  int waves;
  // the fused solve's stage slot of out (its stages kept in LDS)
  int kslot;
};

MfmaArgs mfma_args(int B, int D, int din, int H, int cnf, const int32_t* status,
                   const float* y, const float* K, float* Y7, const float* hs,
                   const double* t, const float* eps, const MfmaWeights& w);

// row_tile 0 picks the default for the shape.
hipError_t launch_field_mfma(const MfmaArgs& a, int row_tile, hipStream_t s);

// One stage s of the discrete adjoint for a batch of rows: mu_s =
// J_f(Y_s)^T kappa_s on MFMA (the field's hidden layers recomputed), the
// stage's entries of the parameter-gradient tape, and the row updates
// kappa_j += h a_sj mu_s, lambda_next += mu_s (Lambda = lambda + mu at the
// last stage, lambda = lambda_next after the first).
struct MfmaVjpArgs {
  int B, D, din, H, cnf;
  const int32_t* act;  // rows with kRunning are differentiated
  const float* Y;      // [B, D] stage input
  const float* kap_s;  // [B, D] kappa_s
  const float* eps;    // [B, D] probe (CNF)
  const float* bh;     // [B] step size
  const double* bt;    // [B] t_n
  double c;            // c_s
  MfmaWeights w;
  // tape, sample-major [K][feature]; this stage's rows start at kb
  float *T1in, *T1g, *T2in, *T2g, *T3in, *T3g;
  long K, kb;
  int s, n;
  int kidx[6];
  float coef[6];
  float *lam, *lamn, *kap;  // kap: [7, B, D]
  // Continuous adjoint: if not null, mu_s is stored here ([B, D], zero in
  // the columns the field does not read) instead of the row updates above.
  float* mu_out;
  // If not null, the hidden layers' values of this stage as a field kernel
  // stored them (MfmaArgs::act_out's layout): the two forward layers are
  // read instead of recomputed.
  const float* act_in;
};

hipError_t launch_vjp_mfma(const MfmaVjpArgs& a, hipStream_t s);

// Up to seven stages of one step, each with its own arguments, in one
// launch, in the order given (same shape and weights in every entry).
// The step's dense-output cotangents and step view, formed by the
// workgroup of each tile before its first stage (the discrete adjoint's
// dense-output kernel, folded in): zero lambda_next and the seven kappa
// rows, add h w_j(theta) g to kappa_j and g to lambda_next for every
// evaluation time the step answers, and (setup) the step view act, bh, bt.
struct VjpDense {
  int on, setup, step, cap, E;
  const int32_t* nacc;   // [B] accepted steps in the record
  const double* hacc;    // [B, cap] accepted step sizes
  const double* tn;      // [B, cap + 1] step start times
  const int32_t* owner;  // [B, E] step answering each evaluation time
  const double* t_eval;  // [B, E]
  const float* g_eval;   // [B, E, D] cotangents of the outputs
  float P[7][4];         // interpolant weights: w_j = th (P0 + th (P1 + ...))
  int32_t* act;          // [B] step view (setup)
  float* bh;
  double* bt;
};

struct MfmaVjpSteps {
  MfmaVjpArgs st[7];
  int n;
  VjpDense dense;
  int cl_off;  // set by the launcher
};
hipError_t launch_vjp_steps_mfma(const MfmaVjpSteps& v, hipStream_t s);

struct MfmaSteps {
  MfmaArgs st[7];
  int n;
  // kl = 1: the caller reads none of the stage values, which may then stay
  // in the tile's LDS ([7][rows][D] at byte kl_off, st[i].kslot each stage's
  // slot) instead of going to st[i].out; kl_off is set by the launcher
  int kl, kl_off;
};
hipError_t launch_field_steps_mfma(const MfmaSteps& v, hipStream_t s);
// both travel as kernel arguments
static_assert(sizeof(MfmaVjpSteps) <= 4096 && sizeof(MfmaSteps) <= 4096,
              "step arguments exceed the kernel-argument space");

}  // namespace bode
