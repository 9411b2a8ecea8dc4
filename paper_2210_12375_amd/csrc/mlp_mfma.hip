// Neural right-hand sides on the matrix cores of gfx950: weight packing,
// the per-stage field kernel and the adjoint-stage kernel (the building
// blocks and operand policies are in mlp_mfma_tile.hpp).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "mlp_mfma.hpp"
#include "mlp_mfma_tile.hpp"

namespace bode {

namespace {

using namespace mtile;

__device__ __forceinline__ void cvt(uint16_t& d, float v) { d = f2bf(v); }
__device__ __forceinline__ void cvt(float& d, float v) { d = v; }

// One weight matrix to pack: M = W (trans = 0) or W^T into the fragment
// layout of mtile (W row-major with leading dimension ldw, K rows of M).
template <typename W>
struct PackJob {
  W* dst;
  const float* Wm;
  int K, ldw, nk, nn, trans;
};

template <typename W>
__device__ void pack_one(const PackJob<W>& j, int blk, int nblk) {
  const long total = (long)j.nk * j.nn * 512;
  for (long e = blk * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)nblk * blockDim.x) {
    const int i = e & 7, l = (e >> 3) & 63;
    const long f = e >> 9;
    const int kb = int(f / j.nn), nb = int(f % j.nn);
    const int k = kb * 32 + (l >> 4) * 8 + i, n = nb * 16 + (l & 15);
    const long src = j.trans ? (long)n * j.ldw + k : (long)k * j.ldw + n;
    cvt(j.dst[e], k < j.K ? j.Wm[src] : 0.f);
  }
}

// The three layers (and, with the transposed copies, their transposes)
// and the vector block (b1, W1's time row, b2, b3) in one launch: grid y
// selects the job, the last one being the vector block.
template <typename W>
__global__ void pack_weights_kernel(PackJob<W> j0, PackJob<W> j1,
                                    PackJob<W> j2, PackJob<W> j3,
                                    PackJob<W> j4, PackJob<W> j5, int njobs,
                                    float* f, const float* W1, const float* b1,
                                    const float* b2, const float* b3, int din,
                                    int H) {
  const int y = blockIdx.y;
  if (y < njobs) {
    const PackJob<W>& j = y == 0 ? j0 : y == 1 ? j1 : y == 2 ? j2
                        : y == 3 ? j3 : y == 4 ? j4 : j5;
    pack_one(j, blockIdx.x, gridDim.x);
    return;
  }
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < 3 * H + din;
       c += gridDim.x * blockDim.x) {
    float v;
    if (c < H)
      v = b1[c];
    else if (c < 2 * H)
      v = W1[(long)din * H + (c - H)];  // time row of W1
    else if (c < 3 * H)
      v = b2[c - 2 * H];
    else
      v = b3[c - 3 * H];
    f[c] = v;
  }
}

template <class Op, int NTW, bool CNF, int WV>
__global__ __launch_bounds__(64 * WV) void field_mfma_kernel(MfmaArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  field_tile<Op, NTW, CNF, WV>(a, blockIdx.x * (CNF ? 8 : 16), smem_raw);
}

// Several stage evaluations of one step in one launch, in order: a tile's
// stage inputs depend only on its own rows' earlier stages, which pass
// between the tile's waves through memory (the barrier orders them).
// KL: the stage values stay in LDS (v.kl_off) between the stages.
template <class Op, int NTW, bool CNF, int WV, bool KL>
__global__ __launch_bounds__(64 * WV) void field_steps_kernel(MfmaSteps v) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* kl = KL ? reinterpret_cast<float*>(smem_raw + v.kl_off) : nullptr;
  for (int i = 0; i < v.n; ++i) {
    field_tile<Op, NTW, CNF, WV, true, KL>(v.st[i], blockIdx.x * (CNF ? 8 : 16),
                                           smem_raw, kl);
    __syncthreads();
  }
}

template <class Op, int NTW, bool CNF, int WV>
hipError_t launch_t(const MfmaArgs& a, const MfmaSteps* v, hipStream_t s) {
  constexpr int PR = CNF ? 8 : 16;
  const size_t sm = mfma_smem<Op, NTW, CNF, WV>(a.din);
  if (sm > 65536) return hipErrorInvalidValue;
  if (v != nullptr) {
    MfmaSteps w = *v;
    w.kl_off = (int)((sm + 15) / 16 * 16);
    const size_t smk = w.kl_off + sizeof(float) * 7 * PR * (size_t)a.D;
    if (w.kl && smk <= 65536)
      hipLaunchKernelGGL((field_steps_kernel<Op, NTW, CNF, WV, true>),
                         dim3((a.B + PR - 1) / PR), dim3(64 * WV), smk, s, w);
    else
      hipLaunchKernelGGL((field_steps_kernel<Op, NTW, CNF, WV, false>),
                         dim3((a.B + PR - 1) / PR), dim3(64 * WV), sm, s, w);
  } else
    hipLaunchKernelGGL((field_mfma_kernel<Op, NTW, CNF, WV>),
                       dim3((a.B + PR - 1) / PR), dim3(64 * WV), sm, s, a);
  return hipGetLastError();
}


// Adjoint stage on MFMA.  The hidden layers are recomputed as in the field
// kernel; each lane keeps, for its accumulator elements, the activation
// (primal rows) or the pre-activation tangent (CNF tangent rows), so the
// backward epilogues need no second pass over LDS.  The backward chain runs
// the same GEMM on the transposed layers: S2 = gbar W3^T, G2 = tanh'(p2) S2
// (plus the CNF's second-order term), S1 = G2 W2^T, G1 = tanh'(p1) S1,
// mu = G1 W1^T.  For the CNF, gbar's tangent rows hold -kappa_l eps, the
// cotangent of the tangent output.
// The CNF kernel at width 512 asks for four wavefronts per SIMD (two
// workgroups per compute unit): it spills a few registers, but the second
// workgroup hides more of the three-layer dependent chain (measured 156 ->
// 133 us per stage for 8192 instances).
// CL: the step's stage cotangents kappa and lambda_next of the tile's rows
// are a [8][rows][D] block in LDS at cl (slots 0-6: kappa_1..7, slot 7:
// lambda_next) instead of the arrays a.kap, a.lamn; lambda stays in HBM.
// Elements of a tile's [PR, din] block each thread handles, for din up to
// DMAX.
template <int PR, int WV, int DMAX = 256>
constexpr int vjp_ne() {
  return (PR * DMAX + 64 * WV - 1) / (64 * WV);
}

// A stage's stored values the VJP of a tile reads from memory: the stage
// input Y (NE elements a thread) and the two stored hidden layers at this
// lane's accumulator elements.
template <int NE, int NTW>
struct VjpFront {
  float Y[NE];
  float keep[2][NTW][4];
};

// Requests them, at clamped rows and unconditionally, so that no load waits
// on a branch (rows without the step are zeroed where they are used).
template <bool CNF, int WV, int NE, int NTW>
__device__ __forceinline__ void vjp_front_load(const MfmaVjpArgs& a,
                                               VjpFront<NE, NTW>& f) {
  constexpr int PR = CNF ? 8 : 16, H = NTW * 16 * WV;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rq = (lane >> 4) * 4, col = lane & 15;
  const int din = a.din, D = a.D, B = a.B, r0 = blockIdx.x * PR;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int idx = tid + e * (int)blockDim.x;
    const int ii = idx < PR * din ? idx : 0;
    const int r = ii / din, c = ii % din;
    f.Y[e] = a.Y[(long)(r0 + r < B ? r0 + r : B - 1) * D + c];
  }
#pragma unroll
  for (int layer = 0; layer < 2; ++layer)
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      const int n = (wave * NTW + t) * 16 + col;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rq + i;
        const bool primal = !CNF || row < PR;
        const int g = r0 + (primal ? row : row - PR);
        f.keep[layer][t][i] =
            a.act_in[((long)((g < B ? g : B - 1) + (primal ? 0 : B)) * 2 +
                      layer) * H + n];
      }
    }
}

// PF (stored layers, steps launch, din <= 64): the stage's VjpFront was requested
// during the previous stage (or before the launch's dense-output part) into
// *pf, and this stage requests nxt's (the last stage: its own again) into it
// once its own are used, so their memory latency overlaps this stage's last phase; the
// tile's step view (running rows, t, h) is read from memory at the first
// stage only.
template <class Op, int NTW, bool CNF, int WV, bool CL = false,
          bool PF = false>
__device__ __forceinline__ void vjp_tile(
    const MfmaVjpArgs& a, unsigned char* smem_raw, float* cl = nullptr,
    VjpFront<vjp_ne<CNF ? 8 : 16, WV, 64>(), NTW>* pf = nullptr,
    const MfmaVjpArgs& nxt = MfmaVjpArgs{}, bool first = true) {
  typedef typename Op::A A;
  typedef typename Op::W W;
  constexpr int RT = 16, PR = CNF ? 8 : 16, H = NTW * 16 * WV,
                SA = H + Op::kPad;
  // weight blocks in flight: two for the CNF, whose kernel is held to 128
  // registers (four wavefronts per SIMD)
  constexpr int PD = CNF ? 2 : mtile::ring_depth(NTW, Op::kFragRegs),
                PD4 = CNF ? 2 : mtile::ring_depth(4, Op::kFragRegs);
  const int din = a.din, D = a.D, B = a.B;
  const Dims dm = dims(din, H);
  const DimsT dt = dims_t(din, H);
  const int SX = dm.K1 + Op::kPad;
  const int PX = RT * SX, PA = RT * SA;
  A* Xh = reinterpret_cast<A*>(smem_raw);
  A* Ah = Xh + Op::kPlanes * PX;
  float* tcol = reinterpret_cast<float*>(Ah + Op::kPlanes * PA);  // [PR]
  float* MU = reinterpret_cast<float*>(Xh);  // [PR][din], after S2 is read
  __shared__ int any_running;
  __shared__ int onr[PR];  // the tile's rows that have this step
  __shared__ double tstep[PR];  // their t_n and h_n
  __shared__ float hstep[PR];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = blockIdx.x * PR;
  // Weight rings of the transposed layers.  With the stored forward layers
  // (and outside the register-bound CNF kernel) each is requested one
  // phase ahead: W3^T's at entry, W2^T's after S2's products, W1^T's after
  // S1's.
  const W* wt = static_cast<const W*>(a.w.packedT);
  const bool ahead = !CNF && a.act_in != nullptr;
  const int ntiles1 = (dt.nn1 - wave + WV - 1) / WV;
  WRing<Op, NTW, PD> r3;
  WRing<Op, NTW, PD, H / 32> r2;
  WRing<Op, 4, PD4, H / 32> r1;
  if (ahead) r3.start(wt, dt.nk3, dt.nn3, wave * NTW, 1, NTW, lane);
  if (!PF || first) {
    if (tid == 0) any_running = 0;
    __syncthreads();
    if (tid < PR) {
      const int o = r0 + tid < B && a.act[r0 + tid] == kRunning;
      onr[tid] = o;
      if (o) any_running = 1;
    }
    __syncthreads();
  }
  const long kb = a.kb;
  const long l1 = din + 2;  // tape row widths: T1in din + 2, T2in/T3in H + 1
  if (!any_running) {
    // no row of the tile has this step: its rows of the tape are zero (the
    // gradient GEMMs read every row; a tape holds several steps, so these
    // rows may hold an earlier step's values, or nothing yet)
    const int nr = CNF ? 2 : 1;
    for (int idx = tid; idx < PR * (H + 1); idx += blockDim.x) {
      const int r = idx / (H + 1), c = idx % (H + 1), row = r0 + r;
      if (row >= B) continue;
      for (int q = 0; q < nr; ++q) {
        const long k = kb + row + q * B;
        if (c < H) {
          a.T1g[k * H + c] = 0.f;
          a.T2g[k * H + c] = 0.f;
        }
        a.T2in[k * (H + 1) + c] = 0.f;
        a.T3in[k * (H + 1) + c] = 0.f;
      }
    }
    for (int idx = tid; idx < PR * l1; idx += blockDim.x) {
      const int r = idx / l1, c = idx % l1, row = r0 + r;
      if (row >= B) continue;
      for (int q = 0; q < nr; ++q) {
        const long k = kb + row + q * B;
        a.T1in[k * l1 + c] = 0.f;
        if (c < din) a.T3g[k * din + c] = 0.f;
      }
    }
    return;
  }
  auto on = [&](int row) { return onr[row - r0] != 0; };  // row in the tile

  const float* b1 = a.w.fvec;
  const float* w1t = b1 + H;
  const float* b2 = b1 + 2 * H;
  const int rq = (lane >> 4) * 4, col = lane & 15;
  // tape column of accumulator row `row` of the 16-row tile (-1: none)
  auto tk = [&](int row) -> long {
    const bool primal = !CNF || row < PR;
    const int g = r0 + (primal ? row : row - PR);
    if (g >= B) return -1;
    return kb + g + (primal ? 0 : B);
  };
  float keep[2][NTW][4];
  if (a.act_in != nullptr) {
    // The forward layers as the stage's field evaluation stored them: no
    // layer is recomputed, so nothing here waits on anything but memory,
    // and every load of the kernel's front half is issued at once (stage
    // input, cotangent, probe, stored layers, time) before the first store.
    constexpr int NE = vjp_ne<PR, WV, PF ? 64 : 256>();
    VjpFront<NE, NTW> fl;
    VjpFront<NE, NTW>* fp = &fl;
    if constexpr (PF)
      fp = pf;
    else
      vjp_front_load<CNF, WV>(a, fl);
    VjpFront<NE, NTW>& f = *fp;
    float(&Yr)[NE] = f.Y;
    float Kz[NE], Er[NE], Kl[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int idx = tid + e * (int)blockDim.x;
      const int ii = idx < PR * din ? idx : 0;
      const int r = ii / din, c = ii % din;
      const long o = (long)(r0 + r < B ? r0 + r : B - 1) * D;
      const float* ks = CL ? cl + ((a.s - 1) * PR + r) * D : a.kap_s + o;
      Kz[e] = ks[c];
      if (CNF) {
        Er[e] = a.eps[o + c];
        Kl[e] = ks[din];
      }
    }
    // the time column's t and h (clamped row), kept in LDS for the row
    // updates (and, PF, for the later stages)
    const int trow = r0 + (tid < PR ? tid : 0) < B ? r0 + (tid < PR ? tid : 0)
                                                  : B - 1;
    double tb;
    float hb;
    if (!PF || first) {
      tb = a.bt[trow];
      hb = a.bh[trow];
    } else {
      tb = tstep[tid < PR ? tid : 0];
      hb = hstep[tid < PR ? tid : 0];
    }
    if (tid < PR) {
      tstep[tid] = tb;
      hstep[tid] = hb;
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int idx = tid + e * (int)blockDim.x;
      if (idx < PR * din && !onr[idx / din]) Yr[e] = Kz[e] = Er[e] = Kl[e] = 0.f;
    }
#pragma unroll
    for (int layer = 0; layer < 2; ++layer)
#pragma unroll
      for (int t = 0; t < NTW; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = rq + i;
          const int pr = !CNF || row < PR ? row : row - PR;
          keep[layer][t][i] =
              r0 + pr >= B || !onr[pr] ? 0.f : f.keep[layer][t][i];
        }
    const float tv = tid < PR && r0 + tid < B && onr[tid]
                         ? float(tb + a.c * double(hb))
                         : 0.f;
    // layer-1 inputs and the cotangent gbar (kappa_z on primal rows,
    // -kappa_l eps on tangent rows) into the tape; gbar into LDS
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int idx = tid + e * (int)blockDim.x;
      if (idx < PR * din) {
        const int r = idx / din, c = idx % din, row = r0 + r;
        Op::put(Xh, PX, r * SX + c, Kz[e]);
        if (row < B) {
          a.T1in[(kb + row) * l1 + c] = Yr[e];
          a.T3g[(kb + row) * din + c] = Kz[e];
        }
        if (CNF) {
          const float gg = -Kl[e] * Er[e];
          Op::put(Xh, PX, (PR + r) * SX + c, gg);
          if (row < B) {
            a.T1in[(kb + B + row) * l1 + c] = Er[e];
            a.T3g[(kb + B + row) * din + c] = gg;
          }
        }
      }
    }
    if (tid < PR && r0 + tid < B) {
      const int row = r0 + tid;
      a.T1in[(kb + row) * l1 + din] = tv;
      a.T1in[(kb + row) * l1 + din + 1] = 1.f;
      if (CNF) {
        a.T1in[(kb + B + row) * l1 + din] = 0.f;
        a.T1in[(kb + B + row) * l1 + din + 1] = 0.f;
      }
    }
    // layer-2 and layer-3 inputs (the activations; on tangent rows the
    // tangent activation from the partner row's tanh') and bias features
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
      float* Tin = layer == 0 ? a.T2in : a.T3in;
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        const int n = (wave * NTW + t) * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = rq + i;
          const bool primal = !CNF || row < PR;
          float act = keep[layer][t][i];
          if (CNF) {
            const float ap = __shfl_xor(act, 32, 64);
            if (!primal) act = (1.f - ap * ap) * act;
          }
          const long k = tk(row);
          if (k >= 0) Tin[k * (H + 1) + n] = act;
        }
      }
    }
    for (int r = tid; r < RT; r += blockDim.x) {
      const long k = tk(r);
      if (k < 0) continue;
      const float one = (!CNF || r < PR) ? 1.f : 0.f;
      a.T2in[k * (H + 1) + H] = one;
      a.T3in[k * (H + 1) + H] = one;
    }
    for (int idx = tid; idx < RT * (dm.K1 - din); idx += blockDim.x) {
      const int r = idx / (dm.K1 - din), c = din + idx % (dm.K1 - din);
      Op::put(Xh, PX, r * SX + c, 0.f);
    }
    __syncthreads();
  } else {
  // prologue: Y_s and the probe into LDS, the layer-1 inputs into the tape
  for (int idx = tid; idx < PR * din; idx += blockDim.x) {
    const int r = idx / din, c = idx % din, row = r0 + r;
    const bool o = on(row);
    const float Yv = o ? a.Y[(long)row * D + c] : 0.f;
    Op::put(Xh, PX, r * SX + c, Yv);
    if (row < B) a.T1in[(kb + row) * l1 + c] = Yv;
    if (CNF) {
      const float e = o ? a.eps[(long)row * D + c] : 0.f;
      Op::put(Xh, PX, (PR + r) * SX + c, e);
      if (row < B) a.T1in[(kb + B + row) * l1 + c] = e;
    }
  }
  for (int idx = tid; idx < RT * (dm.K1 - din); idx += blockDim.x) {
    const int r = idx / (dm.K1 - din), c = din + idx % (dm.K1 - din);
    Op::put(Xh, PX, r * SX + c, 0.f);
  }
  for (int r = tid; r < PR; r += blockDim.x) {
    const int row = r0 + r;
    const float tv =
        on(row) ? float(a.bt[row] + a.c * double(a.bh[row])) : 0.f;
    tcol[r] = tv;
    hstep[r] = row < B ? a.bh[row] : 0.f;
    if (row < B) {
      a.T1in[(kb + row) * l1 + din] = tv;
      a.T1in[(kb + row) * l1 + din + 1] = 1.f;
      if (CNF) {
        a.T1in[(kb + B + row) * l1 + din] = 0.f;
        a.T1in[(kb + B + row) * l1 + din + 1] = 0.f;
      }
    }
  }
  __syncthreads();


#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    f32x4 acc[1][NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) acc[0][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (layer == 0)
      gemm<Op, 1, NTW, PD>(acc, Xh, PX, SX, static_cast<const W*>(a.w.packed), dm.nk1, dm.nn1, wave * NTW, 1,
                   NTW, lane);
    else
      gemm<Op, 1, NTW, PD, H / 32>(acc, Ah, PA, SA, static_cast<const W*>(a.w.packed) + dm.off2, dm.nk2, dm.nn2,
                   wave * NTW, 1, NTW, lane);
    __syncthreads();
    const float* bias = layer == 0 ? b1 : b2;
    float* Tin = layer == 0 ? a.T2in : a.T3in;
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      const int n = (wave * NTW + t) * 16 + col;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rq + i;
        float v = acc[0][t][i];
        const bool primal = !CNF || row < PR;
        if (primal) {
          v += bias[n];
          if (layer == 0) v += tcol[row] * w1t[n];
        }
        float act = primal ? fast_tanh(v) : 0.f;
        if (CNF) {
          const float ap = __shfl_xor(act, 32, 64);
          if (!primal) act = (1.f - ap * ap) * v;
        }
        keep[layer][t][i] = primal ? act : v;
        Op::put(Ah, PA, row * SA + n, act);
        const long k = tk(row);
        if (k >= 0) Tin[k * (H + 1) + n] = act;
      }
    }
    __syncthreads();
  }
  // bias features of layers 2 and 3 (0 on tangent rows)
  for (int r = tid; r < RT; r += blockDim.x) {
    const long k = tk(r);
    if (k < 0) continue;
    const float one = (!CNF || r < PR) ? 1.f : 0.f;
    a.T2in[k * (H + 1) + H] = one;
    a.T3in[k * (H + 1) + H] = one;
  }

  // gbar: kappa_z on primal rows, -kappa_l eps on tangent rows
  for (int idx = tid; idx < PR * din; idx += blockDim.x) {
    const int r = idx / din, c = idx % din, row = r0 + r;
    const bool o = on(row);
    const float* ks =
        CL ? cl + ((a.s - 1) * PR + r) * D : a.kap_s + (long)row * D;
    const float kz = o ? ks[c] : 0.f;
    Op::put(Xh, PX, r * SX + c, kz);
    if (row < B) a.T3g[(kb + row) * din + c] = kz;
    if (CNF) {
      const float g = o ? -ks[din] * a.eps[(long)row * D + c] : 0.f;
      Op::put(Xh, PX, (PR + r) * SX + c, g);
      if (row < B) a.T3g[(kb + B + row) * din + c] = g;
    }
  }
  __syncthreads();

  }
  // S2 = gbar W3^T, then S1 = G2 W2^T; epilogues form G2, G1
#pragma unroll
  for (int layer = 1; layer >= 0; --layer) {
    f32x4 acc[1][NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) acc[0][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (layer == 1) {
      if (!ahead) r3.start(wt, dt.nk3, dt.nn3, wave * NTW, 1, NTW, lane);
      r3.template run<1>(acc, Xh, PX, SX);
      r2.start(wt + dt.off2, dt.nk2, dt.nn2, wave * NTW, 1, NTW, lane);
    } else {
      r2.template run<1>(acc, Ah, PA, SA);
      if (ahead && ntiles1 > 0)
        r1.start(wt + dt.off1, dt.nk1, dt.nn1, wave, WV, ntiles1, lane);
    }
    __syncthreads();
    float* Tg = layer == 1 ? a.T2g : a.T1g;
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      const int n = (wave * NTW + t) * 16 + col;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rq + i;
        const float sv = acc[0][t][i], kv = keep[layer][t][i];
        float g;
        if (CNF) {
          const float s_o = __shfl_xor(sv, 32, 64);  // partner row's S
          const float k_o = __shfl_xor(kv, 32, 64);  // partner's keep
          if (row < PR)  // primal: a = kv, tangent pre-activation = k_o
            g = (1.f - kv * kv) * (sv - 2.f * kv * k_o * s_o);
          else  // tangent: tanh' of the primal row
            g = (1.f - k_o * k_o) * sv;
        } else {
          g = (1.f - kv * kv) * sv;
        }
        Op::put(Ah, PA, row * SA + n, g);
        const long k = tk(row);
        if (k >= 0) Tg[k * H + n] = g;
      }
    }
    __syncthreads();
  }

  // mu = G1 W1^T (primal rows); column tiles nb = wave, wave + WV, ...
  {
    const int ntiles = ntiles1;
    f32x4 acc[1][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[0][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (ntiles > 0) {
      if (!ahead)
        r1.start(wt + dt.off1, dt.nk1, dt.nn1, wave, WV, ntiles, lane);
      r1.template run<1>(acc, Ah, PA, SA);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t >= ntiles) continue;
      const int n = (wave + WV * t) * 16 + col;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rq + i;
        if (row < PR) MU[row * din + n] = acc[0][t][i];
      }
    }
  }
  __syncthreads();

  // row updates (or, for the continuous adjoint, mu itself), NU elements
  // a thread at a time: every value they read is loaded before any is
  // written (they write distinct addresses, which the compiler cannot
  // know, so it would otherwise wait for each load in turn)
  // (PF: the next stage's front is requested here, ahead of the updates,
  // which then read only LDS but for lambda at stage 7; unconditionally, so
  // that the front just used is no longer live)
  if constexpr (PF) vjp_front_load<CNF, WV>(nxt, *pf);
  constexpr int NU = CNF ? 1 : 2;
  for (int i0 = tid; i0 < PR * D; i0 += NU * (int)blockDim.x) {
    float lam[NU], lamn[NU], kp[NU][6], h[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int idx = i0 + u * (int)blockDim.x;
      const int r = idx / D, c = idx % D, row = r0 + r;
      if (idx >= PR * D || !on(row) || a.mu_out != nullptr) continue;
      const long o = (long)row * D + c;
      h[u] = hstep[r];
      if (a.s == 7) lam[u] = a.lam[o];
      lamn[u] = CL ? cl[(7 * PR + r) * D + c] : a.lamn[o];
#pragma unroll
      for (int j = 0; j < 6; ++j)
        if (j < a.n)
          kp[u][j] = CL ? cl[(a.kidx[j] * PR + r) * D + c]
                        : a.kap[((long)a.kidx[j] * B + row) * D + c];
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int idx = i0 + u * (int)blockDim.x;
      const int r = idx / D, c = idx % D, row = r0 + r;
      if (idx >= PR * D || !on(row)) continue;
      const long o = (long)row * D + c;
      float mu = c < din ? MU[r * din + c] : 0.f;
      if (a.mu_out != nullptr) {
        a.mu_out[o] = mu;
        continue;
      }
      if (a.s == 7) {
        mu = lam[u] + mu;  // Lambda
        a.lam[o] = mu;
      }
      const float ln = lamn[u] + mu;
      if (CL)
        cl[(7 * PR + r) * D + c] = ln;
      else
        a.lamn[o] = ln;
#pragma unroll
      for (int j = 0; j < 6; ++j)
        if (j < a.n) {
          const float v = kp[u][j] + h[u] * a.coef[j] * mu;
          if (CL)
            cl[(a.kidx[j] * PR + r) * D + c] = v;
          else
            a.kap[((long)a.kidx[j] * B + row) * D + c] = v;
        }
      if (a.s == 1) a.lam[o] = ln;
    }
  }
}

template <class Op, int NTW, bool CNF, int WV>
__global__ __launch_bounds__(64 * WV) __attribute__((
    amdgpu_waves_per_eu(CNF ? 4 : 1))) void vjp_mfma_kernel(MfmaVjpArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  vjp_tile<Op, NTW, CNF, WV>(a, smem_raw);
}

// The stages of one step in one launch (stage 7 first): a tile's rows
// depend on no other tile's, so its workgroup runs the stages in turn, the
// cotangents passing between them through memory (the barrier orders them;
// all of the tile's waves share the compute unit's cache).
// The dense-output part of a step for the tile's PR instances, one
// wavefront per row (the same arithmetic as the separate kernel).
template <int PR, int WV, bool CL>
__device__ __forceinline__ void vjp_dense_rows(const MfmaVjpSteps& v,
                                               float* cl) {
  const VjpDense& d = v.dense;
  const MfmaVjpArgs& a = v.st[0];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int B = a.B, D = a.D;
  for (int r = wave; r < PR; r += WV) {
    const int row = blockIdx.x * PR + r;
    if (row >= B) continue;
    const int n = d.step;
    const bool on = n < d.nacc[row];
    if (d.setup && lane == 0) {
      d.act[row] = on ? kRunning : kSuccess;
      d.bh[row] = on ? float(d.hacc[(long)row * d.cap + n]) : 0.f;
      d.bt[row] = on ? d.tn[(long)row * (d.cap + 1) + n] : 0.0;
    }
    // kappa_j of (row, c): the tile's LDS block or HBM
    auto kap = [&](int j, int c) -> float& {
      return CL ? cl[(j * PR + r) * D + c] : a.kap[((long)j * B + row) * D + c];
    };
    auto lamn = [&](int c) -> float& {
      return CL ? cl[(7 * PR + r) * D + c] : a.lamn[(long)row * D + c];
    };
    for (int c = lane; c < D; c += 64) {
      lamn(c) = 0.f;
      for (int j = 0; j < 7; ++j) kap(j, c) = 0.f;
    }
    if (!on || d.E == 0) continue;
    const double h = d.hacc[(long)row * d.cap + n];
    const double t = d.tn[(long)row * (d.cap + 1) + n];
    const int32_t* own = d.owner + (long)row * d.E;
    for (int e = 0; e < d.E; ++e) {
      if (own[e] != n) continue;
      const float th = float((d.t_eval[(long)row * d.E + e] - t) / h);
      float w[7];
#pragma unroll
      for (int j = 0; j < 7; ++j)
        w[j] = th * (d.P[j][0] +
                     th * (d.P[j][1] + th * (d.P[j][2] + th * d.P[j][3])));
      for (int c = lane; c < D; c += 64) {
        const float g = d.g_eval[((long)row * d.E + e) * D + c];
        for (int j = 0; j < 7; ++j) kap(j, c) += float(h) * w[j] * g;
        lamn(c) += g;
      }
    }
  }
}

// CL: the cotangents stay in LDS through the step (v.cl_off: their block's
// byte offset; the dense-output part must run in the same launch, since it
// is what clears and seeds them).
// PF: the stage fronts are requested a stage ahead (the first one before
// the dense-output part); only with the stored layers and the LDS block.
template <class Op, int NTW, bool CNF, int WV, bool CL, bool PF>
__global__ __launch_bounds__(64 * WV) __attribute__((
    amdgpu_waves_per_eu(CNF ? 4 : 1))) void vjp_steps_kernel(MfmaVjpSteps v) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* cl = CL ? reinterpret_cast<float*>(smem_raw + v.cl_off) : nullptr;
  VjpFront<vjp_ne<CNF ? 8 : 16, WV, 64>(), NTW> f;
  if constexpr (PF) vjp_front_load<CNF, WV>(v.st[0], f);
  if (v.dense.on) {
    vjp_dense_rows<CNF ? 8 : 16, WV, CL>(v, cl);
    __syncthreads();
  }
  for (int i = 0; i < v.n; ++i) {
    vjp_tile<Op, NTW, CNF, WV, CL, PF>(v.st[i], smem_raw, cl, &f,
                                       v.st[i + 1 < v.n ? i + 1 : i], i == 0);
    __syncthreads();
  }
}

template <class Op, int NTW, bool CNF, int WV>
hipError_t launch_vjp_t(const MfmaVjpArgs& a, const MfmaVjpSteps* v,
                        hipStream_t s) {
  constexpr int PR = CNF ? 8 : 16;
  const size_t sm = mfma_smem<Op, NTW, CNF, WV>(a.din);
  if (sm > 65536) return hipErrorInvalidValue;
  if (v != nullptr) {
    // the cotangent block in LDS while it fits beside the kernel's LDS
    MfmaVjpSteps w = *v;
    w.cl_off = (int)((sm + 15) / 16 * 16);
    const size_t smc = w.cl_off + sizeof(float) * 8 * PR * (size_t)a.D;
    bool stored = true;  // every stage reads its stored layers
    for (int i = 0; i < w.n; ++i) stored = stored && w.st[i].act_in;
    // (the fronts a stage ahead: while the kernel's registers allow)
    constexpr bool kPF = !CNF && NTW <= 2;
    if (w.dense.on && smc <= 65536 && stored && kPF && a.din <= 64)
      hipLaunchKernelGGL((vjp_steps_kernel<Op, NTW, CNF, WV, true, kPF>),
                         dim3((a.B + PR - 1) / PR), dim3(64 * WV), smc, s, w);
    else if (w.dense.on && smc <= 65536)
      hipLaunchKernelGGL((vjp_steps_kernel<Op, NTW, CNF, WV, true, false>),
                         dim3((a.B + PR - 1) / PR), dim3(64 * WV), smc, s, w);
    else
      hipLaunchKernelGGL((vjp_steps_kernel<Op, NTW, CNF, WV, false, false>),
                         dim3((a.B + PR - 1) / PR), dim3(64 * WV), sm, s, w);
  } else
    hipLaunchKernelGGL((vjp_mfma_kernel<Op, NTW, CNF, WV>),
                       dim3((a.B + PR - 1) / PR), dim3(64 * WV), sm, s, a);
  return hipGetLastError();
}

template <class Op>
hipError_t pack_all(const MfmaWeights& w, int din, int H, const float* W1,
                    const float* b1, const float* W2, const float* b2,
                    const float* W3, const float* b3, hipStream_t s) {
  typedef typename Op::W W;
  const Dims d = dims(din, H);
  W* p = static_cast<W*>(w.packed);
  PackJob<W> j[6] = {{p, W1, din, H, d.nk1, d.nn1, 0},
                     {p + d.off2, W2, H, H, d.nk2, d.nn2, 0},
                     {p + d.off3, W3, H, din, d.nk3, d.nn3, 0}};
  int n = 3;
  if (w.packedT != nullptr) {
    const DimsT t = dims_t(din, H);
    W* q = static_cast<W*>(w.packedT);
    j[3] = {q, W3, din, din, t.nk3, t.nn3, 1};
    j[4] = {q + t.off2, W2, H, H, t.nk2, t.nn2, 1};
    j[5] = {q + t.off1, W1, H, H, t.nk1, t.nn1, 1};
    n = 6;
  }
  hipLaunchKernelGGL(pack_weights_kernel<W>, dim3(128, n + 1), dim3(256), 0,
                     s, j[0], j[1], j[2], j[3], j[4], j[5], n, w.fvec, W1, b1,
                     b2, b3, din, H);
  return hipGetLastError();
}

// Hidden width -> (column tiles per wavefront, wavefronts): 8 wavefronts
// from H = 128 up, so a tile's layers run on two wavefronts per SIMD; the
// CNF field at H = 512 keeps 4 (8 column tiles each), which measured faster
// for its 8 primal + 8 tangent rows (62 vs 75 us per stage at 8192
// instances), while its VJP is faster on 8.
template <class Op, bool CNF>
hipError_t field_h(const MfmaArgs& a, const MfmaSteps* v, hipStream_t s) {
  const int wv = mfma_waves(a.H, CNF, a.B, a.waves);
  switch (a.H) {
    case 512:
      return wv == 4 ? launch_t<Op, 8, CNF, 4>(a, v, s)
                     : launch_t<Op, 4, CNF, 8>(a, v, s);
    case 256:
      return wv == 4 ? launch_t<Op, 4, CNF, 4>(a, v, s)
                     : launch_t<Op, 2, CNF, 8>(a, v, s);
    case 128:
      return wv == 4 ? launch_t<Op, 2, CNF, 4>(a, v, s)
                     : launch_t<Op, 1, CNF, 8>(a, v, s);
    default: return launch_t<Op, 1, CNF, 4>(a, v, s);
  }
}

template <class Op, bool CNF>
hipError_t vjp_h(const MfmaVjpArgs& a, const MfmaVjpSteps* v, hipStream_t s) {
  switch (a.H) {
    case 512: return launch_vjp_t<Op, 4, CNF, 8>(a, v, s);
    case 256: return launch_vjp_t<Op, 2, CNF, 8>(a, v, s);
    case 128: return launch_vjp_t<Op, 1, CNF, 8>(a, v, s);
    default: return launch_vjp_t<Op, 1, CNF, 4>(a, v, s);
  }
}

}  // namespace

size_t mfma_packed_bytes(int din, int H, int f32) {
  const Dims d = dims(din, H);
  return (d.off3 + (size_t)d.nk3 * d.nn3 * 512) * (f32 ? 4 : 2);
}

size_t mfma_packedT_bytes(int din, int H, int f32) {
  return dims_t(din, H).total * (f32 ? 4 : 2);
}

size_t mfma_fvec_elems(int din, int H) { return 3 * (size_t)H + din; }

int mfma_waves(int H, bool cnf, int B, int requested) {
  if (H <= 64) return 4;  // one 16-column tile per wavefront at most
  if (requested == 4 || requested == 8) return requested;
  // measured defaults: 8 wavefronts (two per SIMD) from width 128 up while
  // the tiles are about one per compute unit; 4 once there are two or more
  // tiles per compute unit, so that two workgroups share one (MLP at width
  // 256, fused solve: 16,384 instances 1.45 -> 1.15 ms, 65,536 5.13 -> 3.98
  // ms, 4096 0.45 vs 0.51 ms on 4); and 4 for the CNF at width 512 (its
  // tangent rows double the epilogue registers; 62 vs 75 us per stage
  // evaluation of 8192 instances)
  if (cnf && H == 512) return 4;
  const long tiles = (B + (cnf ? 7 : 15)) / (cnf ? 8 : 16);
  return H >= 256 && tiles >= 512 ? 4 : 8;
}

std::string mfma_supported(int din, int H) {
  if (din < 16 || din % 16 != 0 || din > 256)
    return "matrix-core fields need a state width that is a multiple of 16, "
           "<= 256";
  if (H != 64 && H != 128 && H != 256 && H != 512)
    return "matrix-core fields are built for hidden widths 64, 128, 256, 512";
  return "";
}

hipError_t mfma_pack_weights(const MfmaWeights& w, int din, int H,
                             const float* W1, const float* b1, const float* W2,
                             const float* b2, const float* W3, const float* b3,
                             hipStream_t s) {
  return w.f32 ? pack_all<F32>(w, din, H, W1, b1, W2, b2, W3, b3, s)
               : pack_all<Bf3>(w, din, H, W1, b1, W2, b2, W3, b3, s);
}

MfmaArgs mfma_args(int B, int D, int din, int H, int cnf, const int32_t* status,
                   const float* y, const float* K, float* Y7, const float* hs,
                   const double* t, const float* eps, const MfmaWeights& w) {
  MfmaArgs a{};
  a.B = B;
  a.D = D;
  a.din = din;
  a.H = H;
  a.cnf = cnf;
  a.status = status;
  a.y = y;
  a.K = K;
  a.Y7 = Y7;
  a.hs = hs;
  a.t = t;
  a.eps = eps;
  a.w = w;
  return a;
}

static hipError_t vjp_any(const MfmaVjpArgs& a, const MfmaVjpSteps* v,
                          hipStream_t s) {
  if (a.w.packedT == nullptr || a.w.plain) return hipErrorInvalidValue;
  if (a.w.f32)
    return a.cnf ? vjp_h<F32, true>(a, v, s) : vjp_h<F32, false>(a, v, s);
  return a.cnf ? vjp_h<Bf3, true>(a, v, s) : vjp_h<Bf3, false>(a, v, s);
}

hipError_t launch_vjp_mfma(const MfmaVjpArgs& a, hipStream_t s) {
  return vjp_any(a, nullptr, s);
}

hipError_t launch_vjp_steps_mfma(const MfmaVjpSteps& v, hipStream_t s) {
  if (v.n < 1 || v.n > 7) return hipErrorInvalidValue;
  return vjp_any(v.st[0], &v, s);
}

static hipError_t field_any(const MfmaArgs& a, const MfmaSteps* v,
                            hipStream_t s) {
  if (a.w.f32)
    return a.cnf ? field_h<F32, true>(a, v, s) : field_h<F32, false>(a, v, s);
  if (a.w.plain)
    return a.cnf ? field_h<Bf1, true>(a, v, s) : field_h<Bf1, false>(a, v, s);
  return a.cnf ? field_h<Bf3, true>(a, v, s) : field_h<Bf3, false>(a, v, s);
}

hipError_t launch_field_mfma(const MfmaArgs& a, int row_tile, hipStream_t s) {
  (void)row_tile;
  return field_any(a, nullptr, s);
}

hipError_t launch_field_steps_mfma(const MfmaSteps& v, hipStream_t s) {
  if (v.n < 1 || v.n > 7) return hipErrorInvalidValue;
  return field_any(v.st[0], &v, s);
}

}  // namespace bode
