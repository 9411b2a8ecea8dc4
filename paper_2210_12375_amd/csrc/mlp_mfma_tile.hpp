// Device building blocks of the neural-field kernels on the matrix cores of
// gfx950, shared by the per-stage field kernel, the adjoint-stage kernel
// and the fused persistent solver.
//
// Two operand policies: BF16 mode (Bf3) issues v_mfma_f32_16x16x32_bf16
// with BF16 weights and activations split into three BF16 terms hi + mid +
// lo (24 significant bits, FP32's precision, so activation rounding does not
// masquerade as local error at tolerances near 1e-5); FP32 mode (F32) issues
// v_mfma_f32_16x16x4_f32 with FP32 weights and activations (each 32-wide k
// block is eight 4-wide products over the same lane layout, so packing and
// LDS addressing are shared).  Weights are packed once per solve into 16x32
// B-fragments (64 lanes x 8 elements contiguous per fragment), read straight
// from L2 by each wavefront.  Accumulation is FP32; biases, the time input
// (a rank-1 term t * W1[t, :]) and tanh are applied in the epilogue, whose
// output goes back to LDS for the next layer.
//
// For the CNF field the tangent rows (the Jacobian-vector product with the
// Rademacher probe) are stacked under the primal rows of the same 16-row
// MFMA tile (8 + 8): the tangent epilogue takes tanh' from the partner lane
// (lane ^ 32 holds the same column of the primal row 8 above).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "mlp_mfma.hpp"

namespace bode {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace mtile {

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u)  // inf / nan stay inf / nan
    return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return uint16_t(u >> 16);
}


struct Dims {
  int K1, nk1, nn1, nk2, nn2, nk3, nn3;
  size_t off2, off3;  // packed offsets (elements) of layers 2 and 3
};

__host__ __device__ inline Dims dims(int din, int H) {
  Dims d;
  d.K1 = (din + 31) / 32 * 32;
  d.nk1 = d.K1 / 32;
  d.nn1 = H / 16;
  d.nk2 = H / 32;
  d.nn2 = H / 16;
  d.nk3 = H / 32;
  d.nn3 = din / 16;
  d.off2 = (size_t)d.nk1 * d.nn1 * 512;
  d.off3 = d.off2 + (size_t)d.nk2 * d.nn2 * 512;
  return d;
}

// Packed layout: fragment f = kb * nn + nb, lane l, element i holds
// M[kb*32 + (l/16)*8 + i][nb*16 + l%16] (zero beyond K rows), where M is a
// layer W or its transpose.
//
// Transposed layers: W3^T [din x H], W2^T [H x H], W1^T [H x din].
struct DimsT {
  int nk3, nn3, nk2, nn2, nk1, nn1;
  size_t off2, off1, total;
};

__host__ __device__ inline DimsT dims_t(int din, int H) {
  DimsT d;
  d.nk3 = (din + 31) / 32;
  d.nn3 = H / 16;
  d.nk2 = H / 32;
  d.nn2 = H / 16;
  d.nk1 = H / 32;
  d.nn1 = din / 16;
  d.off2 = (size_t)d.nk3 * d.nn3 * 512;
  d.off1 = d.off2 + (size_t)d.nk2 * d.nn2 * 512;
  d.total = d.off1 + (size_t)d.nk1 * d.nn1 * 512;
  return d;
}

__device__ __forceinline__ bf16x8 lds8(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

__device__ __forceinline__ bf16x8 gld8(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// v = hi + mid + lo in bf16 (terms at Ah, Ah + plane, Ah + 2 plane), by
// truncation: hi keeps v's top 16 bits (8 significant), the residual v - hi
// is exact with at most 16 significant bits, mid keeps its top 8, and the
// last residual has at most 8, so it is a bf16 value: the sum is v exactly.
__device__ __forceinline__ void put_split(uint16_t* Ah, int plane, int off,
                                          float v) {
  const uint32_t u = __float_as_uint(v);
  const float r1 = v - __uint_as_float(u & 0xffff0000u);
  const uint32_t u1 = __float_as_uint(r1);
  const float r2 = r1 - __uint_as_float(u1 & 0xffff0000u);
  Ah[off] = uint16_t(u >> 16);
  Ah[plane + off] = uint16_t(u1 >> 16);
  Ah[2 * plane + off] = uint16_t(__float_as_uint(r2) >> 16);
}

// tanh x = 1 - 2 / (1 + e^{2x}), e^{2x} = 2^(2 x log2 e) by the hardware
// exp2 and reciprocal: absolute error about 1e-7 (FP32's own rounding of an
// activation), and the limits come out exactly (e^{2x} = inf gives 1, 0
// gives -1).
__device__ __forceinline__ float fast_tanh(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);
  return 1.f - 2.f * __builtin_amdgcn_rcpf(1.f + e);
}

// k blocks of weight fragments a product keeps in flight: about 64
// registers of ring (regs: registers per fragment), between 2 and 8 blocks.
constexpr int ring_depth(int ntw, int regs) {
  return 64 / (ntw * regs) < 2 ? 2 : (64 / (ntw * regs) > 8 ? 8 : 64 / (ntw * regs));
}

struct f32x8 {
  f32x4 lo, hi;
};

// Weight fragments of the next P k blocks of a tile product (NK > 0: the
// product has NK blocks, known at compile time), held in registers.
template <class F, int NTW, int P, int NK>
struct Ring {
  static constexpr int kP = NK > 0 && NK < P ? NK : P, kNK = NK;
  F f[kP][NTW];
};

// Requests the ring's first blocks.  Called ahead of the product (at the
// start of the layer before, say), so their L2 latency overlaps other work.
template <int NTW, class R, class Load>
__device__ __forceinline__ void ring_start(R& r, int nk, int ntiles,
                                           Load load) {
  const int n = R::kNK > 0 ? R::kNK : nk;
#pragma unroll
  for (int p = 0; p < R::kP; ++p)
    if (p < n)
#pragma unroll
      for (int t = 0; t < NTW; ++t)
        r.f[p][t] = load(p, t < ntiles ? t : 0);
  if constexpr (R::kP > 2) __builtin_amdgcn_sched_barrier(0);
}

// The k loop over nk blocks of 32: block kb's products (body), then block
// kb + kP requested into the registers block kb used (a block's L2 latency
// overlaps the products of the kP - 1 blocks before it).  The refills are
// unconditional (blocks past the last re-read valid fragments), so the
// compiler waits for each fragment exactly when it is used; the scheduler
// is kept from sinking them next to their use.
template <int NTW, class R, class Load, class Body>
__device__ __forceinline__ void ring_run(R& r, int nk, int ntiles, Load load,
                                         Body body) {
  constexpr int PP = R::kP;
  auto fill = [&](auto& d, int kb) {
#pragma unroll
    for (int t = 0; t < NTW; ++t) d[t] = load(kb, t < ntiles ? t : 0);
    if constexpr (PP > 2) __builtin_amdgcn_sched_barrier(0);
  };
  if constexpr (R::kNK > 0) {
#pragma unroll
    for (int kb = 0; kb < R::kNK; ++kb) {
      body(kb, r.f[kb % PP]);
      if (kb + PP < R::kNK) fill(r.f[kb % PP], kb + PP);
    }
  } else {
    for (int k0 = 0; k0 < nk; k0 += PP) {
#pragma unroll
      for (int p = 0; p < PP; ++p) {
        const int kb = k0 + p;
        if (kb >= nk) break;
        body(kb, r.f[p]);
        fill(r.f[p], kb + PP < nk ? kb + PP : nk - 1);
      }
    }
  }
}

// Operand policies.  Each has a fragment type Frag (one lane's share of a
// 32 x 16 weight block), frag() to load one, and block() to issue the
// products of one k block of 32 for MT 16-row tiles and NTW column tiles.

struct Bf3 {
  typedef uint16_t W;  // packed weight element
  typedef uint16_t A;  // LDS activation element
  typedef bf16x8 Frag;
  static constexpr int kPlanes = 3, kPad = 8, kFragRegs = 4;
  __device__ static __forceinline__ void put(A* p, int plane, int off,
                                             float v) {
    put_split(p, plane, off, v);
  }
  __device__ static __forceinline__ Frag frag(const W* Bp, long f, int lane) {
    return gld8(Bp + (f * 64 + lane) * 8);
  }
  // C[MT][NTW] += A(LDS hi + mid + lo at Ah, Ah + plane, Ah + 2 plane;
  // columns kb * 32 ..) x B(block kb of the column tiles)
  template <int MT, int NTW>
  __device__ static __forceinline__ void block(f32x4 (&acc)[MT][NTW],
                                               const A* Ah, int plane,
                                               int lda, int kb,
                                               const Frag (&b)[NTW],
                                               int ntiles, int lane) {
    const int r = lane & 15, kq = (lane >> 4) * 8;
    bf16x8 ah[MT], am[MT], al[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int off = (mt * 16 + r) * lda + kb * 32 + kq;
      ah[mt] = lds8(Ah + off);
      am[mt] = lds8(Ah + plane + off);
      al[mt] = lds8(Ah + 2 * plane + off);
    }
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      if (t < ntiles) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          acc[mt][t] = mfma(al[mt], b[t], acc[mt][t]);
          acc[mt][t] = mfma(am[mt], b[t], acc[mt][t]);
          acc[mt][t] = mfma(ah[mt], b[t], acc[mt][t]);
        }
      }
    }
  }
};

// Plain BF16 policy: the same BF16 weights, but every activation rounded
// once to the nearest BF16 value (8 significant bits) and one MFMA per
// fragment: a third of Bf3's matrix-core work, at the price of activation
// rounding of relative size 2^-9 in every layer.
struct Bf1 {
  typedef uint16_t W;
  typedef uint16_t A;
  typedef bf16x8 Frag;
  static constexpr int kPlanes = 1, kPad = 8, kFragRegs = 4;
  __device__ static __forceinline__ void put(A* p, int, int off, float v) {
    p[off] = f2bf(v);
  }
  __device__ static __forceinline__ Frag frag(const W* Bp, long f, int lane) {
    return gld8(Bp + (f * 64 + lane) * 8);
  }
  template <int MT, int NTW>
  __device__ static __forceinline__ void block(f32x4 (&acc)[MT][NTW],
                                               const A* Ah, int, int lda,
                                               int kb, const Frag (&b)[NTW],
                                               int ntiles, int lane) {
    const int r = lane & 15, kq = (lane >> 4) * 8;
    bf16x8 ah[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      ah[mt] = lds8(Ah + (mt * 16 + r) * lda + kb * 32 + kq);
#pragma unroll
    for (int t = 0; t < NTW; ++t)
      if (t < ntiles)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt][t] = mfma(ah[mt], b[t], acc[mt][t]);
  }
};

// FP32 policy: A and B fragments are 8 FP32 values per lane; product q of
// a 32-wide k block takes element q of both (the 4 k indices of one
// 16x16x4 product are kb*32 + g*8 + q, g = lane / 16).
struct F32 {
  typedef float W;
  typedef float A;
  typedef f32x8 Frag;
  static constexpr int kPlanes = 1, kPad = 4, kFragRegs = 8;
  __device__ static __forceinline__ void put(A* p, int, int off, float v) {
    p[off] = v;
  }
  __device__ static __forceinline__ Frag frag(const W* Bp, long f, int lane) {
    const W* q = Bp + (f * 64 + lane) * 8;
    return f32x8{*reinterpret_cast<const f32x4*>(q),
                 *reinterpret_cast<const f32x4*>(q + 4)};
  }
  template <int MT, int NTW>
  __device__ static __forceinline__ void block(f32x4 (&acc)[MT][NTW],
                                               const A* Ah, int, int lda,
                                               int kb, const Frag (&b)[NTW],
                                               int ntiles, int lane) {
    const int r = lane & 15, kq = (lane >> 4) * 8;
    f32x4 a0[MT], a1[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const A* q = Ah + (mt * 16 + r) * lda + kb * 32 + kq;
      a0[mt] = *reinterpret_cast<const f32x4*>(q);
      a1[mt] = *reinterpret_cast<const f32x4*>(q + 4);
    }
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      if (t < ntiles) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                a0[mt][q], b[t].lo[q], acc[mt][t], 0, 0, 0);
#pragma unroll
          for (int q = 0; q < 4; ++q)
            acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                a1[mt][q], b[t].hi[q], acc[mt][t], 0, 0, 0);
        }
      }
    }
  }
};

// A layer product's weight ring: NTW column tiles nb0 + t * nstep of the
// packed layer at Bp (nn column tiles a k block), P blocks in flight.
template <class Op, int NTW, int P = ring_depth(NTW, Op::kFragRegs),
          int NK = 0>
struct WRing {
  Ring<typename Op::Frag, NTW, P, NK> r;
  const typename Op::W* Bp;
  int nk, nn, nb0, nstep, ntiles, lane;
  __device__ __forceinline__ typename Op::Frag load(int kb, int t) const {
    return Op::frag(Bp, (long)kb * nn + nb0 + t * nstep, lane);
  }
  __device__ __forceinline__ void start(const typename Op::W* bp, int nk_,
                                        int nn_, int nb0_, int nstep_,
                                        int ntiles_, int lane_) {
    Bp = bp;
    nk = nk_;
    nn = nn_;
    nb0 = nb0_;
    nstep = nstep_;
    ntiles = ntiles_;
    lane = lane_;
    ring_start<NTW>(r, nk, ntiles, [&](int kb, int t) { return load(kb, t); });
  }
  // C[MT][NTW] += A (LDS, Op's layout) x the layer
  template <int MT>
  __device__ __forceinline__ void run(f32x4 (&acc)[MT][NTW],
                                      const typename Op::A* Ah, int plane,
                                      int lda) {
    ring_run<NTW>(r, nk, ntiles, [&](int kb, int t) { return load(kb, t); },
                  [&](int kb, const typename Op::Frag(&b)[NTW]) {
                    Op::template block<MT, NTW>(acc, Ah, plane, lda, kb, b,
                                                ntiles, lane);
                  });
  }
};

// C[MT][NTW] += A(LDS at Ah, K = 32 nk) x B(packed layer at Bp, column
// tiles nb0 + t * nstep, t < ntiles), the weights requested here.
template <class Op, int MT, int NTW, int P = ring_depth(NTW, Op::kFragRegs),
          int NK = 0>
__device__ __forceinline__ void gemm(f32x4 (&acc)[MT][NTW],
                                     const typename Op::A* Ah, int plane,
                                     int lda, const typename Op::W* Bp, int nk,
                                     int nn, int nb0, int nstep, int ntiles,
                                     int lane) {
  WRing<Op, NTW, P, NK> w;
  w.start(Bp, nk, nn, nb0, nstep, ntiles, lane);
  w.template run<MT>(acc, Ah, plane, lda);
}

// The field for the 16-row tile starting at instance r0 (MLP: 16
// instances; CNF: 8 instances and their 8 tangent rows), by a workgroup of
// WV wavefronts; NTW = H / (16 WV) column tiles per wavefront in the hidden
// layers.  smem_raw: mfma_smem<Op, NTW, CNF, WV>(din) bytes of LDS.
// DEEP: several k blocks of weights in flight (ring_depth) and the layer
// values stored to a.act_out when it is set; otherwise two blocks and no
// layer store, which keeps the persistent solve kernels (the field, the
// error norm and the controller in one body) within their registers.
// KL: the stage values are a [7][rows][D] block in LDS at kl (the fused
// solve keeps its tile's stages there) instead of the [7, B, D] array a.K;
// the output is stage a.kslot of that block.
template <class Op, int NTW, bool CNF, int WV, bool DEEP = true,
          bool KL = false>
__device__ __forceinline__ void field_tile(const MfmaArgs& a, int r0,
                                           unsigned char* smem_raw,
                                           float* kl = nullptr) {
  constexpr int MT = 1;
  typedef typename Op::A A;
  typedef typename Op::W W;
  constexpr int RT = 16 * MT;
  constexpr int PR = CNF ? 8 : RT;  // instances per workgroup
  constexpr int H = NTW * 16 * WV;
  constexpr int SA = H + Op::kPad;  // LDS row stride (bank spread)
  constexpr int PH = DEEP ? ring_depth(NTW, Op::kFragRegs) : 2,
                P4 = DEEP ? ring_depth(4, Op::kFragRegs) : 2,
                NKH = DEEP ? H / 32 : 0;
  const int din = a.din, D = a.D, B = a.B;
  const Dims dm = dims(din, H);
  const int SX = dm.K1 + Op::kPad;
  const int PX = RT * SX, PA = RT * SA;  // split-term planes
  A* Xh = reinterpret_cast<A*>(smem_raw);
  A* Ah = Xh + Op::kPlanes * PX;
  float* tcol = reinterpret_cast<float*>(Ah + Op::kPlanes * PA);  // [PR]
  float* red = tcol + PR;                                 // [PR][nn3]
  __shared__ int any_running;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Weight rings of the three layers.  DEEP: each is requested one phase
  // ahead (layer 1's at entry, layer 2's after layer 1's products, layer
  // 3's after layer 2's), so its first blocks arrive during other work.
  const W* wp = static_cast<const W*>(a.w.packed);
  const int ntiles3 = (dm.nn3 - wave + WV - 1) / WV;
  WRing<Op, NTW, DEEP ? (PH < 4 ? PH : 4) : 2> w1;
  WRing<Op, NTW, PH, NKH> w2;
  WRing<Op, 4, P4, NKH> w3;
  if constexpr (DEEP) w1.start(wp, dm.nk1, dm.nn1, wave * NTW, 1, NTW, lane);

  if (tid == 0) any_running = 0;
  __syncthreads();
  if (tid < PR && r0 + tid < B && a.status[r0 + tid] == kRunning)
    any_running = 1;
  __syncthreads();
  if (!any_running) return;

  // prologue: stage input (FP32) -> split bf16 in LDS; tangent rows = probe.
  // Two elements a thread at a time, every load first (at clamped rows):
  // the stage-input store may alias them as far as the compiler knows, so
  // loads after it would each wait for the one before.
  // (The time column's t and h, and for the CNF the probe, are requested
  // with the first elements' loads, so the prologue waits once.)
  double tt = 0.0;
  float th = 0.f;
  for (int i0 = tid; i0 < PR * D; i0 += 2 * (int)blockDim.x) {
    float kv[2][6], yv[2], hv[2], ev[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int idx = i0 + u * (int)blockDim.x;
      const int ii = idx < PR * D ? idx : 0;
      const int c = ii % D, row = r0 + ii / D < B ? r0 + ii / D : B - 1;
#pragma unroll
      for (int j = 0; j < 6; ++j)
        kv[u][j] = j >= a.n ? 0.f
                   : KL     ? kl[(a.kidx[j] * PR + ii / D) * D + c]
                            : a.K[((long)a.kidx[j] * B + row) * D + c];
      yv[u] = a.y[(long)row * D + c];
      hv[u] = a.hs[row];
      ev[u] = CNF ? a.eps[(long)row * D + c] : 0.f;
    }
    if (i0 == tid && tid < PR) {
      const int row = r0 + tid < B ? r0 + tid : B - 1;
      tt = a.t[row];
      th = a.hs[row];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int idx = i0 + u * (int)blockDim.x;
      if (idx >= PR * D) continue;
      const int r = idx / D, c = idx % D, row = r0 + r;
      float Yv = 0.f;
      if (row < B) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < 6; ++j)
          if (j < a.n) acc += a.coef[j] * kv[u][j];
        Yv = yv[u] + hv[u] * acc;
        if (a.write_y7) a.Y7[(long)row * D + c] = Yv;  // stage input out
      }
      if (c < din) {
        Op::put(Xh, PX, r * SX + c, Yv);
        if (CNF) Op::put(Xh, PX, (PR + r) * SX + c, row < B ? ev[u] : 0.f);
      }
    }
  }
  const float tv = float(tt + a.c * double(th));
  for (int idx = tid; idx < RT * (dm.K1 - din); idx += blockDim.x) {
    const int r = idx / (dm.K1 - din), c = din + idx % (dm.K1 - din);
    Op::put(Xh, PX, r * SX + c, 0.f);
  }
  if (tid < PR) tcol[tid] = r0 + tid < B ? tv : 0.f;
  __syncthreads();

  const float* b1 = a.w.fvec;
  const float* w1t = b1 + H;
  const float* b2 = b1 + 2 * H;
  const float* b3 = b1 + 3 * H;
  const int rq = (lane >> 4) * 4, col = lane & 15;

  // hidden layers: wave w owns column tiles w * NTW .. w * NTW + NTW - 1
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    f32x4 acc[MT][NTW];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int t = 0; t < NTW; ++t) acc[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the layer's bias (and time weight) at this lane's columns, requested
    // ahead of the products: in the epilogue they would be re-read after
    // every store that might alias them
    constexpr bool kHoist = DEEP || NTW <= 4;
    float bn[NTW], wn[NTW];
    if constexpr (kHoist) {
      const float* bias = layer == 0 ? b1 : b2;
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        const int n = (wave * NTW + t) * 16 + col;
        bn[t] = bias[n];
        wn[t] = layer == 0 ? w1t[n] : 0.f;
      }
    }
    if (layer == 0) {
      if constexpr (!DEEP)
        w1.start(wp, dm.nk1, dm.nn1, wave * NTW, 1, NTW, lane);
      w1.template run<MT>(acc, Xh, PX, SX);
      if constexpr (DEEP)
        w2.start(wp + dm.off2, dm.nk2, dm.nn2, wave * NTW, 1, NTW, lane);
    } else {
      if constexpr (!DEEP)
        w2.start(wp + dm.off2, dm.nk2, dm.nn2, wave * NTW, 1, NTW, lane);
      w2.template run<MT>(acc, Ah, PA, SA);
      if (DEEP && ntiles3 > 0)
        w3.start(wp + dm.off3, dm.nk3, dm.nn3, wave, WV, ntiles3, lane);
    }
    __syncthreads();  // every wave has read its layer input
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        const int n = (wave * NTW + t) * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = mt * 16 + rq + i;
          float v = acc[mt][t][i];
          const bool primal = !CNF || row < PR;
          if (primal) {
            if constexpr (kHoist) {
              v += bn[t];
              if (layer == 0) v += tcol[row] * wn[t];
            } else {
              v += (layer == 0 ? b1 : b2)[n];
              if (layer == 0) v += tcol[row] * w1t[n];
            }
          }
          float act = primal ? fast_tanh(v) : 0.f;
          if (CNF) {
            const float ap = __shfl_xor(act, 32, 64);  // primal of row - 8
            if (!primal) act = (1.f - ap * ap) * v;
          }
          Op::put(Ah, PA, row * SA + n, act);
          if (DEEP && a.act_out != nullptr) {
            const int g = r0 + (primal ? row : row - PR);
            if (g < B)
              a.act_out[((long)(g + (primal ? 0 : B)) * 2 + layer) * H + n] =
                  primal ? act : v;
          }
        }
      }
    __syncthreads();
  }

  // output layer: column tiles nb = wave, wave + WV, ...
  {
    const int ntiles = ntiles3;
    f32x4 acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // output bias and (CNF tangent rows, DEEP) probe values, ahead of the
    // products
    float b3n[4], ep[MT][4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int n = (wave + WV * t) * 16 + col;
      b3n[t] = t < ntiles ? b3[n] : 0.f;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = mt * 16 + rq + i, row = r0 + r - PR;
          ep[mt][t][i] = DEEP && CNF && t < ntiles && r >= PR && row < B
                             ? a.eps[(long)row * D + n]
                             : 0.f;
        }
    }
    if (ntiles > 0) {
      if constexpr (!DEEP)
        w3.start(wp + dm.off3, dm.nk3, dm.nn3, wave, WV, ntiles, lane);
      w3.template run<MT>(acc, Ah, PA, SA);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t >= ntiles) continue;
        const int nb = wave + WV * t;
        const int n = nb * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = mt * 16 + rq + i;
          const float v = acc[mt][t][i];
          if (!CNF || r < PR) {
            const int row = r0 + r;
            if (KL)
              kl[(a.kslot * PR + r) * D + n] = v + b3n[t];
            else if (row < B)
              a.out[(long)row * D + n] = v + b3n[t];
          } else {
            // tangent row: eps_n * (dg/dz eps)_n, summed over the 16 columns
            const int pr = r - PR, row = r0 + pr;
            float q = DEEP ? ep[mt][t][i] * v
                           : (row < B ? a.eps[(long)row * D + n] * v : 0.f);
            q += __shfl_xor(q, 1, 64);
            q += __shfl_xor(q, 2, 64);
            q += __shfl_xor(q, 4, 64);
            q += __shfl_xor(q, 8, 64);
            if (col == 0) red[pr * dm.nn3 + nb] = q;
          }
        }
      }
    if (CNF) {
      __syncthreads();
      for (int pr = tid; pr < PR; pr += blockDim.x) {
        const int row = r0 + pr;
        float q = 0.f;
        for (int nb = 0; nb < dm.nn3; ++nb) q += red[pr * dm.nn3 + nb];
        if (KL)
          kl[(a.kslot * PR + pr) * D + din] = -q;
        else if (row < B)
          a.out[(long)row * D + din] = -q;
      }
    }
  }
}

template <class Op, int NTW, bool CNF, int WV>
__host__ __device__ inline size_t mfma_smem(int din) {
  constexpr int MT = 1;
  constexpr int RT = 16 * MT, PR = CNF ? 8 : RT, H = NTW * 16 * WV;
  const Dims dm = dims(din, H);
  return sizeof(typename Op::A) * Op::kPlanes *
             ((size_t)RT * (dm.K1 + Op::kPad) + RT * (H + Op::kPad)) +
         sizeof(float) * (PR + PR * dm.nn3);
}

}  // namespace mtile
}  // namespace bode
