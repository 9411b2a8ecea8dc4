// Achievable ceilings of the GPU, measured beside the datasheet peaks that
// the roofline fractions are quoted against.  Measurement only: the solver
// library does not use this code.
//
//  - ceil_triad: c = a + s b over n floats (12 bytes per element), the
//    streaming HBM bandwidth a scan-like kernel can reach;
//  - ceil_mfma_bf16 / ceil_mfma_f32: each wavefront issues 8 independent
//    chains of v_mfma_f32_16x16x32_bf16 (16 x 16 x 32 x 2 flops) or
//    v_mfma_f32_16x16x4_f32 (16 x 16 x 4 x 2 flops) on register operands;
//  - ceil_fma_f32: 16 independent chains of scalar-per-lane FP32 FMAs, the
//    vector peak without packed FP32 instructions (which this library never
//    emits).
// Each kernel writes one value per thread so nothing is optimised away.
#include <hip/hip_runtime.h>

#include <cstdint>

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Each thread moves U 16-byte vectors of each operand per iteration, all
// loads issued before the first store (U x 2 loads in flight per lane), with
// non-temporal hints (streamed data is not kept in the caches); consecutive
// lanes touch consecutive vectors, so every load instruction of a wavefront
// covers 1 KiB contiguous.
template <int U>
__global__ __launch_bounds__(256) void triad_kernel(const float* a,
                                                    const float* b, float* c,
                                                    long n, float s) {
  const long nv = n / 4;  // whole vectors
  const f32x4* av = reinterpret_cast<const f32x4*>(a);
  const f32x4* bv = reinterpret_cast<const f32x4*>(b);
  f32x4* cv = reinterpret_cast<f32x4*>(c);
  const long T = (long)gridDim.x * blockDim.x;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long i = t;
  for (; i + (U - 1) * T < nv; i += U * T) {
    f32x4 x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      x[u] = __builtin_nontemporal_load(av + i + u * T);
      y[u] = __builtin_nontemporal_load(bv + i + u * T);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      __builtin_nontemporal_store(x[u] + s * y[u], cv + i + u * T);
  }
  for (; i < nv; i += T) cv[i] = av[i] + s * bv[i];
  if (t == 0)
    for (long k = nv * 4; k < n; ++k) c[k] = a[k] + s * b[k];
}

__global__ __launch_bounds__(256) void mfma_bf16_kernel(float* out,
                                                        int iters) {
  const int lane = threadIdx.x & 63;
  bf16x8 a, b;
  for (int k = 0; k < 8; ++k) {
    a[k] = (__bf16)(0.001f * (lane + k));
    b[k] = (__bf16)(0.002f * (lane - k));
  }
  f32x4 acc[8];
  for (int q = 0; q < 8; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
  }
  float s = 0.f;
  for (int q = 0; q < 8; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  out[(long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void mfma_f32_kernel(float* out, int iters) {
  const int lane = threadIdx.x & 63;
  const float a = 0.001f * lane, b = 0.002f * lane;
  f32x4 acc[8];
  for (int q = 0; q < 8; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
  }
  float s = 0.f;
  for (int q = 0; q < 8; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  out[(long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void fma_f32_kernel(float* out, int iters,
                                                      float m) {
  float x[16];
  for (int q = 0; q < 16; ++q) x[q] = 0.001f * (threadIdx.x + q);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = __builtin_fmaf(x[q], m, 0.5f);
  }
  float s = 0.f;
  for (int q = 0; q < 16; ++q) s += x[q];
  out[(long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

extern "C" {

// c[0, n) = a + s b.  Device pointers; stream may be null.  Returns the HIP
// error code of the launch.
int ceil_triad(const float* a, const float* b, float* c, long n, float s,
               void* stream) {
  if (!a || !b || !c || n < 0) return (int)hipErrorInvalidValue;
  // 16-byte vectors need 16-byte aligned operands
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
       reinterpret_cast<uintptr_t>(c)) % 16 != 0)
    return (int)hipErrorInvalidValue;
  const int blocks = 256 * 8 * 4;
  hipLaunchKernelGGL(triad_kernel<4>, dim3(blocks), dim3(256), 0,
                     (hipStream_t)stream, a, b, c, n, s);
  return (int)hipGetLastError();
}

// ceil_triad with a chosen unroll (1, 2, 4 or 8 vectors per operand in
// flight per lane) and grid (blocks of 256 threads), for a sweep of the
// streaming kernel's shape.
int ceil_triad_shape(const float* a, const float* b, float* c, long n,
                     float s, int unroll, int blocks, void* stream) {
  if (!a || !b || !c || n < 0 || blocks < 1) return (int)hipErrorInvalidValue;
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
       reinterpret_cast<uintptr_t>(c)) % 16 != 0)
    return (int)hipErrorInvalidValue;
  hipStream_t st = (hipStream_t)stream;
  switch (unroll) {
    case 1: hipLaunchKernelGGL(triad_kernel<1>, dim3(blocks), dim3(256), 0, st, a, b, c, n, s); break;
    case 2: hipLaunchKernelGGL(triad_kernel<2>, dim3(blocks), dim3(256), 0, st, a, b, c, n, s); break;
    case 4: hipLaunchKernelGGL(triad_kernel<4>, dim3(blocks), dim3(256), 0, st, a, b, c, n, s); break;
    case 8: hipLaunchKernelGGL(triad_kernel<8>, dim3(blocks), dim3(256), 0, st, a, b, c, n, s); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

// blocks x 256 threads, each wavefront 8 x iters MFMAs; out holds
// blocks x 256 floats.  Flops = blocks * 4 * iters * 8 * (16 16 32 2).
int ceil_mfma_bf16(float* out, int blocks, int iters, void* stream) {
  if (!out || blocks < 1 || iters < 1) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(mfma_bf16_kernel, dim3(blocks), dim3(256), 0,
                     (hipStream_t)stream, out, iters);
  return (int)hipGetLastError();
}

// As ceil_mfma_bf16 with 16 x 16 x 4 FP32 MFMAs.
int ceil_mfma_f32(float* out, int blocks, int iters, void* stream) {
  if (!out || blocks < 1 || iters < 1) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(mfma_f32_kernel, dim3(blocks), dim3(256), 0,
                     (hipStream_t)stream, out, iters);
  return (int)hipGetLastError();
}

// blocks x 256 threads, 16 x iters FMAs each (2 flops per FMA).
int ceil_fma_f32(float* out, int blocks, int iters, void* stream) {
  if (!out || blocks < 1 || iters < 1) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(fma_f32_kernel, dim3(blocks), dim3(256), 0,
                     (hipStream_t)stream, out, iters, 0.999f);
  return (int)hipGetLastError();
}

}  // extern "C"
