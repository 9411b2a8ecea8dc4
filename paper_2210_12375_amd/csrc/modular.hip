// Neural right-hand sides (MLP / CNF): batched modular solver.
#include <hip/hip_runtime.h>

#include "modular.hpp"

namespace bode {

__global__ void count_equal_kernel(const int32_t* a, int n, int32_t v,
                                   int32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool hit = i < n && a[i] == v;
  const unsigned long long m = __ballot(hit);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(out, (int)__popcll(m));
}

hipError_t launch_count_equal(const int32_t* a, int n, int32_t v, int32_t* out,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(count_equal_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     s, a, n, v, out);
  return hipGetLastError();
}

size_t modular_layout(const bode_config&, void*, ModularPlan*) { return 256; }
std::string modular_supported(const bode_config&) {
  return "neural right-hand sides are not built yet";
}
hipError_t modular_init(ModularPlan&, const bode_config&, const bode_problem&,
                        hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t modular_run(ModularPlan&, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t modular_eval(ModularPlan&, const double*, void*, int32_t*,
                        hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t modular_backward(ModularPlan&, const void*, const void*, void*,
                            void*, hipStream_t) {
  return hipErrorNotSupported;
}
void modular_release(ModularPlan&) {}

}  // namespace bode
