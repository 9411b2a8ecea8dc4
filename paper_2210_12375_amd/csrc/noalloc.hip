// Library-owned device scratch of solver_solve_noalloc.
//
// The array below is the workspace of that entry point, for callers that
// cannot allocate device memory.  Each GPU the library runs on holds its own
// copy (kNoallocBytes) from the load of the code object until the process
// ends.  In host code the array's name is only a host-side stand-in, so its
// device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and only that address is ever handed to
// kernels or copies.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "noalloc.hpp"

static __device__ __align__(256) unsigned char scratch[bode::kNoallocBytes];

namespace bode {

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device ordinal -> address of scratch
}  // namespace

hipError_t noalloc_scratch(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (ptr == nullptr || reinterpret_cast<uintptr_t>(ptr) % 256 != 0)
    return hipErrorInvalidSymbol;
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return hipSuccess;
}

}  // namespace bode
