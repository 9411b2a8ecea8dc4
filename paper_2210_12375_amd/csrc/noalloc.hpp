// Device scratch of solver_solve_noalloc (defined in noalloc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace bode {

// Size of the static device array: 32 MiB per GPU.
constexpr size_t kNoallocBytes = size_t(32) << 20;

// Device address of the calling thread's current device's copy of the
// array, looked up with hipGetSymbolAddress on the first call for that
// device and cached.  256-byte aligned.
hipError_t noalloc_scratch(void** out);

}  // namespace bode
