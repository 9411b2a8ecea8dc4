// Discrete adjoint of the batched solve (filled in with the neural fields).
#include <hip/hip_runtime.h>

#include "modular.hpp"

namespace bode {

hipError_t modular_backward(ModularPlan&, const void*, const void*, void*,
                            void*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace bode
