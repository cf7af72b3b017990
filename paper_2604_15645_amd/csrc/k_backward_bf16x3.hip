// k_backward_bf16x3.hip -- the backward kernels at precision kBF16X3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "k_backward_impl.h"

namespace pinn {

template int bwd_a<kBF16X3>(int act, int H, bool embed, const BwdArgs& a, int grid, size_t lds, hipStream_t s);

}  // namespace pinn
