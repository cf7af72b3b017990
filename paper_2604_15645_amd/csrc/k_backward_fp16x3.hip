// k_backward_fp16x3.hip -- the backward kernels at precision kFP16X3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "k_backward_impl.h"

namespace pinn {

template int bwd_a<kFP16X3>(int act, int H, bool embed, const BwdArgs& a, int grid, size_t lds, hipStream_t s);

}  // namespace pinn
