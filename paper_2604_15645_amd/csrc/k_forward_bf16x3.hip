// k_forward_bf16x3.hip -- the forward kernels at precision kBF16X3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "k_forward_impl.h"

namespace pinn {

template int fwd_a<kBF16X3>(int act, int H, int P, const FwdArgs& a, int grid, size_t lds, hipStream_t s);

}  // namespace pinn
