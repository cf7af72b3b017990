// k_backward_fp32.hip -- the backward kernels at precision kFP32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "k_backward_impl.h"

namespace pinn {

template int bwd_a<kFP32>(int act, int H, bool embed, const BwdArgs& a, int grid, size_t lds, hipStream_t s);

int launch_backward(int prec, int act, int H, bool embed, const BwdArgs& a, int grid, size_t lds, hipStream_t s) {
  if (prec == kFP32) return bwd_a<kFP32>(act, H, embed, a, grid, lds, s);
  if (prec == kFP16X3) return bwd_a<kFP16X3>(act, H, embed, a, grid, lds, s);
  return bwd_a<kBF16X3>(act, H, embed, a, grid, lds, s);
}


}  // namespace pinn
