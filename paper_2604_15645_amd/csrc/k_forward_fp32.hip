// k_forward_fp32.hip -- the forward kernels at precision kFP32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "k_forward_impl.h"

namespace pinn {

template int fwd_a<kFP32>(int act, int H, int P, const FwdArgs& a, int grid, size_t lds, hipStream_t s);

int launch_forward(int prec, int act, int H, int P, const FwdArgs& a, int grid, size_t lds, hipStream_t s) {
  if (prec == kFP32) return fwd_a<kFP32>(act, H, P, a, grid, lds, s);
  if (prec == kFP16X3) return fwd_a<kFP16X3>(act, H, P, a, grid, lds, s);
  return fwd_a<kBF16X3>(act, H, P, a, grid, lds, s);
}


}  // namespace pinn
