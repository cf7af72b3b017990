// pinn_noalloc.hip -- the fused step for callers that cannot allocate device memory: its
// workspace is a fixed-size array of the library's own, one per GPU, held for the life of
// the process.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/pinn.h"
#include "pinn_internal.h"

namespace pinn {
int run_bwd_untimed(const pinn_net* net, const pinn_pde* pde, const float* params, const float* B,
                    const float* points, int64_t n_points, const pinn_anchor* anchors, int n_anchor, int prec,
                    uint32_t flags, const pinn_tune* tune, float* residual, double* loss, double* grad,
                    void* workspace, size_t ws_bytes, pinn_stream_t stream);
}  // namespace pinn

namespace {

// The workspace of pinn_residual_bwd_noalloc.  Host code never uses this name as an
// address (on the host it is a stand-in, not device memory): the device address comes
// from hipGetSymbolAddress, per GPU.
__device__ __align__(256) char scratch[PINN_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` on each GPU, once looked up

// Device address of the scratch array on the current GPU (looked up on the first call made
// with that GPU current, then kept).
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return PINN_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return PINN_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PINN_E_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return PINN_OK;
}

}  // namespace

extern "C" int pinn_residual_bwd_noalloc(const pinn_net* net, const pinn_pde* pde, const float* params,
                                         const float* fourier_B, const float* points, int64_t n_points,
                                         const pinn_anchor* anchors, int n_anchor, int prec, uint32_t flags,
                                         const pinn_tune* tune, float* residual, double* loss, double* grad,
                                         pinn_stream_t stream) {
  size_t need = 0;
  int rc = pinn_workspace_bytes(net, pde, n_points, anchors, n_anchor, prec, 1, tune, &need);
  if (rc) return rc;
  if (need > (size_t)PINN_NOALLOC_MAX_BYTES) return PINN_E_WORKSPACE;  // before any HIP call
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  return pinn::run_bwd_untimed(net, pde, params, fourier_B, points, n_points, anchors, n_anchor, prec, flags, tune,
                               residual, loss, grad, ws, (size_t)PINN_NOALLOC_MAX_BYTES, stream);
}
