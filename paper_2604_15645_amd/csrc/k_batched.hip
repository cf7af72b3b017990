// k_batched.hip -- many independent networks in one persistent launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pinn_device.h"

namespace pinn {

// ================================================================== many networks, one launch

// Work item i: instance items[i].inst, padded points [p0, p1) of that instance (multiples
// of 128).  A work-group takes items from the counter in the order `order` (longest first),
// runs the forward over the item's tiles and then every layer's backward over the same
// points, keeping each layer's weight-gradient sums in registers over the item, and writes
// them with the loss sums to the item's own FP64 slots.  Slots are per item, so the
// result does not depend on which work-group ran which item.
// Largest value of m over the work-group (every thread calls it; red: kWaves floats).
__device__ __forceinline__ float wg_max(float m, float* red) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  float r = red[0];
  for (int w = 1; w < kWaves; ++w) r = fmaxf(r, red[w]);
  return r;
}

template <int PREC, int ACT, int H>
__device__ __forceinline__ void run_item(const BatchArgs& A, const BatchInst& in, const BatchItem& it, int64_t item,
                                         char* smem, float* red) {
  constexpr int PF = H == 256 ? 32 : H == 128 ? 64 : H == 64 ? 64 : 128;
  constexpr int PB = 2048 / H;
  const NetDev& net = in.net;
  float* scratch = A.scratch + (size_t)blockIdx.x * A.scratch_per_wg;
  float* zs = scratch;
  float* zb[2] = {scratch + in.zb_off[0], scratch + in.zb_off[1]};
  const float4* pts = A.pts + in.pts_off + it.p0;
  const int64_t npts = it.p1 - it.p0;
  double* loss_slot = A.loss_slots + (size_t)item * kMaxTerms;
  double* gslot = A.grad_slots + it.slot_off;
  PdeDev pde = A.pde;
  for (int c = 0; c < kMaxOut; ++c) pde.seed_scale[c] = 2.0f * A.lambda_res[c] / (float)in.n;
  // forward over the item's tiles; amx: largest magnitude of the adjoint the forward writes
  // (FP16X3 scales each layer's adjoint by the item's own largest magnitude)
  float amx = 0.0f;
  {
    const FwdLds s = fwd_carve<H, PF>(smem, r_stride(in.kmax));
    const int ld = Tile<PREC>::ld(in.kmax, PF);
    fwd_begin<H, PF>(s, net);
    for (int64_t t = 0; t < npts / PF; ++t) {
      const int64_t nv = in.n - (it.p0 + t * PF);
      TileSeg sg;
      sg.nvalid = nv < 0 ? 0 : (nv > PF ? PF : (int)nv);
      sg.kind = 0;
      sg.term = 0;
      sg.targets = nullptr;
      sg.out_mask = 0;
      sg.lam = 0.0f;
      sg.residual = nullptr;
      fwd_tile<PREC, ACT, H, PF>(net, pde, pts + t * PF, zs, in.zs_stride, zb[0], t * (PF / 4), sg, ld, true, s,
                                 amx);
    }
    const int nL = net.layer[net.L].n_in;
    fwd_end<H, PF>(s, loss_slot, gslot + in.eff_off[net.L], net.d_out, nL, true);
  }
  // backward, hidden layers last to first
  int cur = 0;
  for (int j = net.L - 1; j >= 1; --j) {
    using S = BwdShape<H / 16, H / 16, PB>;
    f4 accw[S::NOBW][S::NIBW];
#pragma unroll
    for (int i = 0; i < S::NOBW; ++i)
#pragma unroll
      for (int k = 0; k < S::NIBW; ++k) accw[i][k] = f4{0.f, 0.f, 0.f, 0.f};
    float bsum[S::NOBW];
#pragma unroll
    for (int i = 0; i < S::NOBW; ++i) bsum[i] = 0.f;
    float asc = 1.0f;
    if constexpr (PREC == kFP16X3) asc = adj_scale<PREC>(__float_as_uint(wg_max(amx, red)));
    amx = 0.0f;
    bwd_range<PREC, ACT, H / 16, H / 16, PB>(net, j, pts, 0, 1, npts / PB, zb[cur], zb[cur ^ 1],
                                             zs + (j - 1) * in.zs_stride, smem, accw, bsum, asc, amx);
    bwd_flush<H / 16, H / 16, PB>(accw, bsum, gslot + in.eff_off[j], net.layer[j].n_out, net.layer[j].n_in,
                                  1.0f / asc);
    cur ^= 1;
  }
  // first layer (identity embedding)
  grad0_range(zb[cur], pts, net.layer[0].n_out, net.d_in, 0, npts / 4, gslot + in.eff_off[0],
              reinterpret_cast<float*>(smem));
  __syncthreads();
}

template <int PREC, int ACT>
__global__ __launch_bounds__(kThreads, 1) void k_batched(const BatchArgs A) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ int s_q;
  __shared__ float s_red[kWaves];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_q = atomicAdd(A.counter, 1);
    __syncthreads();
    const int q = __builtin_amdgcn_readfirstlane(s_q);
    if (q >= A.n_items) break;
    const int64_t item = A.order[q];
    const BatchItem it = A.items[item];
    const BatchInst& in = A.inst[it.inst];
    switch (in.H) {
      case 32: run_item<PREC, ACT, 32>(A, in, it, item, smem, s_red); break;
      case 64: run_item<PREC, ACT, 64>(A, in, it, item, smem, s_red); break;
      case 128: run_item<PREC, ACT, 128>(A, in, it, item, smem, s_red); break;
      default: run_item<PREC, ACT, 256>(A, in, it, item, smem, s_red); break;
    }
  }
}


// ================================================================== launcher

size_t batched_lds(int kmax, int H) {
  const int PF = H == 256 ? 32 : H == 128 ? 64 : H == 64 ? 64 : 128;
  const int PB = 2048 / H;
  const int WN = H / 16 < kWaves ? H / 16 : kWaves;
  const int WC = kWaves / WN;
  size_t f = (size_t)4 * PF * r_stride(kmax) + (size_t)PF * 16 + (size_t)PF * kMaxOut * 4 * 4 * 2 + kWaves * 8 * 4 +
             kMaxTerms * 8 + (size_t)WC * kMaxOut * H * 8 + kMaxOut * 8 + kFourierLds + kOutLds + 16;
  size_t b = bwd_lds_bytes(PB, H, H, true);
  size_t g = (size_t)kWaves * 256 * 4 * sizeof(float);
  size_t m = f > b ? f : b;
  return m > g ? m : g;
}

template <int PREC, int ACT>
int batched_k(const BatchArgs& a, int grid, size_t lds, hipStream_t s) {
  auto k = k_batched<PREC, ACT>;
  if (set_lds(k, lds)) return -5;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, s, a);
  return launch_status(hipGetLastError());
}

template <int PREC>
int batched_a(int act, const BatchArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (act) {
    case kTanh: return batched_k<PREC, kTanh>(a, grid, lds, s);
    case kSin: return batched_k<PREC, kSin>(a, grid, lds, s);
    case kTanh | kLapFlag: return batched_k<PREC, kTanh | kLapFlag>(a, grid, lds, s);
    case kSin | kLapFlag: return batched_k<PREC, kSin | kLapFlag>(a, grid, lds, s);
    default: return -2;
  }
}

int launch_batched(int prec, int act, const BatchArgs& a, int grid, size_t lds, hipStream_t s) {
  if (prec == kFP32) return batched_a<kFP32>(act, a, grid, lds, s);
  if (prec == kFP16X3) return batched_a<kFP16X3>(act, a, grid, lds, s);
  return batched_a<kBF16X3>(act, a, grid, lds, s);
}

}  // namespace pinn
