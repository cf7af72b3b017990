// k_forward_impl.h -- the fused forward kernel (embedding jets, hidden layers, output layer,
// residual, loss partial sums, adjoint seed, output-layer backward) and its launcher.
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma once
#include "pinn_device.h"

namespace pinn {

template <int PREC, int ACT, int H, int P, int NW = fwd_waves(H, P)>
__global__ __launch_bounds__(64 * NW, 8 / NW) void k_forward(const FwdArgs A) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const FwdLds s = fwd_carve<H, P, NW>(smem, r_stride(A.kmax));
  const int ld = Tile<PREC>::ld(A.kmax, P);
  fwd_begin<H, P, NW>(s, A.net);
  float amx = 0.0f;
  PdeDev pde = A.pde;
  if (A.wscale) {  // a device-side weight of the residual term (causality segments)
    const float w = (float)*A.wscale;
    for (int c = 0; c < kMaxOut; ++c) pde.seed_scale[c] *= w;
  }
  for (int64_t tile = blockIdx.x; tile < A.n_tiles; tile += gridDim.x) {
    const int64_t p0 = tile * P;
    const int sid = seg_of(A.seg, p0);
    const int64_t nv = A.seg.start[sid] + A.seg.n[sid] - p0;
    TileSeg sg;
    sg.nvalid = nv < 0 ? 0 : (nv > P ? P : (int)nv);
    sg.kind = sid == 0 ? 0 : 1;
    sg.term = sid == 0 ? 0 : A.pde.n_res + (sid - 1);
    sg.targets = sid == 0 ? nullptr : A.seg.targets[sid - 1] + (p0 - A.seg.start[sid]) * A.net.d_out;
    sg.out_mask = sid == 0 ? 0 : A.seg.out_mask[sid - 1];
    sg.lam = sid == 0 ? 0.0f : A.seg.lam_anchor[sid - 1];
    sg.residual = (sid == 0 && A.residual) ? A.residual + (p0 - A.seg.start[0]) * A.pde.n_res : nullptr;
    fwd_tile<PREC, ACT, H, P, NW>(A.net, pde, A.work.pts + p0, A.work.zs0, A.work.zs_stride, A.work.zb[0],
                                  tile * (P / 4), sg, ld, A.with_grad != 0, s, amx);
  }
  if constexpr (PREC == kFP16X3)
    if (A.with_grad) amax_publish(amx, &A.work.amax[A.net.L - 1]);
  fwd_end<H, P, NW>(s, A.work.loss_slots + (size_t)blockIdx.x * kMaxTerms,
                A.with_grad ? A.work.out_slots + (size_t)blockIdx.x * A.net.d_out * (A.net.layer[A.net.L].n_in + 1)
                            : nullptr,
                A.net.d_out, A.net.layer[A.net.L].n_in, A.with_grad != 0);
}


// ================================================================== launcher
// (instantiated per precision in k_forward_<precision>.hip, so that the three compile in
// parallel)

namespace {

template <int PREC, int ACT, int H, int P>
int fwd(const FwdArgs& a, int grid, size_t lds, hipStream_t s) {
  auto k = k_forward<PREC, ACT, H, P>;
  if (set_lds(k, lds)) return -5;
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * fwd_waves(H, P)), lds, s, a);
  return launch_status(hipGetLastError());
}

template <int PREC, int ACT, int H>
int fwd_p(int P, const FwdArgs& a, int grid, size_t lds, hipStream_t s) {
  constexpr int PD = fwd_default_p(H), PH = fwd_half_p(H);
  if (P == PD) return fwd<PREC, ACT, H, PD>(a, grid, lds, s);
  if constexpr (PH > 0)
    if (P == PH) return fwd<PREC, ACT, H, PH>(a, grid, lds, s);
  if (P == 16) return fwd<PREC, ACT, H, 16>(a, grid, lds, s);
  return -2;
}

template <int PREC, int ACT>
int fwd_h(int H, int P, const FwdArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (H) {
    case 32: return fwd_p<PREC, ACT, 32>(P, a, grid, lds, s);
    case 64: return fwd_p<PREC, ACT, 64>(P, a, grid, lds, s);
    case 128: return fwd_p<PREC, ACT, 128>(P, a, grid, lds, s);
    case 256: return fwd_p<PREC, ACT, 256>(P, a, grid, lds, s);
    default: return -2;
  }
}

}  // namespace

template <int PREC>
int fwd_a(int act, int H, int P, const FwdArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (act) {
    case kTanh: return fwd_h<PREC, kTanh>(H, P, a, grid, lds, s);
    case kSin: return fwd_h<PREC, kSin>(H, P, a, grid, lds, s);
    case kTanh | kLapFlag: return fwd_h<PREC, kTanh | kLapFlag>(H, P, a, grid, lds, s);
    case kSin | kLapFlag: return fwd_h<PREC, kSin | kLapFlag>(H, P, a, grid, lds, s);
    default: return -2;
  }
}

// Each precision is instantiated in its own translation unit.
extern template int fwd_a<kFP32>(int act, int H, int P, const FwdArgs& a, int grid, size_t lds, hipStream_t s);
extern template int fwd_a<kBF16X3>(int act, int H, int P, const FwdArgs& a, int grid, size_t lds, hipStream_t s);
extern template int fwd_a<kFP16X3>(int act, int H, int P, const FwdArgs& a, int grid, size_t lds, hipStream_t s);

}  // namespace pinn
