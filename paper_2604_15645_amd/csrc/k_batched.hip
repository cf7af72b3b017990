// k_batched.hip -- many independent networks in one persistent launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pinn_device.h"

namespace pinn {

// ================================================================== many networks, one launch

// Work item i: instance items[i].inst, padded points [p0, p1) of that instance (multiples
// of 128).  A work-group takes items from the counter in the order `order` (longest first),
// runs the forward over the item's tiles and then every layer's backward over the same
// points, keeping each layer's weight-gradient sums in registers over the item (bf16x3 at
// width 256: in a second pass after the input adjoint, so that neither the weights nor the
// sums have to be streamed), and writes them with the loss sums to the item's own FP64
// slots.  Slots are per item, so the
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

// Backward of hidden layer j (n_in = n_out = H = 256, bf16x3) over the item's
// n_sub sub-tiles of PB points in two passes: first the input adjoint with the layer's
// weight fragments resident in registers (written to zb_out, with the activation adjoint),
// then the weight gradient with its sums resident, the output adjoint and the
// pre-activations read a second time.  The same loops as the two roles of the split-role
// kernel, one after the other in one work-group: the weights are read once per item and
// layer instead of once per sub-tile.  Sums go to the item's slot [n_out][n_in], [n_out].
// With g0_slot (layer 1 over an identity embedding, points pts) the input adjoint is not
// written: the first layer's weight and bias sums are formed from it in pass 1 and go to
// g0_slot [n_in][d_in], [n_in].
template <int PREC, int ACT, int H>
__device__ __noinline__ void item_layer_two_pass(const NetDev& net, int j, int64_t n_sub, const float* zb_in,
                                                    float* zb_out, const float* z_prev, char* smem, double* slot,
                                                    float asc, float& amx, const float4* pts, double* g0_slot) {
  constexpr int PB = wide_pb(H), NOB = H / 16;
  using S = SplitShape<NOB, NOB, PB>;
  using Pr = Prec<PREC>;
  using T = Tile<PREC>;
  constexpr int CPB = S::CPB, NIBW = S::NIBW, NOBC = S::NOBC, KC = S::KC;
  constexpr bool kLap = (ACT & kLapFlag) != 0;
  const LayerDev& ly = net.layer[j];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int nib = NOB, nob = NOB;
  const int rld = T::ld(H, PB);
  float lw1, lw2;
  lap_weights(net, lw1, lw2);
  char* STG = smem;
  char* R = smem + (size_t)PB * NOB * 256;
  const int zb_bytes = CPB * nob * 1024;
  auto zb_src = [&](int64_t s) { return reinterpret_cast<const char*>(zb_in) + s * zb_bytes; };
  f4 zp[NIBW][CPB];
  auto load_zp = [&](int64_t s) {
#pragma unroll
    for (int q = 0; q < NIBW; ++q)
#pragma unroll
      for (int cb = 0; cb < CPB; ++cb)
        zp[q][cb] = to_f4(*jet_frag(const_cast<float*>(z_prev), s * CPB + cb, wave + 8 * q, nib, lane));
  };
  if (n_sub <= 0) {
    if (g0_slot)
      for (int i = threadIdx.x; i < H * (net.d_in + 1); i += kThreads) g0_slot[i] = 0.0;
    return;
  }
  __syncthreads();  // the previous user of the LDS is done

  // ---- pass 1: input adjoint and activation adjoint
  {
    float g0s[NIBW][4];
#pragma unroll
    for (int q = 0; q < NIBW; ++q) g0s[q][0] = g0s[q][1] = g0s[q][2] = g0s[q][3] = 0.0f;
    float4 xp[CPB];
    async_copy(STG, zb_src(0), zb_bytes);
    Raw wreg[NIBW][KC];
#pragma unroll
    for (int q = 0; q < NIBW; ++q)
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) wreg[q][kc] = glob_frag(ly.wb, wave + 8 * q, kc, KC, lane);
    wait_vm<0>();
    for (int64_t s = 0; s < n_sub; ++s) {
      const int64_t cb0 = s * CPB;
      if (s == 0 || g0_slot)
        wait_vm<0>();
      else
        wait_vm<S::NSTORE>();  // the staged adjoint; the previous sub-tile's stores may run on
      barrier_lds();
#pragma unroll
      for (int q = 0; q < NOBC; ++q) {  // STG -> R (T layout)
        const int ob = wave + 8 * q;
        if (ob >= NOB) continue;
#pragma unroll
        for (int cb = 0; cb < CPB; ++cb) {
          const f4 zb = to_f4(*reinterpret_cast<const float4*>(STG + ((size_t)(cb * nob + ob) * 64 + lane) * 16));
          T::put(R, rld, 4 * cb + g, 16 * ob + l16, ascale<PREC>(zb, asc));
        }
      }
      load_zp(s);
      if (g0_slot)
#pragma unroll
        for (int cb = 0; cb < CPB; ++cb) xp[cb] = pts[(cb0 + cb) * 4 + g];
      barrier_lds();  // R complete; STG free
      f4 acca[NIBW][CPB];
      split_adjoint_product<PREC, NIBW, CPB, KC>(acca, STG, R, rld, wreg, s + 1 < n_sub ? zb_src(s + 1) : nullptr,
                                                 zb_bytes, lane);
#pragma unroll
      for (int q = 0; q < NIBW; ++q) {
        const int ib = wave + 8 * q;
#pragma unroll
        for (int cb = 0; cb < CPB; ++cb) {
          const f4 z = zp[q][cb];
          float s0v, s1v, s2v, s3v;
          act_eval<ACT>(z.x, net.w0, s0v, s1v, s2v, s3v);
          const f4 zb = jet_act_adj<kLap>(z, ascale<PREC>(acca[q][cb], 1.0f / asc), s1v, s2v, s3v, lw1, lw2);
          if (g0_slot) {
            // the identity input's jets are (x_k, e_k, 0)
            g0s[q][0] += zb.x * xp[cb].x + zb.y;
            g0s[q][1] += zb.x * xp[cb].y + zb.z;
            g0s[q][2] += zb.x * xp[cb].z + zb.w;
            g0s[q][3] += zb.x;
          } else {
            *jet_frag(zb_out, cb0 + cb, ib, nib, lane) = to_float4(zb);
          }
          if constexpr (PREC == kFP16X3) amx = fmaxf(amx, jet_absmax(zb));
        }
      }
    }
    if (g0_slot) {
      // every neuron block belongs to one wave: sums over its four lane groups only
      const int d = net.d_in;
#pragma unroll
      for (int q = 0; q < NIBW; ++q) {
        const int n = 16 * (wave + 8 * q) + l16;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float v = g0s[q][k];
          v += __shfl_xor(v, 16, 64);
          v += __shfl_xor(v, 32, 64);
          if (g == 0) {
            if (k < d) g0_slot[(size_t)n * d + k] = (double)v;
            if (k == 3) g0_slot[(size_t)H * d + n] = (double)v;
          }
        }
      }
    }
  }

  // ---- pass 2: weight and bias gradient
  f4 accw[NOB][NIBW];
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
    for (int q = 0; q < NIBW; ++q) accw[ob][q] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum[NOBC];
#pragma unroll
  for (int q = 0; q < NOBC; ++q) bsum[q] = 0.f;
  barrier_lds();  // every wave is past its last read of R and STG in pass 1
  async_copy(STG, zb_src(0), zb_bytes);
  load_zp(0);
  for (int64_t s = 0; s < n_sub; ++s) {
    wait_vm<0>();
    barrier_lds();  // sub-tile s staged and its pre-activations loaded; R free
#pragma unroll
    for (int q = 0; q < NOBC; ++q) {  // STG -> A operands of the weight gradient (ZT layout in R)
      const int ob = wave + 8 * q;
      if (ob >= NOB) continue;
#pragma unroll
      for (int cc = 0; cc < CPB / 2; ++cc) {
        const float4 v0 = *reinterpret_cast<const float4*>(STG + ((size_t)((2 * cc) * nob + ob) * 64 + lane) * 16);
        const float4 v1 = *reinterpret_cast<const float4*>(STG + ((size_t)((2 * cc + 1) * nob + ob) * 64 + lane) * 16);
        const float f[8] = {ascale<PREC>(v0.x, asc), ascale<PREC>(v0.y, asc), ascale<PREC>(v0.z, asc),
                            ascale<PREC>(v0.w, asc), ascale<PREC>(v1.x, asc), ascale<PREC>(v1.y, asc),
                            ascale<PREC>(v1.z, asc), ascale<PREC>(v1.w, asc)};
        const Raw op = Pr::make(f);
        uint4* d = reinterpret_cast<uint4*>(R + ((size_t)(ob * (CPB / 2) + cc) * 64 + lane) * 32);
        d[0] = op.a;
        d[1] = op.b;
        bsum[q] += v0.x + v1.x;
      }
    }
    barrier_lds();  // ZT complete; STG free
    Raw aop[NIBW][CPB / 2];
#pragma unroll
    for (int q = 0; q < NIBW; ++q)
#pragma unroll
      for (int cc = 0; cc < CPB / 2; ++cc) {
        float f[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const f4 z = zp[q][2 * cc + h];
          float s0v, s1v, s2v, s3v;
          act_eval<ACT>(z.x, net.w0, s0v, s1v, s2v, s3v);
          const f4 a = jet_act<kLap>(z, s0v, s1v, s2v, lw1, lw2);
          f[4 * h] = a.x;
          f[4 * h + 1] = a.y;
          f[4 * h + 2] = a.z;
          f[4 * h + 3] = a.w;
        }
        aop[q][cc] = Pr::make(f);
      }
    if (s + 1 < n_sub) load_zp(s + 1);  // the next sub-tile's pre-activations load under the product
    split_weight_grad_product<PREC, NOB, NIBW, CPB>(accw, aop, STG, R, s + 1 < n_sub ? zb_src(s + 1) : nullptr,
                                                    zb_bytes, lane);
  }
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
    for (int q = 0; q < NIBW; ++q) {
      const int ib = wave + 8 * q;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        slot[(size_t)(16 * ob + 4 * g + r) * H + 16 * ib + l16] = (double)accw[ob][q][r] * (double)(1.0f / asc);
    }
#pragma unroll
  for (int q = 0; q < NOBC; ++q) {
    const int ob = wave + 8 * q;
    float v = bsum[q];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (g == 0 && ob < NOB) slot[(size_t)H * H + 16 * ob + l16] = (double)v;
  }
  __syncthreads();
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
    // (bf16x3 only, where it was measured faster: width 128 keeps the one-pass loop, whose
    // weights are a quarter of the size, and the second read of the jets cost more than
    // streaming them; fp16x3 ran no faster with it at width 256 and its width-128 items
    // ran slower with it compiled into the same kernel)
    if constexpr (PREC == kBF16X3 && H == 256) {
      if (net.layer[j].n_in == H && net.layer[j].n_out == H) {
        float asc = 1.0f;
        if constexpr (PREC == kFP16X3) asc = adj_scale<PREC>(__float_as_uint(wg_max(amx, red)));
        amx = 0.0f;
        item_layer_two_pass<PREC, ACT, H>(net, j, npts / wide_pb(H), zb[cur], zb[cur ^ 1],
                                          zs + (j - 1) * in.zs_stride, smem, gslot + in.eff_off[j], asc, amx, pts,
                                          j == 1 ? gslot + in.eff_off[0] : nullptr);
        cur ^= 1;
        continue;
      }
    }
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
                                             zs + (j - 1) * in.zs_stride, smem, accw, bsum, asc, amx,
                                             j == 1 ? gslot + in.eff_off[0] : nullptr);
    bwd_flush<H / 16, H / 16, PB>(accw, bsum, gslot + in.eff_off[j], net.layer[j].n_out, net.layer[j].n_in,
                                  1.0f / asc);
    cur ^= 1;
  }
  // first layer (identity embedding): summed by layer 1's backward when there is one
  if (net.L == 1)
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
  const size_t b2 = H == 256 ? (size_t)2 * wide_pb(H) * (H / 16) * 256 : 0;  // two-pass layer backward
  if (b2 > b) b = b2;
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
