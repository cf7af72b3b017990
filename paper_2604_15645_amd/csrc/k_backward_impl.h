// k_backward_impl.h -- one linear layer's backward: the generic, wide and split-role kernels
// and their launcher.
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma once
#include "pinn_device.h"

namespace pinn {

template <int PREC, int ACT, int NOB, int NIB, int PB>
__global__ __launch_bounds__(kThreads, 1) void k_backward(const BwdArgs A) {
  using S = BwdShape<NOB, NIB, PB>;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  f4 accw[S::NOBW][S::NIBW];
#pragma unroll
  for (int i = 0; i < S::NOBW; ++i)
#pragma unroll
    for (int k = 0; k < S::NIBW; ++k) accw[i][k] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum[S::NOBW];
#pragma unroll
  for (int i = 0; i < S::NOBW; ++i) bsum[i] = 0.f;
  const int64_t count = A.n_sub > blockIdx.x ? (A.n_sub - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
  const float asc = adj_scale<PREC>(A.work.amax[A.layer]);
  float amx = 0.0f;
  // layer 1 over an identity embedding: the first layer's sums from the input adjoint
  double* g0 = A.g0_slots ? A.g0_slots + (size_t)blockIdx.x * A.net.layer[0].n_out * (A.net.d_in + 1) : nullptr;
  bwd_range<PREC, ACT, NOB, NIB, PB>(A.net, A.layer, A.work.pts, blockIdx.x, gridDim.x, count, A.zb_in, A.zb_out,
                                     A.z_prev, smem, accw, bsum, asc, amx, g0);
  if constexpr (PREC == kFP16X3)
    if (A.z_prev) amax_publish(amx, &A.work.amax[A.layer - 1]);
  const LayerDev& ly = A.net.layer[A.layer];
  bwd_flush<NOB, NIB, PB>(accw, bsum, A.slots + (size_t)blockIdx.x * ly.n_out * (ly.n_in + 1), ly.n_out, ly.n_in,
                          1.0f / asc);
}

// ================================================================== backward (one layer, wide)

// Layer backward for bf16x3 when the layer input width is a multiple of 128 (8 waves x
// 16-column blocks).  Wave w owns input blocks ib = w + 8 k: it computes the input adjoint
// (and, for a hidden layer, the activation adjoint) for those columns over the whole
// sub-tile, and the weight-gradient columns of those blocks for every output row.  The
// weight-gradient product then takes its B operand (activation jets of the layer input,
// in accumulator order) straight from the wave's registers and its A operand (output
// adjoint, 8 cp per lane) from the R tile by plain 8-byte reads, so no second LDS tile is
// needed and sub-tiles can be twice as large as in bwd_range.
// LDS: STG and R (T layout), both PB x (16 NOB) x 16 bytes.  STG holds, in turn, the staged
// output-adjoint fragments of the sub-tile (copied in during the previous sub-tile's weight
// gradient) and the staged layer-input pre-activations (copied in during the input-adjoint
// product).
template <int NOB, int NIB, int PB>
struct WideShape {
  static constexpr int CPB = PB / 4;
  static constexpr int NIBW = NIB / 8;             // input blocks per wave (upper bound)
  static constexpr int NOBC = (NOB + 7) / 8;       // output blocks converted per wave
  static_assert(NIB % 8 == 0 && CPB % 2 == 0, "wide backward shape");
};

__host__ __device__ constexpr size_t wide_lds_bytes(int PB, int n_out) { return (size_t)2 * PB * n_out * 16; }

// A operand of the weight gradient for output block ob and cp chunk cc (points 8 cc ..
// 8 cc + 7): lane (g, l16) takes output o = 16 ob + l16 and the 4 channels of points
// 8 cc + g and 8 cc + 4 + g -- the cp order of the accumulator fragments.
__device__ __forceinline__ Raw wide_zbar_op(const char* R, int ld, int ob, int cc, int lane) {
  const int g = lane >> 4, o = 16 * ob + (lane & 15);
  const int p0 = 8 * cc + g, p1 = p0 + 4;
  const char* c0 = R + (size_t)((o >> 5) * ld + (p0 >> 2)) * 2048 + t_cell_off(p0, o);
  const char* c1 = R + (size_t)((o >> 5) * ld + (p1 >> 2)) * 2048 + t_cell_off(p1, o);
  const uint2 h0 = *reinterpret_cast<const uint2*>(c0), h1 = *reinterpret_cast<const uint2*>(c1);
  const uint2 l0 = *reinterpret_cast<const uint2*>(c0 + 1024), l1 = *reinterpret_cast<const uint2*>(c1 + 1024);
  Raw r;
  r.a = make_uint4(h0.x, h0.y, h1.x, h1.y);
  r.b = make_uint4(l0.x, l0.y, l1.x, l1.y);
  return r;
}

template <int PREC, int ACT, int NOB, int NIB, int PB>
__device__ __forceinline__ void bwd_wide_range(const NetDev& net, int layer, const float4* pts, int64_t s0,
                                               int64_t stride, int64_t count, const float* zb_in, float* zb_out,
                                               const float* z_prev, char* smem,
                                               f4 (&accw)[NOB][WideShape<NOB, NIB, PB>::NIBW],
                                               float (&bsum)[WideShape<NOB, NIB, PB>::NOBC], float asc, float& amx) {
  using S = WideShape<NOB, NIB, PB>;
  using Pr = Prec<PREC>;
  using T = Tile<PREC>;
  constexpr int CPB = S::CPB, NIBW = S::NIBW, NOBC = S::NOBC;
  constexpr bool kLap = (ACT & kLapFlag) != 0;
  const LayerDev& ly = net.layer[layer];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int n_in = ly.n_in, n_out = ly.n_out;
  const int nob = n_out / 16, nib = n_in / 16;
  const bool has_prev = z_prev != nullptr;
  const int rld = T::ld(n_out, PB);
  float lw1, lw2;
  lap_weights(net, lw1, lw2);
  char* STG = smem;
  char* R = smem + (size_t)PB * NOB * 256;  // STG sized for the widest layer of the kernel
  const int zb_bytes = CPB * nob * 1024, zp_bytes = CPB * nib * 1024;
  auto zb_src = [&](int64_t s) { return reinterpret_cast<const char*>(zb_in) + s * zb_bytes; };

  if (count <= 0) return;
  __syncthreads();  // the previous user of the LDS is done
  async_copy(STG, zb_src(s0), zb_bytes);

  for (int64_t k = 0; k < count; ++k) {
    const int64_t s = s0 + k * stride;
    const int64_t cb0 = s * CPB;
    wait_async();
    barrier_lds();  // sub-tile s staged; the previous sub-tile is done with R
    // (1) output adjoint into R (T layout); bias sums of the converted output blocks
#pragma unroll
    for (int q = 0; q < NOBC; ++q) {
      const int ob = wave + 8 * q;
      if (ob < nob) {
#pragma unroll
        for (int cb = 0; cb < CPB; ++cb) {
          const f4 zb = to_f4(*reinterpret_cast<const float4*>(STG + ((size_t)(cb * nob + ob) * 64 + lane) * 16));
          T::put(R, rld, 4 * cb + g, 16 * ob + l16, ascale<PREC>(zb, asc));
          bsum[q] += zb.x;
        }
      }
    }
    barrier_lds();  // R complete; STG free
    // (2)-(3) per owned input block: layer-input jets a (B operand of the weight gradient)
    // and, for a hidden layer, the input adjoint and the activation adjoint
    Raw aop[NIBW][CPB / 2];
    if (has_prev) {
      async_copy(STG, reinterpret_cast<const char*>(z_prev) + s * zp_bytes, zp_bytes);
      f4 acca[NIBW][CPB];
#pragma unroll
      for (int q = 0; q < NIBW; ++q)
#pragma unroll
        for (int cb = 0; cb < CPB; ++cb) acca[q][cb] = f4{0.f, 0.f, 0.f, 0.f};
      {
        int blk[NIBW];
#pragma unroll
        for (int q = 0; q < NIBW; ++q) blk[q] = wave + 8 * q;
        gemm_tile<PREC, NIBW, CPB>(acca, R, rld, 0, ly.wb, ly.kco, blk, lane);
      }
      wait_async();
      barrier_lds();  // pre-activations of sub-tile s staged
#pragma unroll
      for (int q = 0; q < NIBW; ++q) {
        const int ib = wave + 8 * q;
#pragma unroll
        for (int cc = 0; cc < CPB / 2; ++cc) {
          float f[8];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int cb = 2 * cc + h;
            const f4 z = to_f4(*reinterpret_cast<const float4*>(STG + ((size_t)(cb * nib + ib) * 64 + lane) * 16));
            float s0v, s1v, s2v, s3v;
            act_eval<ACT>(z.x, net.w0, s0v, s1v, s2v, s3v);
            const f4 a = jet_act<kLap>(z, s0v, s1v, s2v, lw1, lw2);
            f[4 * h] = a.x;
            f[4 * h + 1] = a.y;
            f[4 * h + 2] = a.z;
            f[4 * h + 3] = a.w;
            const f4 zb = jet_act_adj<kLap>(z, ascale<PREC>(acca[q][cb], 1.0f / asc), s1v, s2v, s3v, lw1, lw2);
            *jet_frag(zb_out, cb0 + cb, ib, nib, lane) = to_float4(zb);
            if constexpr (PREC == kFP16X3) amx = fmaxf(amx, jet_absmax(zb));
          }
          aop[q][cc] = Pr::make(f);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else {
      // Fourier-feature jets of the owned columns: column i < m is cos(x B_i), i >= m sin
      const int m = net.n_freq;
      const float4* sp = pts + s * PB;
#pragma unroll
      for (int q = 0; q < NIBW; ++q) {
        const int i = 16 * min(wave + 8 * q, nib - 1) + l16;
        const int j = i < m ? i : i - m;
#pragma unroll
        for (int cc = 0; cc < CPB / 2; ++cc) {
          float f[8];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            f4 cj, sj;
            rff_jets(net, net.B, sp[4 * (2 * cc + h) + g], j, cj, sj);
            const f4 a = i < m ? cj : sj;
            f[4 * h] = a.x;
            f[4 * h + 1] = a.y;
            f[4 * h + 2] = a.z;
            f[4 * h + 3] = a.w;
          }
          aop[q][cc] = Pr::make(f);
        }
      }
    }
    barrier_lds();  // STG no longer read
    if (k + 1 < count) async_copy(STG, zb_src(s + stride), zb_bytes);
    // (4) weight gradient: W_bar[o][i] += sum_cp zbar[cp][o] a[cp][i] for the owned columns
#pragma unroll
    for (int cc = 0; cc < CPB / 2; ++cc)
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob) {
        const Raw ao = wide_zbar_op(R, rld, min(ob, nob - 1), cc, lane);
#pragma unroll
        for (int q = 0; q < NIBW; ++q) Pr::mma(accw[ob][q], ao, aop[q][cc]);
      }
  }
}

// Weight-gradient sums of the wide backward into a slot [n_out][n_in] then [n_out].
template <int NOB, int NIB, int PB>
__device__ __forceinline__ void bwd_wide_flush(const f4 (&accw)[NOB][WideShape<NOB, NIB, PB>::NIBW],
                                               const float (&bsum)[WideShape<NOB, NIB, PB>::NOBC], double* slot,
                                               int n_out, int n_in, float inv) {
  using S = WideShape<NOB, NIB, PB>;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int nob = n_out / 16, nib = n_in / 16;
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob) {
    if (ob >= nob) continue;
#pragma unroll
    for (int q = 0; q < S::NIBW; ++q) {
      const int ib = wave + 8 * q;
      if (ib >= nib) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        slot[(size_t)(16 * ob + 4 * g + r) * n_in + 16 * ib + l16] = (double)accw[ob][q][r] * (double)inv;
    }
  }
#pragma unroll
  for (int q = 0; q < S::NOBC; ++q) {
    const int ob = wave + 8 * q;
    float v = bsum[q];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (ob < nob && g == 0) slot[(size_t)n_out * n_in + 16 * ob + l16] = (double)v;
  }
}

template <int PREC, int ACT, int NOB, int NIB, int PB>
__global__ __launch_bounds__(kThreads, 1) void k_backward_wide(const BwdArgs A) {
  using S = WideShape<NOB, NIB, PB>;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  f4 accw[NOB][S::NIBW];
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
    for (int q = 0; q < S::NIBW; ++q) accw[ob][q] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum[S::NOBC];
#pragma unroll
  for (int q = 0; q < S::NOBC; ++q) bsum[q] = 0.f;
  const int64_t count = A.n_sub > blockIdx.x ? (A.n_sub - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
  const float asc = adj_scale<PREC>(A.work.amax[A.layer]);
  float amx = 0.0f;
  bwd_wide_range<PREC, ACT, NOB, NIB, PB>(A.net, A.layer, A.work.pts, blockIdx.x, gridDim.x, count, A.zb_in,
                                          A.zb_out, A.z_prev, smem, accw, bsum, asc, amx);
  if constexpr (PREC == kFP16X3)
    if (A.z_prev) amax_publish(amx, &A.work.amax[A.layer - 1]);
  const LayerDev& ly = A.net.layer[A.layer];
  bwd_wide_flush<NOB, NIB, PB>(accw, bsum, A.slots + (size_t)blockIdx.x * ly.n_out * (ly.n_in + 1), ly.n_out, ly.n_in,
                               1.0f / asc);
}

// ================================================================== backward (one layer, split roles)

// Hidden-layer backward for bf16x3 at input widths that are multiples of 128, with the
// work-groups split into two roles that sweep the same sub-tiles:
//   role 0  input adjoint and activation adjoint (abar = zbar W, then zbar_prev), with the
//           layer's weight fragments held in registers for the whole launch (no weight
//           traffic per sub-tile);
//   role 1  weight gradient W_bar += zbar^T a_prev and bias gradient, the sums held in
//           registers over the work-group's sub-tiles.
// Each role keeps half the matrix-core work of a sub-tile.  Work-groups b and b + 8 (one
// of each role) take the same sub-tiles; dispatch places them on the same XCD, so the
// second reader of a sub-tile's jets finds them in cache.  Both roles stage the output
// adjoint of the next sub-tile into LDS (STG) and load the pre-activations of the current
// one into registers before they are needed; vector-memory counters complete in issue
// order, and the loop waits only for what it needs (role 0 leaves its adjoint stores
// outstanding across the wait).
constexpr int kPaceSpin = 512;  // polls of a pacing wait before it goes on regardless

template <int PREC, int ACT, int NOB, int NIB, int PB, bool EMB, bool FUSE0 = false>
__global__ __launch_bounds__(kThreads, 1) void k_backward_split(const BwdArgs A) {
  using S = SplitShape<NOB, NIB, PB>;
  using Pr = Prec<PREC>;
  using T = Tile<PREC>;
  constexpr int CPB = S::CPB, NIBW = S::NIBW, NOBC = S::NOBC, KC = S::KC;
  constexpr bool kLap = (ACT & kLapFlag) != 0;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const NetDev& net = A.net;
  const LayerDev& ly = net.layer[A.layer];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int n_in = ly.n_in, n_out = ly.n_out;
  const int nib = n_in / 16, nob = n_out / 16;
  const int rld = T::ld(n_out, PB);
  float lw1, lw2;
  lap_weights(net, lw1, lw2);
  char* STG = smem;
  char* R = smem + (size_t)PB * NOB * 256;
  float* BF = reinterpret_cast<float*>(R + (size_t)PB * NOB * 256);  // Fourier matrix (EMB)
  if (EMB)
    for (int i = threadIdx.x; i < net.d_in * net.n_freq; i += kThreads) BF[i] = net.B[i];
  const int zb_bytes = CPB * nob * 1024;
  const float asc = adj_scale<PREC>(A.work.amax[A.layer]);
  // role and index within the role (blocks b and b + 8 share a sub-tile sequence)
  // (EMB: the Fourier-embedding layer -- weight gradient only, every work-group)
  const int b = blockIdx.x;
  const int role = EMB ? 1 : (b >> 3) & 1;
  const int rb = EMB ? b : ((b >> 4) << 3) | (b & 7);
  const int G = EMB ? gridDim.x : gridDim.x >> 1;
  const int64_t count = A.n_sub > rb ? (A.n_sub - rb + G - 1) / G : 0;
  auto zb_src = [&](int64_t s) { return reinterpret_cast<const char*>(A.zb_in) + s * zb_bytes; };
  f4 zp[NIBW][CPB];
  auto load_zp = [&](int64_t s) {
#pragma unroll
    for (int q = 0; q < NIBW; ++q)
#pragma unroll
      for (int cb = 0; cb < CPB; ++cb)
        zp[q][cb] = to_f4(*jet_frag(const_cast<float*>(A.z_prev), s * CPB + cb, wave + 8 * q, nib, lane));
  };
  auto convert = [&](float* bsum) {  // STG -> R (T layout), bias sums of the converted blocks
#pragma unroll
    for (int q = 0; q < NOBC; ++q) {
      const int ob = wave + 8 * q;
      if (ob >= NOB) continue;
#pragma unroll
      for (int cb = 0; cb < CPB; ++cb) {
        const f4 zb = to_f4(*reinterpret_cast<const float4*>(STG + ((size_t)(cb * nob + ob) * 64 + lane) * 16));
        T::put(R, rld, 4 * cb + g, 16 * ob + l16, ascale<PREC>(zb, asc));
        if (bsum) bsum[q] += zb.x;
      }
    }
  };
  if (count > 0) async_copy(STG, zb_src(rb), zb_bytes);

  if (!EMB && role == 0) {
    // ---- input adjoint and activation adjoint
    Raw wreg[NIBW][KC];  // B operand fragments of the owned input blocks, all chunks
#pragma unroll
    for (int q = 0; q < NIBW; ++q)
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) wreg[q][kc] = glob_frag(ly.wb, wave + 8 * q, kc, KC, lane);
    wait_vm<0>();  // resident from here on: no wait for them inside the loop
    bool held = false;  // the partner had not reached the previous sub-tile when last read
    float amx = 0.0f;
    // FUSE0: the first layer's sums per owned input block: W_bar[n][k] (k < d_in), b_bar[n]
    float g0s[FUSE0 ? NIBW : 1][4];
    if constexpr (FUSE0) {
#pragma unroll
      for (int q = 0; q < NIBW; ++q) g0s[q][0] = g0s[q][1] = g0s[q][2] = g0s[q][3] = 0.0f;
    }
    for (int64_t k = 0; k < count; ++k) {
      const int64_t s = rb + k * G;
      const int64_t cb0 = s * CPB;
      if (k == 0 || FUSE0)
        wait_vm<0>();  // (FUSE0 stores nothing: the last operations issued are the copy's)
      else
        wait_vm<S::NSTORE>();  // the staged adjoint; the previous sub-tile's stores may run on
      if (held && threadIdx.x == 0) {
        // pacing: this role reads each sub-tile first and its partner must find the jets
        // still in L2, so it runs at most one sub-tile ahead of the partner (a bounded wait:
        // it goes on regardless after kPaceSpin polls)
        const unsigned long long want = (A.launch << 20) + (unsigned long long)(k - 1);
        for (int it = 0; it < kPaceSpin; ++it) {
          if (__hip_atomic_load(&A.pace[rb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want) break;
          __builtin_amdgcn_s_sleep(2);
        }
      }
      barrier_lds();
      convert(nullptr);
      load_zp(s);  // after the staged reads: waiting for these must not wait for the next copy
      float4 xp[FUSE0 ? CPB : 1];  // FUSE0: the sub-tile's points, loaded under the product
      if constexpr (FUSE0) {
#pragma unroll
        for (int cb = 0; cb < CPB; ++cb) xp[cb] = A.work.pts[(cb0 + cb) * 4 + g];
      }
      unsigned long long seen = ~0ull;
      if (A.pace) seen = __hip_atomic_load(&A.pace[rb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      barrier_lds();  // R complete; STG free
      f4 acca[NIBW][CPB];
      split_adjoint_product<PREC, NIBW, CPB, KC>(acca, STG, R, rld, wreg, k + 1 < count ? zb_src(s + G) : nullptr,
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
          if constexpr (FUSE0) {
            // identity embedding: the jets of input k are (x_k, e_k, 0), so the point
            // contributes zbar.value x_k + zbar.d_k to W_bar[n][k] and zbar.value to b_bar[n]
            const float4 x = xp[cb];
            g0s[q][0] += zb.x * x.x + zb.y;
            g0s[q][1] += zb.x * x.y + zb.z;
            g0s[q][2] += zb.x * x.z + zb.w;  // (input 2 only when d_in = 3; dropped otherwise)
            g0s[q][3] += zb.x;
          } else {
            // streamed past the caches: the next launch reads it, long after this one
            __builtin_nontemporal_store(zb, reinterpret_cast<f4*>(jet_frag(A.zb_out, cb0 + cb, ib, nib, lane)));
          }
          if constexpr (PREC == kFP16X3) amx = fmaxf(amx, jet_absmax(zb));
        }
      }
      // read beside the pre-activations, compared once they are in use
      held = A.pace && seen < (A.launch << 20) + (unsigned long long)k;
    }
    if constexpr (PREC == kFP16X3) amax_publish(amx, &A.work.amax[A.layer - 1]);
    if constexpr (FUSE0) {
      // slot rb: [n_in][d_in] weight sums, then [n_in] bias sums (the first layer's layout)
      const int d = A.net.d_in;
      double* slot = A.g0_slots + (size_t)rb * n_in * (d + 1);
#pragma unroll
      for (int q = 0; q < NIBW; ++q) {
        const int n = 16 * (wave + 8 * q) + l16;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float v = g0s[q][k];
          v += __shfl_xor(v, 16, 64);
          v += __shfl_xor(v, 32, 64);
          g0s[q][k] = v;
        }
        if (g == 0) {
          for (int k = 0; k < d; ++k) slot[(size_t)n * d + k] = (double)g0s[q][k];
          slot[(size_t)n_in * d + n] = (double)g0s[q][3];
        }
      }
    }
  } else {
    // ---- weight and bias gradient
    f4 accw[NOB][NIBW];
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
      for (int q = 0; q < NIBW; ++q) accw[ob][q] = f4{0.f, 0.f, 0.f, 0.f};
    float bsum[NOBC];
#pragma unroll
    for (int q = 0; q < NOBC; ++q) bsum[q] = 0.f;
    if (!EMB && count > 0) load_zp(rb);
    for (int64_t k = 0; k < count; ++k) {
      const int64_t s = rb + k * G;
      wait_vm<0>();
      // progress for the partner's pacing: sub-tile s read, the next one about to be
      if (!EMB && A.pace && threadIdx.x == 0)
        __hip_atomic_store(&A.pace[rb], (A.launch << 20) + (unsigned long long)k, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      barrier_lds();  // sub-tile s staged and its pre-activations loaded; ZT free
      // output adjoint as weight-gradient A operands in the ZT layout: for output block ob
      // and cp chunk cc, lane (g, l16) holds 8 cp of output 16 ob + l16 (points 8 cc + g,
      // 8 cc + 4 + g, accumulator order), bf16 hi then lo, 32 bytes per lane
#pragma unroll
      for (int q = 0; q < NOBC; ++q) {
        const int ob = wave + 8 * q;
        if (ob >= NOB) continue;
#pragma unroll
        for (int cc = 0; cc < CPB / 2; ++cc) {
          const float* f0 = reinterpret_cast<const float*>(STG + ((size_t)((2 * cc) * nob + ob) * 64 + lane) * 16);
          const float* f1 = reinterpret_cast<const float*>(STG + ((size_t)((2 * cc + 1) * nob + ob) * 64 + lane) * 16);
          const float4 v0 = *reinterpret_cast<const float4*>(f0), v1 = *reinterpret_cast<const float4*>(f1);
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
      if constexpr (EMB && NIB == 16) {
        // 128 frequencies: the lane's two input blocks (wave, wave + 8) are the cosine and the
        // sine column of one frequency, whose jets come from one evaluation
        const int j = 16 * wave + l16;
#pragma unroll
        for (int cc = 0; cc < CPB / 2; ++cc) {
          float fc[8], fs[8];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            f4 cj, sj;
            rff_jets(net, BF, A.work.pts[(int64_t)s * PB + 4 * (2 * cc + h) + g], j, cj, sj);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              fc[4 * h + e] = cj[e];
              fs[4 * h + e] = sj[e];
            }
          }
          aop[0][cc] = Pr::make(fc);
          aop[1][cc] = Pr::make(fs);
        }
      } else {
#pragma unroll
        for (int q = 0; q < NIBW; ++q)
#pragma unroll
          for (int cc = 0; cc < CPB / 2; ++cc) {
            float f[8];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              f4 a;
              if constexpr (EMB) {
                // Fourier-feature jets: column i < m is cos(x B_i), column i >= m sin(x B_{i-m})
                const int m = net.n_freq;
                const int i = 16 * (wave + 8 * q) + l16;
                f4 cj, sj;
                rff_jets(net, BF, A.work.pts[(int64_t)s * PB + 4 * (2 * cc + h) + g], i < m ? i : i - m, cj, sj);
                a = i < m ? cj : sj;
              } else {
                const f4 z = zp[q][2 * cc + h];
                float s0v, s1v, s2v, s3v;
                act_eval<ACT>(z.x, net.w0, s0v, s1v, s2v, s3v);
                a = jet_act<kLap>(z, s0v, s1v, s2v, lw1, lw2);
              }
              f[4 * h] = a.x;
              f[4 * h + 1] = a.y;
              f[4 * h + 2] = a.z;
              f[4 * h + 3] = a.w;
            }
            aop[q][cc] = Pr::make(f);
          }
      }
      if (!EMB && k + 1 < count) load_zp(s + G);  // the next sub-tile's pre-activations load under the product
      split_weight_grad_product<PREC, NOB, NIBW, CPB>(accw, aop, STG, R, k + 1 < count ? zb_src(s + G) : nullptr,
                                                zb_bytes, lane);
    }
    // flush: slot rb, [n_out][n_in] then [n_out]
    double* slot = A.slots + (size_t)rb * n_out * (n_in + 1);
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
      for (int q = 0; q < NIBW; ++q) {
        const int ib = wave + 8 * q;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          slot[(size_t)(16 * ob + 4 * g + r) * n_in + 16 * ib + l16] = (double)accw[ob][q][r] * (double)(1.0f / asc);
      }
#pragma unroll
    for (int q = 0; q < NOBC; ++q) {
      const int ob = wave + 8 * q;
      float v = bsum[q];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (g == 0 && ob < NOB) slot[(size_t)n_out * n_in + 16 * ob + l16] = (double)v;
    }
  }
}


// ================================================================== launcher
// (instantiated per precision in k_backward_<precision>.hip, so that the three compile in
// parallel)

namespace {

template <int PREC, int ACT, int NOB, int NIB, int PB>
int bwd(const BwdArgs& a, int grid, size_t lds, hipStream_t s) {
  auto k = k_backward<PREC, ACT, NOB, NIB, PB>;
  if (set_lds(k, lds)) return -5;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, s, a);
  return launch_status(hipGetLastError());
}

template <int PREC, int ACT, int NOB, int NIB, int PB>
int bwd_wide(const BwdArgs& a, int grid, size_t lds, hipStream_t s) {
  auto k = k_backward_wide<PREC, ACT, NOB, NIB, PB>;
  if (set_lds(k, lds)) return -5;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, s, a);
  return launch_status(hipGetLastError());
}

template <int PREC, int ACT, int NOB, int NIB, int PB, bool EMB, bool FUSE0 = false>
int split_k(const BwdArgs& a, int grid, size_t lds, hipStream_t s) {
  auto k = k_backward_split<PREC, ACT, NOB, NIB, PB, EMB, FUSE0>;
  if (set_lds(k, lds)) return -5;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, s, a);
  return launch_status(hipGetLastError());
}

template <int PREC, int ACT, int H>
int bwd_split(const BwdArgs& a, int grid, size_t lds, hipStream_t s) {
  if constexpr (H >= 128) {
    if (a.g0_slots) {
      if (a.pb == wide_pb(H)) return split_k<PREC, ACT, H / 16, H / 16, wide_pb(H), false, true>(a, grid, lds, s);
      if (a.pb == wide_pb(H) / 2)
        return split_k<PREC, ACT, H / 16, H / 16, wide_pb(H) / 2, false, true>(a, grid, lds, s);
      return -2;
    }
    if (a.pb == wide_pb(H)) return split_k<PREC, ACT, H / 16, H / 16, wide_pb(H), false>(a, grid, lds, s);
    if (a.pb == wide_pb(H) / 2) return split_k<PREC, ACT, H / 16, H / 16, wide_pb(H) / 2, false>(a, grid, lds, s);
  }
  return -2;
}

// Fourier-embedding layer (weight gradient only): embedding width 128 or 256.
template <int PREC, int ACT, int H>
int bwd_split_embed(const BwdArgs& a, int grid, size_t lds, hipStream_t s) {
  const int n_in = a.net.layer[0].n_in, n_out = a.net.layer[0].n_out;
  if (n_out != H || n_in % 128 != 0) return -2;
  if constexpr (H >= 64) {
    if (n_in == 128) return split_k<PREC, ACT, H / 16, 8, wide_pb(H), true>(a, grid, lds, s);
    if (n_in == 256) return split_k<PREC, ACT, H / 16, 16, wide_pb(H), true>(a, grid, lds, s);
  }
  return -2;
}

template <int PREC, int ACT, int H>
int bwd_e(bool embed, const BwdArgs& a, int grid, size_t lds, hipStream_t s) {
  if constexpr (is_split(PREC)) {
    if (a.wide == 2 && !embed) {
      // split-role kernel: layer widths must be exactly H (uniform hidden layers)
      if (a.net.layer[a.layer].n_in != H || a.net.layer[a.layer].n_out != H || grid % 16 != 0) return -2;
      return bwd_split<PREC, ACT, H>(a, grid, lds, s);
    }
    if (a.wide == 3 && embed) return bwd_split_embed<PREC, ACT, H>(a, grid, lds, s);
  }
  if constexpr (is_split(PREC)) {
    // wide path (chosen by the plan): input widths that are multiples of 128
    constexpr int PW = wide_pb(H);
    if (a.wide) {
      if (a.net.layer[a.layer].n_in % 128 != 0) return -2;
      if (embed) return bwd_wide<PREC, ACT, H / 16, 16, PW>(a, grid, lds, s);
      if constexpr (H >= 128) return bwd_wide<PREC, ACT, H / 16, H / 16, PW>(a, grid, lds, s);
      return -2;
    }
  }
  constexpr int PB = 2048 / H;
  if (embed) return bwd<PREC, ACT, H / 16, 16, H == 256 ? 8 : 16>(a, grid, lds, s);
  return bwd<PREC, ACT, H / 16, H / 16, PB>(a, grid, lds, s);
}

template <int PREC, int ACT>
int bwd_h(int H, bool embed, const BwdArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (H) {
    case 32: return bwd_e<PREC, ACT, 32>(embed, a, grid, lds, s);
    case 64: return bwd_e<PREC, ACT, 64>(embed, a, grid, lds, s);
    case 128: return bwd_e<PREC, ACT, 128>(embed, a, grid, lds, s);
    case 256: return bwd_e<PREC, ACT, 256>(embed, a, grid, lds, s);
    default: return -2;
  }
}

}  // namespace

template <int PREC>
int bwd_a(int act, int H, bool embed, const BwdArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (act) {
    case kTanh: return bwd_h<PREC, kTanh>(H, embed, a, grid, lds, s);
    case kSin: return bwd_h<PREC, kSin>(H, embed, a, grid, lds, s);
    case kTanh | kLapFlag: return bwd_h<PREC, kTanh | kLapFlag>(H, embed, a, grid, lds, s);
    case kSin | kLapFlag: return bwd_h<PREC, kSin | kLapFlag>(H, embed, a, grid, lds, s);
    default: return -2;
  }
}

// Each precision is instantiated in its own translation unit.
extern template int bwd_a<kFP32>(int act, int H, bool embed, const BwdArgs& a, int grid, size_t lds, hipStream_t s);
extern template int bwd_a<kBF16X3>(int act, int H, bool embed, const BwdArgs& a, int grid, size_t lds, hipStream_t s);
extern template int bwd_a<kFP16X3>(int act, int H, bool embed, const BwdArgs& a, int grid, size_t lds, hipStream_t s);

}  // namespace pinn
