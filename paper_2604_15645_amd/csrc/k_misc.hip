// k_misc.hip -- parameter staging, point gather, identity-embedding first-layer
// gradient, fixed-order FP64 reductions, the non-finite check, and their launchers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pinn_device.h"

namespace pinn {

// ================================================================== staging

// Effective weights and operand fragments of every layer.  One thread per (fragment,
// lane) of either kind, plus the plain FP32 copies.

__device__ __forceinline__ float eff_w(const StageArgs& a, int l, int o, int i) {
  if (o >= a.n_out[l] || i >= a.n_in[l]) return 0.0f;
  float v = a.params[a.off_w[l] + (int64_t)o * a.n_in[l] + i];
  if (a.rwf) v *= expf(a.params[a.off_s[l] + o]);
  return v;
}

template <int PREC>
__device__ __forceinline__ void stage_thread(const StageArgs& a, int64_t t) {
  if (t < 3 && a.omega) {  // omega_k = 2 pi / P_k of the periodic inputs (Sec. 2.6.3)
    const int k = (int)t;
    float w = 0.0f;
    if ((a.periodic_mask >> k) & 1) {
      float P = a.period[k];
      if ((a.period_train_mask >> k) & 1) {
        int r = 0;
        for (int j = 0; j < k; ++j) r += (a.period_train_mask >> j) & 1;
        P = a.params[a.off_p + r];
      }
      w = 6.2831853071795865f / P;
    }
    a.omega[k] = w;
  }
  if (t >= a.cum[a.n_layers]) return;
  int l = 0;
  while (t >= a.cum[l + 1]) ++l;
  t -= a.cum[l];
  const int ni = a.n_in[l], no = a.n_out[l];
  const int nbo = (no + 15) / 16, kci = (ni + 31) / 32;
  const int nbi = (ni + 15) / 16, kco = (no + 31) / 32;
  const int64_t nf = (int64_t)nbo * kci * 64, nb = (int64_t)nbi * kco * 64;
  const int64_t nplain = (int64_t)no * ni;
  if (t < nf) {  // forward fragment lane: neuron 16 blk + lane % 16, inputs 32 ch + 8 (lane/16) + j
    int lane = (int)(t % 64);
    int64_t f = t / 64;
    int ch = (int)(f % kci), blk = (int)(f / kci);
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = eff_w(a, l, 16 * blk + lane % 16, 32 * ch + 8 * (lane / 16) + j);
    Raw r = Prec<PREC>::make(v);
    uint4* p = reinterpret_cast<uint4*>(a.wf[l] + t * 32);
    p[0] = r.a;
    p[1] = r.b;
    return;
  }
  t -= nf;
  if (t < nb) {  // backward fragment lane: input 16 blk + lane % 16, outputs 32 ch + 8 (lane/16) + j
    int lane = (int)(t % 64);
    int64_t f = t / 64;
    int ch = (int)(f % kco), blk = (int)(f / kco);
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = eff_w(a, l, 32 * ch + 8 * (lane / 16) + j, 16 * blk + lane % 16);
    Raw r = Prec<PREC>::make(v);
    uint4* p = reinterpret_cast<uint4*>(a.wb[l] + t * 32);
    p[0] = r.a;
    p[1] = r.b;
    return;
  }
  t -= nb;
  if (t < nplain) {
    a.w[l][t] = eff_w(a, l, (int)(t / ni), (int)(t % ni));
    return;
  }
  t -= nplain;
  if (t < no) a.b[l][t] = a.has_bias ? a.params[a.off_b[l] + t] : 0.0f;
}

// Gather residual and supervision points into one padded (x, y, t, 0) buffer.

__device__ __forceinline__ void points_thread(const PointsArgs& a, int64_t p) {
  if (p < a.n_zero) a.zero[p] = 0u;
  if (p >= a.n_pad) return;
  int s = 0;
  for (int k = 1; k < a.n_seg; ++k)
    if (p >= a.start[k]) s = k;
  int64_t i = p - a.start[s];
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (i < a.n[s]) {
    const float* x = a.src[s] + i * a.d_in;
    v.x = x[0];
    if (a.d_in > 1) v.y = x[1];
    if (a.d_in > 2) v.z = x[2];
  }
  a.dst[p] = v;
}

__global__ void k_points(const PointsArgs a) { points_thread(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x); }

// Points and weight staging in one launch (independent work): the first nbp blocks gather
// the points, the rest stage the weights.
template <int PREC>
__global__ __launch_bounds__(256) void k_prepare(const PointsArgs pa, const StageArgs sa, int nbp) {
  const int b = blockIdx.x;
  if (b < nbp)
    points_thread(pa, (int64_t)b * 256 + threadIdx.x);
  else
    stage_thread<PREC>(sa, (int64_t)(b - nbp) * 256 + threadIdx.x);
}

__global__ __launch_bounds__(kThreads, 1) void k_grad0(const Grad0Args A) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int64_t per = (A.n_cb + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < A.n_cb ? lo + per : A.n_cb;
  if (A.periodic_mask) {
    int ng = 0;
    for (int k = 0; k < A.d_in; ++k) ng += 2 * ((A.period_train_mask >> k) & 1);
    grad0p_range(A, lo, hi, A.slots + (size_t)blockIdx.x * A.n_out * (A.e + 1 + ng), reinterpret_cast<float*>(smem));
    return;
  }
  grad0_range(A.zb, A.pts, A.n_out, A.d_in, lo, hi, A.slots + (size_t)blockIdx.x * A.n_out * (A.d_in + 1),
              reinterpret_cast<float*>(smem));
}

// d(loss)/dP_k of every trained period (one work-group): the G sums of each output reduced
// over the slots in slot order, weighted by the effective first-layer weights, summed over
// the outputs in order, times d omega / dP = -omega / P = -omega^2 / (2 pi).
__global__ void k_reduce_period(const PeriodReduceArgs A) {
  __shared__ double part[256];
  double part0 = 0.0;  // running sum over the output blocks (thread 0)
  int ng = 0;
  for (int k = 0; k < A.d_in; ++k) ng += 2 * ((A.period_train_mask >> k) & 1);
  int f = 0, t = 0, j = 0;
  for (int k = 0; k < A.d_in; ++k) {
    if (!((A.periodic_mask >> k) & 1)) {
      ++f;
      continue;
    }
    if ((A.period_train_mask >> k) & 1) {
      for (int o0 = 0; o0 < A.n_out; o0 += 256) {
        const int o = o0 + (int)threadIdx.x;
        double v = 0.0;
        if (o < A.n_out) {
          double g0 = 0.0, g1 = 0.0;
          for (int sl = 0; sl < A.n_slots; ++sl) {
            const double* G = A.slots + (size_t)sl * A.slot_stride + (size_t)A.n_out * (A.e + 1) + (size_t)o * ng;
            g0 += G[j];
            g1 += G[j + 1];
          }
          const double wa = A.w64 ? A.w64[(size_t)o * A.e + f] : (double)A.w[(size_t)o * A.e + f];
          const double wb = A.w64 ? A.w64[(size_t)o * A.e + f + 1] : (double)A.w[(size_t)o * A.e + f + 1];
          v = wa * g0 + wb * g1;
        }
        __syncthreads();
        part[threadIdx.x] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
          double sum = o0 == 0 ? 0.0 : part0;
          for (int i = 0; i < 256; ++i) sum += part[i];
          part0 = sum;
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        const double w = A.omega64 ? A.omega64[k] : (double)A.omega[k];
        A.grad[A.off_p + t] = part0 * (-w * w / 6.283185307179586) + (A.accumulate ? A.grad[A.off_p + t] : 0.0);
      }
      ++t;
      j += 2;
    }
    f += 2;
  }
}

// ================================================================== reductions

// Sum the per-work-group FP64 slots of one layer in slot order, then map to the parameter
// layout: with factorised weights W = diag(exp s) V, dL/dV = exp(s) dL/dW and
// dL/ds_o = sum_i W_oi dL/dW_oi (Sec. 2.6.2).

__device__ __forceinline__ void reduce_row(const ReduceArgs& A, int o) {
  // kRedThreads threads: kRedGroups groups of consecutive slots x kRedCols columns.  Each
  // thread sums its group's slots in slot order, the groups are then added in group
  // order: a fixed order, independent of timing.  Column n_in is the bias.
  constexpr int NC = kRedThreads / kRedGroups;
  __shared__ double part[kRedThreads];
  __shared__ double red[NC];
  const int tid = threadIdx.x, grp = tid / NC, col0 = tid % NC;
  const int per = (A.n_slots + kRedGroups - 1) / kRedGroups;
  const int s_lo = grp * per, s_hi = min(A.n_slots, s_lo + per);
  const double es = A.rwf ? exp((double)A.params[A.off_s + o]) : 1.0;
  double ssum = 0.0;
  for (int c0 = 0; c0 <= A.n_in; c0 += NC) {
    const int col = c0 + col0;
    double t = 0.0;
    if (col <= A.n_in) {
      const double* p = A.slots + (col < A.n_in ? (int64_t)o * A.n_in + col : (int64_t)A.n_out * A.n_in + o);
      int sl = s_lo;
      for (; sl + 4 <= s_hi; sl += 4) {
        const double v0 = p[sl * A.slot_stride], v1 = p[(sl + 1) * A.slot_stride];
        const double v2 = p[(sl + 2) * A.slot_stride], v3 = p[(sl + 3) * A.slot_stride];
        t += v0;
        t += v1;
        t += v2;
        t += v3;
      }
      for (; sl < s_hi; ++sl) t += p[sl * A.slot_stride];
    }
    part[tid] = t;
    __syncthreads();
    if (grp == 0 && col <= A.n_in) {
      double s = 0.0;
      for (int q = 0; q < kRedGroups; ++q) s += part[q * NC + col0];
      if (col < A.n_in) {
        const double v = (double)A.params[A.off_w + (int64_t)o * A.n_in + col];
        A.grad[A.off_w + (int64_t)o * A.n_in + col] = es * s + (A.accumulate ? A.grad[A.off_w + (int64_t)o * A.n_in + col] : 0.0);
        ssum += s * es * v;
      } else if (A.has_bias) {
        A.grad[A.off_b + o] = s + (A.accumulate ? A.grad[A.off_b + o] : 0.0);
      }
    }
    __syncthreads();
  }
  if (A.rwf) {  // s_bar[o] = sum_i W[o][i] W_bar[o][i], fixed tree over the columns
    if (grp == 0) red[col0] = ssum;
    __syncthreads();
    for (int st = NC / 2; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    if (tid == 0) A.grad[A.off_s + o] = red[0] + (A.accumulate ? A.grad[A.off_s + o] : 0.0);
  }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_layer(const ReduceArgs A) {
  if ((int)blockIdx.x < A.n_out) reduce_row(A, blockIdx.x);
}

// Per-instance reductions of the item slots: one block per (instance, layer, output row).
__global__ __launch_bounds__(kRedThreads) void k_reduce_batched(const BatchReduceArgs A) {
  const int64_t r = blockIdx.x;
  int lo = 0, hi = A.n_entries - 1;
  while (lo < hi) {  // last entry with row0 <= r
    const int mid = (lo + hi + 1) / 2;
    if (A.rows[mid].row0 <= r) lo = mid; else hi = mid - 1;
  }
  const BatchRow e = A.rows[lo];
  ReduceArgs a;
  a.slots = A.grad_slots + e.slot0;
  a.n_slots = e.n_items;
  a.slot_stride = e.slot_stride;
  a.n_out = e.n_out;
  a.n_in = e.n_in;
  a.rwf = e.rwf;
  a.has_bias = e.has_bias;
  a.params = e.params;
  a.off_w = e.off_w;
  a.off_s = e.off_s;
  a.off_b = e.off_b;
  a.grad = e.grad;
  a.accumulate = 0;
  reduce_row(a, (int)(r - e.row0));
}

// Loss terms of one instance per block: item partial sums added in item order by one
// thread per term (an instance has at most a few hundred items).
__global__ void k_reduce_loss_batched(const BatchLossArgs A) {
  const int i = blockIdx.x;
  __shared__ double term[kMaxOut];
  const int k = threadIdx.x;
  if (k < A.n_res) {
    double t = 0.0;
    const double* p = A.loss_slots + (size_t)A.item0[i] * kMaxTerms + k;
    for (int s = 0; s < A.n_items[i]; ++s) t += p[(size_t)s * kMaxTerms];
    t *= A.w_res[i * kMaxOut + k];
    A.losses[(size_t)i * (1 + A.n_res) + 1 + k] = t;
    term[k] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double total = 0.0;
    for (int q = 0; q < A.n_res; ++q) total += term[q];
    A.losses[(size_t)i * (1 + A.n_res)] = total;
  }
}

__global__ void k_zero_int(int* p) { *p = 0; }

// Loss terms: thread s < 256 sums slots s, s + 256, ... (in that order), then a fixed tree
// over those 256 threads per term (any further threads of the block only pass the barriers).
__device__ __forceinline__ void reduce_loss_block(const LossArgs& A) {
  __shared__ double red[kMaxTerms][256];
  const int tid = threadIdx.x;
  const int nt = A.n_res + A.n_anchor;
  if (tid < 256)
    for (int k = 0; k < nt; ++k) {
      double t = 0.0;
      for (int sl = tid; sl < A.n_slots; sl += 256) t += A.slots[(size_t)sl * kMaxTerms + k];
      red[k][tid] = t;
    }
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st)
      for (int k = 0; k < nt; ++k) red[k][tid] += red[k][tid + st];
    __syncthreads();
  }
  if (tid == 0) {
    const double ws = A.wscale ? *A.wscale : 1.0;
    double total = 0.0;
    for (int k = 0; k < nt; ++k) {
      const double t = red[k][0] * (k < A.n_res ? A.w_res[k] * ws : A.w_anchor[k - A.n_res]);
      A.loss[1 + k] = t + (A.accumulate ? A.loss[1 + k] : 0.0);
      total += t;
    }
    A.loss[0] = total + (A.accumulate ? A.loss[0] : 0.0);
  }
}

__global__ __launch_bounds__(256) void k_reduce_loss(const LossArgs A) { reduce_loss_block(A); }

__global__ __launch_bounds__(kRedThreads) void k_reduce_all(const ReduceAllArgs A) {
  const int b = blockIdx.x;
  if (b >= A.row0[A.n_layers]) {
    reduce_loss_block(A.loss);
    return;
  }
  int l = 0;
  while (b >= A.row0[l + 1]) ++l;
  reduce_row(A.layer[l], b - A.row0[l]);
}

// NaN / Inf scan of the parameters (opt-in check).
__global__ void k_zero_flag(int* flag) { *flag = 0; }

__global__ void k_check_finite(const float* p, int64_t n, int* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(p[i])) *flag = 1;
}



// ================================================================== launchers

int launch_check_finite(const float* p, int64_t n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, s, flag);
  if (n > 0) hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, flag);
  return launch_status(hipGetLastError());
}

int launch_points(const PointsArgs& a, hipStream_t s) {
  const int64_t n = a.n_pad > a.n_zero ? a.n_pad : a.n_zero;
  hipLaunchKernelGGL(k_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return launch_status(hipGetLastError());
}

int launch_grad0(const Grad0Args& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_grad0, dim3(grid), dim3(kThreads), kWaves * 256 * 4 * sizeof(float), s, a);
  return launch_status(hipGetLastError());
}

int launch_zero_int(int* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, p);
  return launch_status(hipGetLastError());
}

int launch_reduce_batched(const BatchReduceArgs& a, hipStream_t s) {
  if (a.n_rows > 0) hipLaunchKernelGGL(k_reduce_batched, dim3((unsigned)a.n_rows), dim3(kRedThreads), 0, s, a);
  return launch_status(hipGetLastError());
}

int launch_reduce_loss_batched(const BatchLossArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_loss_batched, dim3(a.n_inst), dim3(64), 0, s, a);
  return launch_status(hipGetLastError());
}

// Loss terms of the per-term call: each term's own call wrote [total, residual
// components, its supervision set]; the caller's array is [total, components, sets].
__global__ void k_assemble_terms(const double* tmp, int n_terms, int n_res, double* loss) {
  if (threadIdx.x != 0) return;
  const int stride = 2 + n_res;
  double total = 0.0;
  for (int c = 0; c < n_res; ++c) {
    loss[1 + c] = tmp[1 + c];
    total += tmp[1 + c];
  }
  for (int t = 1; t < n_terms; ++t) {
    const double v = tmp[(size_t)t * stride + 1 + n_res];
    loss[1 + n_res + t - 1] = v;
    total += v;
  }
  loss[0] = total;
}

// Loss-balancing weights (Sec. 2.6.4): n_t = ||grad_t||_2 (FP64, fixed summation order),
// lambda_hat_t = sum_s n_s / (n_t + eps), lambda_t <- alpha lambda_t + (1 - alpha) lambda_hat_t.
__global__ void k_balance(const double* grads, int n_terms, int64_t n_params, double* lambda, double* hat,
                          double alpha, double eps) {
  __shared__ double part[256];
  __shared__ double norms[16];
  for (int t = 0; t < n_terms; ++t) {
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n_params; i += 256) {
      const double g = grads[(size_t)t * n_params + i];
      v += g * g;
    }
    part[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) norms[t] = sqrt(part[0]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int t = 0; t < n_terms; ++t) sum += norms[t];
    for (int t = 0; t < n_terms; ++t) {
      const double h = sum / (norms[t] + eps);
      if (hat) hat[t] = h;
      lambda[t] = alpha * lambda[t] + (1.0 - alpha) * h;
    }
  }
}

// Causality weights (Sec. 2.6.8) from the segments' residual losses L^i (bin_loss[i * stride],
// the totals of per-segment forward calls): w_0 = 1, w_i = exp(-eps sum_{k<i} L^k); the
// segments' weights in the loss are w_i / M (wbin, read by the fused calls).
__global__ void k_causal_weights(const double* bin_loss, int stride, int n_bins, double eps, double* wbin,
                                 double* bin_loss_out, double* w_out) {
  if (threadIdx.x != 0) return;
  double cum = 0.0;
  for (int i = 0; i < n_bins; ++i) {
    const double L = bin_loss[(size_t)i * stride];
    const double w = exp(-eps * cum);
    wbin[i] = w / (double)n_bins;
    if (bin_loss_out) bin_loss_out[i] = L;
    if (w_out) w_out[i] = w;
    cum += L;
  }
}

int launch_causal_weights(const double* bin_loss, int stride, int n_bins, double eps, double* wbin, double* bin_loss_out,
                          double* w_out, hipStream_t s) {
  hipLaunchKernelGGL(k_causal_weights, dim3(1), dim3(64), 0, s, bin_loss, stride, n_bins, eps, wbin, bin_loss_out, w_out);
  return launch_status(hipGetLastError());
}

int launch_assemble_terms(const double* tmp, int n_terms, int n_res, double* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble_terms, dim3(1), dim3(64), 0, s, tmp, n_terms, n_res, loss);
  return launch_status(hipGetLastError());
}

int launch_balance(const double* grads, int n_terms, int64_t n_params, double* lambda, double* hat, double alpha,
                   double eps, hipStream_t s) {
  hipLaunchKernelGGL(k_balance, dim3(1), dim3(256), 0, s, grads, n_terms, n_params, lambda, hat, alpha, eps);
  return launch_status(hipGetLastError());
}

int launch_reduce_period(const PeriodReduceArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_period, dim3(1), dim3(256), 0, s, a);
  return launch_status(hipGetLastError());
}

int launch_reduce_layer(const ReduceArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_layer, dim3(a.n_out), dim3(kRedThreads), 0, s, a);
  return launch_status(hipGetLastError());
}

int launch_reduce_loss(const LossArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(256), 0, s, a);
  return launch_status(hipGetLastError());
}

int launch_reduce_all(const ReduceAllArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_all, dim3((unsigned)(a.row0[a.n_layers] + 1)), dim3(kRedThreads), 0, s, a);
  return launch_status(hipGetLastError());
}

int launch_prepare(int prec, const PointsArgs& pa, const StageArgs& sa, hipStream_t s) {
  const int64_t np = pa.n_pad > pa.n_zero ? pa.n_pad : pa.n_zero;
  const int nbp = (int)((np + 255) / 256);
  const int nbs = (int)((sa.cum[sa.n_layers] + 255) / 256);
  const dim3 grid((unsigned)(nbp + (nbs > 0 ? nbs : 1)));
  if (prec == kFP32)
    hipLaunchKernelGGL(k_prepare<kFP32>, grid, dim3(256), 0, s, pa, sa, nbp);
  else if (prec == kFP16X3)
    hipLaunchKernelGGL(k_prepare<kFP16X3>, grid, dim3(256), 0, s, pa, sa, nbp);
  else
    hipLaunchKernelGGL(k_prepare<kBF16X3>, grid, dim3(256), 0, s, pa, sa, nbp);
  return launch_status(hipGetLastError());
}

}  // namespace pinn
