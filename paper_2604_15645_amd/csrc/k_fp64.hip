// k_fp64.hip -- the FP64 precision: the whole step in double precision on the vector ALU,
// one thread per point, for tight checks of the method on the GPU (finite differences at
// small steps, parity with an FP64 reference to rounding).  Not a performance path.
//
// Layout of the per-point buffers: value (row, channel) of point p at [(row * 4 + c) * n_pad
// + p], so consecutive threads touch consecutive addresses.  A[l] holds the jets feeding
// linear layer l (A[0] the embedding), Z[l] the pre-activation jets of hidden layer l, ZB[l]
// their adjoints, YB the output-jet adjoint seed, DW the derivative of the embedding
// features of trained periods with respect to omega.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pinn_device.h"

namespace pinn {

namespace {

// sigma and its first three derivatives (tanh, or sin(w0 z)), in double precision.
__device__ __forceinline__ void act64(int act, double w0, double z, double& s0, double& s1, double& s2, double& s3) {
  if (act == kTanh) {
    const double t = tanh(z), d = 1.0 - t * t;
    s0 = t;
    s1 = d;
    s2 = -2.0 * t * d;
    s3 = d * (6.0 * t * t - 2.0);
  } else {
    const double sn = sin(w0 * z), cs = cos(w0 * z);
    s0 = sn;
    s1 = w0 * cs;
    s2 = -w0 * w0 * sn;
    s3 = -w0 * w0 * w0 * cs;
  }
}

__device__ __forceinline__ double& at(double* buf, int64_t n_pad, int row, int c, int64_t p) {
  return buf[((int64_t)row * 4 + c) * n_pad + p];
}
__device__ __forceinline__ double at(const double* buf, int64_t n_pad, int row, int c, int64_t p) {
  return buf[((int64_t)row * 4 + c) * n_pad + p];
}

// Jets of the embedding features of one point into A0 (and, for trained periods, their
// omega-derivatives into DW, one row per trained feature).
__device__ void embed64(const F64Args& A, int64_t p, const float4 x) {
  const int d = A.d_in, e = A.e;
  const double xs[3] = {(double)x.x, (double)x.y, (double)x.z};
  const bool lap = A.lapch == 3;
  for (int f = 0; f < e; ++f)
    for (int c = 0; c < 4; ++c) at(A.a[0], A.n_pad, f, c, p) = 0.0;
  if (A.periodic_mask) {
    int f = 0, t = 0;
    for (int k = 0; k < d; ++k) {
      if (!((A.periodic_mask >> k) & 1)) {
        at(A.a[0], A.n_pad, f, 0, p) = xs[k];
        at(A.a[0], A.n_pad, f, 1 + k, p) = 1.0;
        ++f;
        continue;
      }
      const double w = A.omega[k], xk = xs[k], cv = cos(w * xk), sv = sin(w * xk);
      const bool inl = lap && ((A.lap_mask >> k) & 1);
      at(A.a[0], A.n_pad, f, 0, p) = cv;
      at(A.a[0], A.n_pad, f + 1, 0, p) = sv;
      at(A.a[0], A.n_pad, f, 1 + k, p) = -w * sv;
      at(A.a[0], A.n_pad, f + 1, 1 + k, p) = w * cv;
      if (inl) {
        at(A.a[0], A.n_pad, f, 3, p) = -w * w * cv;
        at(A.a[0], A.n_pad, f + 1, 3, p) = -w * w * sv;
      }
      if ((A.period_train_mask >> k) & 1) {
        for (int c = 0; c < 4; ++c) {
          at(A.dw, A.n_pad, t, c, p) = 0.0;
          at(A.dw, A.n_pad, t + 1, c, p) = 0.0;
        }
        at(A.dw, A.n_pad, t, 0, p) = -xk * sv;
        at(A.dw, A.n_pad, t + 1, 0, p) = xk * cv;
        at(A.dw, A.n_pad, t, 1 + k, p) = -sv - w * xk * cv;
        at(A.dw, A.n_pad, t + 1, 1 + k, p) = cv - w * xk * sv;
        if (inl) {
          at(A.dw, A.n_pad, t, 3, p) = -2.0 * w * cv + w * w * xk * sv;
          at(A.dw, A.n_pad, t + 1, 3, p) = -2.0 * w * sv - w * w * xk * cv;
        }
        t += 2;
      }
      f += 2;
    }
    return;
  }
  if (A.n_freq == 0) {
    for (int k = 0; k < d; ++k) {
      at(A.a[0], A.n_pad, k, 0, p) = xs[k];
      at(A.a[0], A.n_pad, k, 1 + k, p) = 1.0;
    }
    return;
  }
  const int m = A.n_freq;
  for (int j = 0; j < m; ++j) {
    double v = 0.0, bl = 0.0;
    double b[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < d; ++k) {
      b[k] = (double)A.B[k * m + j];
      v += xs[k] * b[k];
      if ((A.lap_mask >> k) & 1) bl += b[k] * b[k];
    }
    const double cv = cos(v), sv = sin(v);
    at(A.a[0], A.n_pad, j, 0, p) = cv;
    at(A.a[0], A.n_pad, m + j, 0, p) = sv;
    for (int k = 0; k < d; ++k) {
      at(A.a[0], A.n_pad, j, 1 + k, p) = -sv * b[k];
      at(A.a[0], A.n_pad, m + j, 1 + k, p) = cv * b[k];
    }
    if (lap) {
      at(A.a[0], A.n_pad, j, 3, p) = -cv * bl;
      at(A.a[0], A.n_pad, m + j, 3, p) = -sv * bl;
    }
  }
}

// Channel weights of the first derivatives inside the Laplacian channel 3.
__device__ __forceinline__ void lapw64(const F64Args& A, double& w1, double& w2) {
  const bool lap = A.lapch == 3;
  w1 = lap && (A.lap_mask & 1) ? 1.0 : 0.0;
  w2 = lap && (A.lap_mask & 2) ? 1.0 : 0.0;
}

}  // namespace

// Forward pass, residual or misfit, loss partial sums (one slot of kMaxTerms per block) and
// the output-jet seed, one thread per padded point.
__global__ __launch_bounds__(256) void k64_forward(const F64Args A) {
  __shared__ double red[kMaxTerms][256];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double part[kMaxTerms];
  for (int k = 0; k < kMaxTerms; ++k) part[k] = 0.0;
  if (p < A.n_pad) {
    const float4 x = A.pts[p];
    embed64(A, p, x);
    double w1, w2;
    lapw64(A, w1, w2);
    // hidden layers
    for (int l = 0; l < A.L; ++l) {
      const int ni = A.n_in[l], no = A.n_out[l];
      const double* W = A.w[l];
      for (int o = 0; o < no; ++o) {
        double z[4] = {A.b[l][o], 0.0, 0.0, 0.0};
        for (int i = 0; i < ni; ++i) {
          const double wv = W[(int64_t)o * ni + i];
          for (int c = 0; c < 4; ++c) z[c] += wv * at(A.a[l], A.n_pad, i, c, p);
        }
        double s0, s1, s2, s3;
        act64(A.act, A.w0, z[0], s0, s1, s2, s3);
        for (int c = 0; c < 4; ++c) at(A.z[l], A.n_pad, o, c, p) = z[c];
        at(A.a[l + 1], A.n_pad, o, 0, p) = s0;
        at(A.a[l + 1], A.n_pad, o, 1, p) = s1 * z[1];
        at(A.a[l + 1], A.n_pad, o, 2, p) = s1 * z[2];
        at(A.a[l + 1], A.n_pad, o, 3, p) =
            A.lapch == 3 ? s2 * (w1 * z[1] * z[1] + w2 * z[2] * z[2]) + s1 * z[3] : s1 * z[3];
      }
    }
    // output layer (linear)
    double y[kMaxOut][4], yb[kMaxOut][4];
    for (int o = 0; o < kMaxOut; ++o)
      for (int c = 0; c < 4; ++c) y[o][c] = yb[o][c] = 0.0;
    const int L = A.L, ni = A.n_in[L];
    for (int o = 0; o < A.d_out; ++o) {
      y[o][0] = A.b[L][o];
      for (int i = 0; i < ni; ++i) {
        const double wv = A.w[L][(int64_t)o * ni + i];
        for (int c = 0; c < 4; ++c) y[o][c] += wv * at(A.a[L], A.n_pad, i, c, p);
      }
    }
    int sid = 0;
    for (int s = 1; s < A.seg.n_seg; ++s)
      if (p >= A.seg.start[s]) sid = s;
    const int64_t i = p - A.seg.start[sid];
    if (i < A.seg.n[sid]) {
      if (sid == 0) {
        double r[kMaxOut], seed[kMaxOut];
        const double ws = A.wscale ? *A.wscale : 1.0;
        for (int c = 0; c < kMaxOut; ++c) seed[c] = A.seed[c] * ws;
        residual_point_t<double>(A.pde_id, A.coef, seed, y, r, yb);
        for (int c = 0; c < A.n_res; ++c) {
          part[c] = r[c] * r[c];
          if (A.residual) A.residual[i * A.n_res + c] = (float)r[c];
        }
      } else {
        const int a = sid - 1;
        const double lam = A.lam_anchor[a];
        for (int o = 0; o < A.d_out; ++o) {
          if (!(A.seg.out_mask[a] & (1 << o))) continue;
          const double dlt = y[o][0] - (double)A.seg.targets[a][i * A.d_out + o];
          part[A.n_res + a] += dlt * dlt;
          yb[o][0] = lam * dlt;
        }
      }
    }
    for (int o = 0; o < A.d_out; ++o)
      for (int c = 0; c < 4; ++c) at(A.yb, A.n_pad, o, c, p) = yb[o][c];
  }
  // block sums in a fixed tree order, one slot per block
  for (int k = 0; k < kMaxTerms; ++k) red[k][threadIdx.x] = part[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < kMaxTerms; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < kMaxTerms) A.loss_slots[(size_t)blockIdx.x * kMaxTerms + threadIdx.x] = red[threadIdx.x][0];
}

// Reverse sweep of one point: adjoints of every hidden layer's pre-activation jets (ZB) and,
// with trained periods, the embedding adjoint is not needed (their gradient comes from the
// first layer's sums).  AB0 / AB1: adjoint of the current layer's input activations.
__global__ __launch_bounds__(256) void k64_backward(const F64Args A) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= A.n_pad) return;
  double w1, w2;
  lapw64(A, w1, w2);
  const int L = A.L;
  // output layer: abar_L = W_out^T ybar
  double* ab = A.ab[0];
  {
    const int ni = A.n_in[L];
    for (int i = 0; i < ni; ++i) {
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      for (int o = 0; o < A.d_out; ++o) {
        const double wv = A.w[L][(int64_t)o * ni + i];
        for (int c = 0; c < 4; ++c) v[c] += wv * at(A.yb, A.n_pad, o, c, p);
      }
      for (int c = 0; c < 4; ++c) at(ab, A.n_pad, i, c, p) = v[c];
    }
  }
  for (int l = L - 1; l >= 0; --l) {
    const int no = A.n_out[l], ni = A.n_in[l];
    // activation adjoint: zbar from abar and the pre-activation jets
    for (int o = 0; o < no; ++o) {
      double z[4], a[4];
      for (int c = 0; c < 4; ++c) {
        z[c] = at(A.z[l], A.n_pad, o, c, p);
        a[c] = at(ab, A.n_pad, o, c, p);
      }
      double s0, s1, s2, s3;
      act64(A.act, A.w0, z[0], s0, s1, s2, s3);
      double zb[4];
      if (A.lapch == 3) {
        const double q = w1 * z[1] * z[1] + w2 * z[2] * z[2];
        zb[0] = a[0] * s1 + a[1] * s2 * z[1] + a[2] * s2 * z[2] + a[3] * (s3 * q + s2 * z[3]);
        zb[1] = a[1] * s1 + 2.0 * a[3] * s2 * w1 * z[1];
        zb[2] = a[2] * s1 + 2.0 * a[3] * s2 * w2 * z[2];
        zb[3] = a[3] * s1;
      } else {
        zb[0] = a[0] * s1 + s2 * (a[1] * z[1] + a[2] * z[2] + a[3] * z[3]);
        zb[1] = a[1] * s1;
        zb[2] = a[2] * s1;
        zb[3] = a[3] * s1;
      }
      for (int c = 0; c < 4; ++c) at(A.zb[l], A.n_pad, o, c, p) = zb[c];
    }
    if (l == 0) break;
    // input adjoint of layer l: abar_{l-1} = W_l^T zbar_l
    double* nab = A.ab[(L - l) & 1];
    for (int i = 0; i < ni; ++i) {
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      for (int o = 0; o < no; ++o) {
        const double wv = A.w[l][(int64_t)o * ni + i];
        for (int c = 0; c < 4; ++c) v[c] += wv * at(A.zb[l], A.n_pad, o, c, p);
      }
      for (int c = 0; c < 4; ++c) at(nab, A.n_pad, i, c, p) = v[c];
    }
    ab = nab;
  }
}

// Weight and bias sums of linear layer l over all points in point order: one thread per
// (output o, column j): j < n_in the weight, j == n_in the bias, j > n_in (first layer,
// trained periods) the omega terms G.  Slot layout [n_out][n_in], [n_out], [n_out][ng].
__global__ __launch_bounds__(256) void k64_wgrad(const F64Args A, int l, double* slot) {
  const int no = l == A.L ? A.d_out : A.n_out[l], ni = A.n_in[l];
  const int ng = l == 0 ? A.ng : 0;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = ni + 1 + ng;
  if (t >= (int64_t)no * per) return;
  const int o = (int)(t / per), j = (int)(t % per);
  const double* zb = l == A.L ? A.yb : A.zb[l];
  double s = 0.0;
  if (j < ni) {
    const double* a = A.a[l];
    for (int64_t p = 0; p < A.n_pad; ++p)
      for (int c = 0; c < 4; ++c) s += at(zb, A.n_pad, o, c, p) * at(a, A.n_pad, j, c, p);
    slot[(int64_t)o * ni + j] = s;
  } else if (j == ni) {
    for (int64_t p = 0; p < A.n_pad; ++p) s += at(zb, A.n_pad, o, 0, p);
    slot[(int64_t)no * ni + o] = s;
  } else {
    const int g = j - ni - 1;
    for (int64_t p = 0; p < A.n_pad; ++p)
      for (int c = 0; c < 4; ++c) s += at(zb, A.n_pad, o, c, p) * at(A.dw, A.n_pad, g, c, p);
    slot[(int64_t)no * (ni + 1) + (int64_t)o * ng + g] = s;
  }
}

// Effective weights W = diag(exp s) V (Sec. 2.6.2) and biases in double, and omega_k =
// 2 pi / P_k of the periodic inputs.
__global__ void k64_stage(const F64StageArgs S) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 3) {
    const int k = (int)t;
    double w = 0.0;
    if ((S.periodic_mask >> k) & 1) {
      double P = (double)S.period[k];
      if ((S.period_train_mask >> k) & 1) {
        int r = 0;
        for (int j = 0; j < k; ++j) r += (S.period_train_mask >> j) & 1;
        P = (double)S.params[S.off_p + r];
      }
      w = 6.283185307179586 / P;
    }
    S.omega[k] = w;
  }
  int64_t u = t;
  for (int l = 0; l < S.n_layers; ++l) {
    const int64_t nw = (int64_t)S.n_out[l] * S.n_in[l];
    if (u < nw) {
      const int o = (int)(u / S.n_in[l]);
      double v = (double)S.params[S.off_w[l] + u];
      if (S.rwf) v *= exp((double)S.params[S.off_s[l] + o]);
      S.w[l][u] = v;
      return;
    }
    u -= nw;
    if (u < S.n_out[l]) {
      S.b[l][u] = S.has_bias ? (double)S.params[S.off_b[l] + u] : 0.0;
      return;
    }
    u -= S.n_out[l];
  }
}

int launch_fp64(const F64StageArgs& s, const F64Args& a, double* const* slots, hipStream_t st) {
  int64_t n = 0;
  for (int l = 0; l < s.n_layers; ++l) n += (int64_t)s.n_out[l] * (s.n_in[l] + 1);
  n = n > 3 ? n : 3;
  hipLaunchKernelGGL(k64_stage, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s);
  const unsigned blocks = (unsigned)((a.n_pad + 255) / 256);
  hipLaunchKernelGGL(k64_forward, dim3(blocks), dim3(256), 0, st, a);
  if (slots) {
    hipLaunchKernelGGL(k64_backward, dim3(blocks), dim3(256), 0, st, a);
    for (int l = 0; l <= a.L; ++l) {
      const int no = l == a.L ? a.d_out : a.n_out[l];
      const int64_t nt = (int64_t)no * (a.n_in[l] + 1 + (l == 0 ? a.ng : 0));
      hipLaunchKernelGGL(k64_wgrad, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, a, l, slots[l]);
    }
  }
  return launch_status(hipGetLastError());
}

}  // namespace pinn
