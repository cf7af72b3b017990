// pinn_api.cpp -- host side of the C ABI declared in include/pinn.h: descriptor checks
// (before any HIP call), launch planning, workspace layout and the launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/pinn.h"
#include "pinn_internal.h"

using namespace pinn;

namespace {

constexpr int64_t kAlign = 256;
constexpr int kGridCap = 256;  // MI355X: 256 compute units, one 512-thread work-group each

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct Dims {
  int L, n_layers, d_in, d_out, e;
  int n_in[kMaxLayers], n_out[kMaxLayers];
  int64_t off_w[kMaxLayers], off_s[kMaxLayers], off_b[kMaxLayers];
  int64_t n_params;
  int64_t off_p;  // first trainable period (after every layer's parameters)
  int n_tp;       // trainable periods
  int hmax;      // widest hidden layer
  int H;         // width bucket of the kernels: 32, 64, 128 or 256
};

int check_net(const pinn_net* net, Dims* d) {
  if (!net) return PINN_E_INVALID;
  if (net->d_in < 1 || net->d_in > 3 || net->d_out < 1 || net->d_out > kMaxOut) return PINN_E_INVALID;
  if (net->n_hidden < 0 || net->n_hidden > kMaxHidden) return PINN_E_INVALID;
  if (net->act != PINN_ACT_TANH && net->act != PINN_ACT_SIN) return PINN_E_INVALID;
  if (net->n_freq < 0 || net->n_freq > 4096) return PINN_E_INVALID;
  if ((net->rwf != 0 && net->rwf != 1) || (net->has_bias != 0 && net->has_bias != 1)) return PINN_E_INVALID;
  if (!std::isfinite(net->w0)) return PINN_E_INVALID;
  for (int l = 0; l < net->n_hidden; ++l)
    if (net->width[l] < 1 || net->width[l] > 4096) return PINN_E_INVALID;
  const int all = (1 << net->d_in) - 1;
  if ((net->periodic_mask & ~all) || (net->period_train_mask & ~net->periodic_mask)) return PINN_E_INVALID;
  for (int k = 0; k < net->d_in; ++k)
    if ((net->periodic_mask >> k) & 1 && !((net->period_train_mask >> k) & 1) &&
        !(std::isfinite(net->period[k]) && net->period[k] != 0.0f))
      return PINN_E_INVALID;
  Dims& D = *d;
  D.L = net->n_hidden;
  D.n_layers = D.L + 1;
  D.d_in = net->d_in;
  D.d_out = net->d_out;
  D.e = net->n_freq > 0 ? 2 * net->n_freq : net->d_in;
  if (net->periodic_mask) {
    D.e = 0;
    for (int k = 0; k < net->d_in; ++k) D.e += (net->periodic_mask >> k) & 1 ? 2 : 1;
  }
  int64_t off = 0;
  D.hmax = 0;
  for (int l = 0; l < D.n_layers; ++l) {
    D.n_in[l] = l == 0 ? D.e : net->width[l - 1];
    D.n_out[l] = l == D.L ? D.d_out : net->width[l];
    if (l < D.L) D.hmax = std::max(D.hmax, D.n_out[l]);
    D.off_w[l] = off;
    off += (int64_t)D.n_in[l] * D.n_out[l];
    D.off_s[l] = -1;
    D.off_b[l] = -1;
    if (net->rwf) { D.off_s[l] = off; off += D.n_out[l]; }
    if (net->has_bias) { D.off_b[l] = off; off += D.n_out[l]; }
  }
  D.off_p = off;
  D.n_tp = 0;
  for (int k = 0; k < net->d_in; ++k) D.n_tp += (net->period_train_mask >> k) & 1;
  D.n_params = off + D.n_tp;
  D.H = D.hmax <= 32 ? 32 : D.hmax <= 64 ? 64 : D.hmax <= 128 ? 128 : 256;
  return PINN_OK;
}

// What the kernels implement (beyond what the descriptor format allows).
int check_supported(const pinn_net* net, const Dims& D, int lap_mask) {
  if (net->n_hidden < 1) return PINN_E_UNSUPPORTED;
  for (int l = 0; l < D.L; ++l)
    if (D.n_out[l] % 32 != 0 || D.n_out[l] > 256) return PINN_E_UNSUPPORTED;
  if (net->n_freq > 0 && (net->n_freq % 16 != 0 || 2 * net->n_freq > 256)) return PINN_E_UNSUPPORTED;
  if (net->periodic_mask && net->n_freq > 0) return PINN_E_UNSUPPORTED;  // one embedding at a time
  const int C = 1 + net->d_in + (lap_mask ? 1 : 0);
  if (C > 4) return PINN_E_UNSUPPORTED;
  if (lap_mask && net->d_in != 2) return PINN_E_UNSUPPORTED;
  return PINN_OK;
}

int check_pde(const pinn_net* net, const pinn_pde* pde) {
  if (!pde) return PINN_E_INVALID;
  if (pde->lap_mask < 0 || (pde->lap_mask & ~((1 << net->d_in) - 1))) return PINN_E_INVALID;
  for (int k = 0; k < kMaxOut; ++k)
    if (!std::isfinite(pde->lambda_res[k]) || pde->lambda_res[k] < 0) return PINN_E_INVALID;
  if (!std::isfinite(pde->norm_N) || pde->norm_N < 0) return PINN_E_INVALID;
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(pde->coef[k])) return PINN_E_INVALID;
  switch (pde->pde_id) {
    case PINN_PDE_BURGERS:  // the Laplacian channel must be u_xx alone
      if (net->d_in != 2 || pde->lap_mask != 1) return PINN_E_UNSUPPORTED;
      return PINN_OK;
    case PINN_PDE_EULER1D:
      if (net->d_in != 2 || net->d_out != 3 || !(pde->coef[0] > 1.0)) return PINN_E_UNSUPPORTED;
      return PINN_OK;
    case PINN_PDE_NS2D_STEADY:
      if (net->d_in != 2 || net->d_out != 3 || (pde->lap_mask & 3) != 3 || pde->coef[0] == 0.0)
        return PINN_E_UNSUPPORTED;
      return PINN_OK;
    case PINN_PDE_MAXWELL_TE2D:
      if (net->d_in != 3 || net->d_out != 3 || pde->coef[0] == 0.0 || pde->coef[1] == 0.0)
        return PINN_E_UNSUPPORTED;
      return PINN_OK;
    case PINN_PDE_ADVECTION:  // first derivatives only
      if (net->d_in != 2 || pde->lap_mask != 0) return PINN_E_UNSUPPORTED;
      return PINN_OK;
    case PINN_PDE_ALLEN_CAHN:  // the Laplacian channel must be u_xx alone
      if (net->d_in != 2 || pde->lap_mask != 1) return PINN_E_UNSUPPORTED;
      return PINN_OK;
    case PINN_PDE_EULER2D:  // first derivatives in x, y, t
      if (net->d_in != 3 || net->d_out != 4 || pde->lap_mask != 0 || !(pde->coef[0] > 1.0))
        return PINN_E_UNSUPPORTED;
      return PINN_OK;
    default:
      return PINN_E_UNSUPPORTED;
  }
}

// Kernel precision code of a public precision, or the status to return for it.
int kernel_prec(int prec, int* kp) {
  switch (prec) {
    case PINN_PREC_FP32: *kp = kFP32; return PINN_OK;
    case PINN_PREC_BF16X3: *kp = kBF16X3; return PINN_OK;
    case PINN_PREC_FP16X3: *kp = kFP16X3; return PINN_OK;
    case PINN_PREC_BF16: return PINN_E_UNSUPPORTED;  // single-product BF16: see pinn.h
    case PINN_PREC_FP64: return PINN_E_UNSUPPORTED;  // its own kernels (run_fp64); not batched
    default: return PINN_E_INVALID;
  }
}

int n_res_of(int pde_id) {
  switch (pde_id) {
    case PINN_PDE_BURGERS:
    case PINN_PDE_ADVECTION:
    case PINN_PDE_ALLEN_CAHN: return 1;
    case PINN_PDE_EULER1D:
    case PINN_PDE_NS2D_STEADY:
    case PINN_PDE_MAXWELL_TE2D: return 3;
    case PINN_PDE_EULER2D: return 4;
    default: return -1;
  }
}

// Forward tile size: the largest of the width bucket's default that fits the LDS budget.
// Kernel activation code: the activation, plus kLapFlag when jet channel 3 carries a Laplacian.
int act_code(const pinn_net* net, const pinn_pde* pde) { return net->act | (pde->lap_mask ? kLapFlag : 0); }

// Launch numbers of the split backward (pacing words carry them; they only grow).
unsigned long long next_launch_id() {
  static std::atomic<unsigned long long> n{1};
  return n.fetch_add(1, std::memory_order_relaxed);
}

int default_fwd_p(int H) { return fwd_default_p(H); }
int default_bwd_p(int H) { return 2048 / H; }
int embed_bwd_p(int H) { return H == 256 ? 8 : 16; }
constexpr size_t kLdsBudget = 160 * 1024;

size_t fwd_lds(int P, int kmax, int H) {
  const int NW = fwd_waves(H, P);
  const int WN = std::min(NW, H / 16);
  const int WC = NW / WN;
  size_t b = (size_t)4 * P * (kmax * 4 + 16) * (fwd_double_x(P) ? 2 : 1);  // X (one or two)
  b += (size_t)P * 16;                           // PT
  b += (size_t)P * kMaxOut * 4 * 4 * 2;          // YJ, YB
  b += NW * 8 * 4;                               // RED
  b += kMaxTerms * 8;                            // LOSS
  b += (size_t)WC * kMaxOut * H * 8 + kMaxOut * 8;  // WL, BL
  b += kFourierLds;                              // BF
  b += kOutLds + 16;                             // OW (16-byte aligned)
  return b;
}
// Layer backward: staged output adjoint (and staged input pre-activations), Q tile, and
// (hidden layers) R tile.
size_t bwd_lds(int PB, int n_in, int n_out, bool with_prev) {
  size_t b = (size_t)PB * n_out * 16 + (size_t)n_in * (4 * PB * 4 + 16);
  if (with_prev) b += (size_t)PB * n_in * 16 + (size_t)4 * PB * (n_out * 4 + 16);
  return b;
}

struct Plan {
  Dims D;
  int prec, act;
  int n_res, n_anchor, n_seg;
  int64_t seg_start[1 + kMaxAnchors], seg_n[1 + kMaxAnchors];
  int64_t n_pad;
  int pf, pb;             // forward tile points, backward sub-tile points (hidden layers)
  int kmax;
  int pb0;
  bool wide, wide0;       // wide bf16x3 backward for the hidden layers / the embedding layer
  bool split;             // split-role bf16x3 backward for the hidden layers
  bool fuse0;             // identity first layer: its gradient summed by layer 1's backward
                          // (split-role or plain kernel; one slot per work-group or pair)
  int64_t n_tiles, n_sub, n_sub0;
  int grid_f, grid_b, grid_b0, grid_g0;
  size_t lds_f, lds_b, lds_b0;
  bool with_grad;
  // workspace offsets
  int64_t o_pts, o_wf[kMaxLayers], o_wb[kMaxLayers], o_w[kMaxLayers], o_b[kMaxLayers];
  int64_t o_zs[kMaxHidden], o_zb[2], o_loss, o_out, o_layer[kMaxLayers], o_flag, o_pace, o_amax, o_omega;
  int ng0;                // period sums per first-layer output (2 per trained period)
  int64_t zs_stride;
  int64_t bytes;
};

// Slots of the first layer's sums when layer 1's backward forms them: one per work-group
// pair of the split-role kernel, one per work-group of the plain kernel.
int fused0_slots(const Plan& p) { return p.split ? p.grid_b / 2 : p.grid_b; }


int make_plan(const pinn_net* net, const pinn_pde* pde, int64_t n_points, const pinn_anchor* anchors,
              int n_anchor, int prec, int with_grad, const pinn_tune* tune, Plan* P) {
  Plan& p = *P;
  std::memset(&p, 0, sizeof(p));
  int rc = check_net(net, &p.D);
  if (rc) return rc;
  rc = check_pde(net, pde);
  if (rc) return rc;
  int kp = 0;
  rc = kernel_prec(prec, &kp);
  if (rc) return rc;
  if (n_points < 0 || n_anchor < 0 || n_anchor > kMaxAnchors) return PINN_E_INVALID;
  if (n_anchor > 0 && !anchors) return PINN_E_INVALID;
  for (int a = 0; a < n_anchor; ++a) {
    if (anchors[a].n < 0 || !std::isfinite(anchors[a].lambda) || anchors[a].lambda < 0) return PINN_E_INVALID;
    if (anchors[a].out_mask <= 0 || anchors[a].out_mask >= (1 << net->d_out)) return PINN_E_INVALID;
  }
  if (n_points + [&] { int64_t t = 0; for (int a = 0; a < n_anchor; ++a) t += anchors[a].n; return t; }() == 0)
    return PINN_E_INVALID;
  rc = check_supported(net, p.D, pde->lap_mask);
  if (rc) return rc;
  const Dims& D = p.D;
  p.prec = kp;
  p.act = net->act;
  p.with_grad = with_grad != 0;
  p.n_res = n_res_of(pde->pde_id);
  p.n_anchor = n_anchor;
  p.n_seg = 1 + n_anchor;
  int64_t cur = 0;
  for (int s = 0; s < p.n_seg; ++s) {
    p.seg_start[s] = cur;
    p.seg_n[s] = s == 0 ? n_points : anchors[s - 1].n;
    cur += align_up(std::max<int64_t>(p.seg_n[s], 1), kSegAlign);
  }
  p.n_pad = cur;
  p.kmax = std::max(D.e, D.hmax);
  if (p.kmax % 32) p.kmax = (int)align_up(p.kmax, 32);
  // tile sizes
  p.pf = default_fwd_p(D.H);
  if (tune && tune->tile_points > 0) {
    int t = tune->tile_points;
    if (t != 16 && t != p.pf && t != fwd_half_p(D.H)) return PINN_E_UNSUPPORTED;
    p.pf = t;
  }
  if (fwd_lds(p.pf, p.kmax, D.H) > kLdsBudget) p.pf = 16;
  if (fwd_lds(p.pf, p.kmax, D.H) > kLdsBudget) return PINN_E_UNSUPPORTED;
  // layer backward: the wide bf16x3 kernel when the layer input width is a multiple of
  // 128 (hidden widths 128 / 256; Fourier embeddings of 64 / 128 frequencies)
  bool wide = is_split(kp) && D.H >= 128;
  for (int j = 1; j < D.L; ++j) wide = wide && D.n_in[j] % 128 == 0;
  const bool wide0 = is_split(kp) && net->n_freq > 0 && (D.e / 16) % 8 == 0;
  p.wide = wide;
  p.wide0 = wide0;
  // split roles: uniform hidden width H (128 or 256); the grid is a multiple of 16
  p.split = wide;
  for (int j = 1; j < D.L; ++j) p.split = p.split && D.n_in[j] == D.H && D.n_out[j] == D.H;
  p.pb = wide ? wide_pb(D.H) : default_bwd_p(D.H);
  if (tune && tune->bwd_points > 0) {  // the split-role kernel's sub-tile: default or half
    if (!p.split || (tune->bwd_points != p.pb && tune->bwd_points != p.pb / 2)) return PINN_E_UNSUPPORTED;
    p.pb = tune->bwd_points;
  }
  p.pb0 = wide0 ? wide_pb(D.H) : embed_bwd_p(D.H);
  p.lds_f = fwd_lds(p.pf, p.kmax, D.H);
  p.lds_b = wide ? (size_t)2 * p.pb * D.H * 16 : bwd_lds(p.pb, D.H, D.H, true);
  p.lds_b0 = wide0 ? (size_t)2 * p.pb0 * D.H * 16 + kFourierLds : bwd_lds(p.pb0, 256, D.H, false);
  if (p.lds_b > kLdsBudget || p.lds_b0 > kLdsBudget) return PINN_E_UNSUPPORTED;
  p.n_tiles = p.n_pad / p.pf;
  p.n_sub = p.n_pad / p.pb;
  p.n_sub0 = p.n_pad / p.pb0;
  int cap = kGridCap;
  if (tune && tune->grid > 0) cap = tune->grid;
  // (several resident forward work-groups per compute unit for the small-wave shapes)
  p.grid_f = (int)std::min<int64_t>(p.n_tiles, tune && tune->grid > 0 ? cap : cap * fwd_wg_per_cu(D.H, p.pf));
  p.grid_b = (int)std::min<int64_t>(p.n_sub, cap);
  if (p.split) {  // two roles of G work-groups each, G a multiple of 8
    const int64_t G = std::min<int64_t>(align_up(std::min<int64_t>(p.n_sub, cap / 2), 8), std::max(8, cap / 2 / 8 * 8));
    p.grid_b = (int)(2 * G);
  }
  p.grid_b0 = (int)std::min<int64_t>(p.n_sub0, cap);
  p.grid_g0 = (int)std::min<int64_t>(std::max<int64_t>(1, p.n_pad / 4 / 64), kGridCap);
  p.fuse0 = p.with_grad && (p.split || !p.wide) && D.L >= 2 && net->n_freq == 0 && !net->periodic_mask;
  // workspace layout
  int64_t o = 0;
  auto take = [&](int64_t bytes) { int64_t r = o; o = align_up(o + bytes, kAlign); return r; };
  p.o_pts = take(p.n_pad * 16);
  for (int l = 0; l < D.n_layers; ++l) {
    const int64_t nbo = (D.n_out[l] + 15) / 16, kci = (D.n_in[l] + 31) / 32;
    const int64_t nbi = (D.n_in[l] + 15) / 16, kco = (D.n_out[l] + 31) / 32;
    p.o_wf[l] = take(nbo * kci * 64 * 32);
    p.o_wb[l] = take(nbi * kco * 64 * 32);
    p.o_w[l] = take((int64_t)D.n_out[l] * D.n_in[l] * 4);
    p.o_b[l] = take((int64_t)D.n_out[l] * 4);
  }
  p.o_loss = take((int64_t)p.grid_f * kMaxTerms * 8);
  p.o_flag = take(16);
  p.o_amax = take(kMaxHidden * 4);
  p.o_omega = take(16);
  p.ng0 = 2 * D.n_tp;
  p.o_pace = take((int64_t)std::max(p.grid_b, 1) * 8);  // split-backward pacing words (any content)
  if (p.with_grad) {
    p.zs_stride = p.n_pad * 4 * D.hmax;
    p.o_zs[0] = take(p.zs_stride * D.L * 4);
    p.o_zb[0] = take(p.n_pad * 4 * D.hmax * 4);
    p.o_zb[1] = take(p.n_pad * 4 * D.hmax * 4);
    p.o_out = take((int64_t)p.grid_f * D.d_out * (D.n_in[D.L] + 1) * 8);
    for (int l = 0; l < D.L; ++l) {
      int grid = l == 0 ? (net->n_freq > 0 ? p.grid_b0 : (p.fuse0 ? fused0_slots(p) : p.grid_g0)) : p.grid_b;
      p.o_layer[l] = take((int64_t)grid * D.n_out[l] * (D.n_in[l] + 1 + (l == 0 ? p.ng0 : 0)) * 8);
    }
  }
  p.bytes = o;
  return PINN_OK;
}

int hip_rc(hipError_t e) { return e == hipSuccess ? PINN_OK : PINN_E_HIP; }

// ---------------------------------------------------------------- optional event timing
struct TimedLaunch {
  const char* name;
  hipEvent_t start, stop;
};
struct Timing {
  std::mutex mu;
  bool on = false;
  std::vector<TimedLaunch> rec;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Timing& timing() {
  static Timing t;
  return t;
}

// Launch through f(), bracketed by events when timing is enabled (and allowed: the
// allocation-free entry point creates no events).
template <typename F>
int timed(bool allow, const char* name, hipStream_t s, F f) {
  Timing& T = timing();
  if (!T.on || !allow) return f();
  std::lock_guard<std::mutex> lk(T.mu);
  TimedLaunch tl{name, T.get(), T.get()};
  if (!tl.start || !tl.stop) return PINN_E_HIP;
  if (hipEventRecord(tl.start, s) != hipSuccess) return PINN_E_HIP;
  int rc = f();
  if (hipEventRecord(tl.stop, s) != hipSuccess) return PINN_E_HIP;
  T.rec.push_back(tl);
  return rc;
}

NetDev make_netdev(const pinn_net* net, const pinn_pde* pde, const Plan& p, char* ws, const float* B) {
  NetDev nd;
  std::memset(&nd, 0, sizeof(nd));
  const Dims& D = p.D;
  nd.L = D.L;
  nd.d_in = D.d_in;
  nd.d_out = D.d_out;
  nd.e = D.e;
  nd.n_freq = net->n_freq;
  nd.periodic_mask = net->periodic_mask;
  nd.omega = reinterpret_cast<const float*>(ws + p.o_omega);
  nd.lap_mask = pde->lap_mask;
  nd.lapch = pde->lap_mask ? 1 + D.d_in : -1;
  nd.w0 = net->w0;
  nd.B = B;
  for (int l = 0; l < D.n_layers; ++l) {
    LayerDev& L = nd.layer[l];
    L.n_in = D.n_in[l];
    L.n_out = D.n_out[l];
    L.nbo = (D.n_out[l] + 15) / 16;
    L.kci = (D.n_in[l] + 31) / 32;
    L.nbi = (D.n_in[l] + 15) / 16;
    L.kco = (D.n_out[l] + 31) / 32;
    L.wf = ws + p.o_wf[l];
    L.wb = ws + p.o_wb[l];
    L.w = reinterpret_cast<const float*>(ws + p.o_w[l]);
    L.b = reinterpret_cast<const float*>(ws + p.o_b[l]);
  }
  return nd;
}

// ---------------------------------------------------------------- FP64 precision

// What the FP64 kernels take: any width, n_hidden 0..8 (a linear read-out of the
// embedding), the same channel rules as the other precisions.
struct Plan64 {
  Dims D;
  int n_res, n_seg, ng;
  int64_t seg_start[1 + kMaxAnchors], seg_n[1 + kMaxAnchors];
  int64_t n_pad;
  int blocks;
  bool with_grad;
  int64_t o_pts, o_w[kMaxLayers], o_b[kMaxLayers], o_omega, o_a[kMaxLayers], o_z[kMaxHidden], o_zb[kMaxHidden],
      o_ab[2], o_yb, o_dw, o_loss, o_slot[kMaxLayers];
  int64_t bytes;
};

int make_plan64(const pinn_net* net, const pinn_pde* pde, int64_t n_points, const pinn_anchor* anchors, int n_anchor,
                int with_grad, Plan64* P) {
  Plan64& p = *P;
  std::memset(&p, 0, sizeof(p));
  int rc = check_net(net, &p.D);
  if (rc) return rc;
  rc = check_pde(net, pde);
  if (rc) return rc;
  if (n_points < 0 || n_anchor < 0 || n_anchor > kMaxAnchors) return PINN_E_INVALID;
  if (n_anchor > 0 && !anchors) return PINN_E_INVALID;
  int64_t tot = n_points;
  for (int a = 0; a < n_anchor; ++a) {
    if (anchors[a].n < 0 || !std::isfinite(anchors[a].lambda) || anchors[a].lambda < 0) return PINN_E_INVALID;
    if (anchors[a].out_mask <= 0 || anchors[a].out_mask >= (1 << net->d_out)) return PINN_E_INVALID;
    tot += anchors[a].n;
  }
  if (tot == 0) return PINN_E_INVALID;
  const Dims& D = p.D;
  for (int l = 0; l < D.L; ++l)
    if (D.n_out[l] > 256) return PINN_E_UNSUPPORTED;
  if (1 + net->d_in + (pde->lap_mask ? 1 : 0) > 4) return PINN_E_UNSUPPORTED;
  if (pde->lap_mask && net->d_in != 2) return PINN_E_UNSUPPORTED;
  if (net->periodic_mask && net->n_freq > 0) return PINN_E_UNSUPPORTED;
  if (net->n_freq > 4096) return PINN_E_UNSUPPORTED;
  p.n_res = n_res_of(pde->pde_id);
  p.n_seg = 1 + n_anchor;
  p.ng = 2 * D.n_tp;
  p.with_grad = with_grad != 0;
  int64_t cur = 0;
  for (int s = 0; s < p.n_seg; ++s) {
    p.seg_start[s] = cur;
    p.seg_n[s] = s == 0 ? n_points : anchors[s - 1].n;
    cur += align_up(std::max<int64_t>(p.seg_n[s], 1), kSegAlign);
  }
  p.n_pad = cur;
  p.blocks = (int)((p.n_pad + 255) / 256);
  int64_t o = 0;
  auto take = [&](int64_t bytes) { int64_t r = o; o = align_up(o + bytes, kAlign); return r; };
  const int64_t col = p.n_pad * 4 * 8;  // one jet row over all points
  p.o_pts = take(p.n_pad * 16);
  for (int l = 0; l < D.n_layers; ++l) {
    p.o_w[l] = take((int64_t)D.n_out[l] * D.n_in[l] * 8);
    p.o_b[l] = take((int64_t)D.n_out[l] * 8);
  }
  p.o_omega = take(32);
  for (int l = 0; l < D.n_layers; ++l) p.o_a[l] = take(col * D.n_in[l]);
  int wmax = D.e;
  for (int l = 0; l < D.L; ++l) {
    p.o_z[l] = take(col * D.n_out[l]);
    wmax = std::max(wmax, D.n_out[l]);
  }
  p.o_yb = take(col * D.d_out);
  p.o_dw = take(col * std::max(p.ng, 1));
  p.o_loss = take((int64_t)p.blocks * kMaxTerms * 8);
  if (p.with_grad) {
    for (int l = 0; l < D.L; ++l) p.o_zb[l] = take(col * D.n_out[l]);
    p.o_ab[0] = take(col * wmax);
    p.o_ab[1] = take(col * wmax);
    for (int l = 0; l < D.n_layers; ++l)
      p.o_slot[l] = take((int64_t)D.n_out[l] * (D.n_in[l] + 1 + (l == 0 ? p.ng : 0)) * 8);
  }
  p.bytes = o;
  return PINN_OK;
}

int run_fp64(const pinn_net* net, const pinn_pde* pde, const float* params, const float* B, const float* points,
             int64_t n_points, const pinn_anchor* anchors, int n_anchor, uint32_t flags, float* residual,
             double* loss, double* grad, void* workspace, size_t ws_bytes, hipStream_t stream, bool with_grad,
             const double* wscale, bool accumulate) {
  Plan64 p;
  int rc = make_plan64(net, pde, n_points, anchors, n_anchor, with_grad, &p);
  if (rc) return rc;
  if (!params || !loss || !workspace || (n_points > 0 && !points)) return PINN_E_INVALID;
  if (with_grad && !grad) return PINN_E_INVALID;
  if (net->n_freq > 0 && !B) return PINN_E_INVALID;
  for (int a = 0; a < n_anchor; ++a)
    if (anchors[a].n > 0 && (!anchors[a].points || !anchors[a].targets)) return PINN_E_INVALID;
  if ((int64_t)ws_bytes < p.bytes) return PINN_E_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return PINN_E_INVALID;
  char* ws = static_cast<char*>(workspace);
  const Dims& D = p.D;
  if (flags & PINN_FLAG_CHECK_FINITE) {
    int* flag = reinterpret_cast<int*>(ws + p.o_loss);  // scratch before the loss slots are written
    rc = launch_check_finite(params, D.n_params, flag, stream);
    if (rc) return rc;
    int h = 0;
    if (hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess) return PINN_E_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return PINN_E_HIP;
    if (h) return PINN_E_NONFINITE;
  }
  {
    PointsArgs a;
    std::memset(&a, 0, sizeof(a));
    a.d_in = D.d_in;
    a.n_seg = p.n_seg;
    for (int s = 0; s < p.n_seg; ++s) {
      a.start[s] = p.seg_start[s];
      a.n[s] = p.seg_n[s];
      a.src[s] = s == 0 ? points : anchors[s - 1].points;
    }
    a.n_pad = p.n_pad;
    a.dst = reinterpret_cast<float4*>(ws + p.o_pts);
    rc = launch_points(a, stream);
    if (rc) return rc;
  }
  F64StageArgs st;
  std::memset(&st, 0, sizeof(st));
  st.n_layers = D.n_layers;
  st.rwf = net->rwf;
  st.has_bias = net->has_bias;
  st.periodic_mask = net->periodic_mask;
  st.period_train_mask = net->period_train_mask;
  for (int k = 0; k < 3; ++k) st.period[k] = net->period[k];
  st.off_p = D.off_p;
  st.params = params;
  st.omega = reinterpret_cast<double*>(ws + p.o_omega);
  F64Args a;
  std::memset(&a, 0, sizeof(a));
  a.n_pad = p.n_pad;
  a.L = D.L;
  a.d_in = D.d_in;
  a.d_out = D.d_out;
  a.e = D.e;
  a.n_freq = net->n_freq;
  a.act = net->act;
  a.periodic_mask = net->periodic_mask;
  a.period_train_mask = net->period_train_mask;
  a.lap_mask = pde->lap_mask;
  a.lapch = pde->lap_mask ? 1 + D.d_in : -1;
  a.ng = p.ng;
  a.w0 = (double)net->w0;
  for (int l = 0; l < D.n_layers; ++l) {
    st.off_w[l] = D.off_w[l];
    st.off_s[l] = D.off_s[l];
    st.off_b[l] = D.off_b[l];
    st.n_in[l] = a.n_in[l] = D.n_in[l];
    st.n_out[l] = a.n_out[l] = D.n_out[l];
    st.w[l] = reinterpret_cast<double*>(ws + p.o_w[l]);
    st.b[l] = reinterpret_cast<double*>(ws + p.o_b[l]);
    a.w[l] = st.w[l];
    a.b[l] = st.b[l];
    a.a[l] = reinterpret_cast<double*>(ws + p.o_a[l]);
  }
  for (int l = 0; l < D.L; ++l) {
    a.z[l] = reinterpret_cast<double*>(ws + p.o_z[l]);
    if (p.with_grad) a.zb[l] = reinterpret_cast<double*>(ws + p.o_zb[l]);
  }
  if (p.with_grad) {
    a.ab[0] = reinterpret_cast<double*>(ws + p.o_ab[0]);
    a.ab[1] = reinterpret_cast<double*>(ws + p.o_ab[1]);
  }
  a.yb = reinterpret_cast<double*>(ws + p.o_yb);
  a.dw = reinterpret_cast<double*>(ws + p.o_dw);
  a.omega = st.omega;
  a.B = B;
  a.pts = reinterpret_cast<const float4*>(ws + p.o_pts);
  a.pde_id = pde->pde_id;
  a.n_res = p.n_res;
  for (int k = 0; k < 4; ++k) a.coef[k] = pde->coef[k];
  const double N = pde->norm_N > 0 ? pde->norm_N : (double)n_points;
  for (int k = 0; k < kMaxOut; ++k) a.seed[k] = N > 0 ? 2.0 * pde->lambda_res[k] / N : 0.0;
  for (int k = 0; k < n_anchor; ++k)
    a.lam_anchor[k] = anchors[k].n > 0 ? 2.0 * anchors[k].lambda / (double)anchors[k].n : 0.0;
  a.wscale = wscale;
  a.seg.n_seg = p.n_seg;
  for (int s = 0; s < p.n_seg; ++s) {
    a.seg.start[s] = p.seg_start[s];
    a.seg.n[s] = p.seg_n[s];
  }
  for (int k = 0; k < n_anchor; ++k) {
    a.seg.targets[k] = anchors[k].targets;
    a.seg.out_mask[k] = anchors[k].out_mask;
  }
  a.residual = residual;
  a.loss_slots = reinterpret_cast<double*>(ws + p.o_loss);
  double* slots[kMaxLayers] = {};
  for (int l = 0; l < D.n_layers; ++l) slots[l] = p.with_grad ? reinterpret_cast<double*>(ws + p.o_slot[l]) : nullptr;
  rc = launch_fp64(st, a, p.with_grad ? slots : nullptr, stream);
  if (rc) return rc;
  if (p.with_grad) {
    for (int l = 0; l < D.n_layers; ++l) {
      ReduceArgs r;
      std::memset(&r, 0, sizeof(r));
      r.slots = slots[l];
      r.n_slots = 1;
      r.slot_stride = (int64_t)D.n_out[l] * (D.n_in[l] + 1 + (l == 0 ? p.ng : 0));
      r.n_out = D.n_out[l];
      r.n_in = D.n_in[l];
      r.rwf = net->rwf;
      r.has_bias = net->has_bias;
      r.params = params;
      r.off_w = D.off_w[l];
      r.off_s = D.off_s[l];
      r.off_b = D.off_b[l];
      r.grad = grad;
      r.accumulate = accumulate;
      rc = launch_reduce_layer(r, stream);
      if (rc) return rc;
    }
    if (D.n_tp > 0) {
      PeriodReduceArgs r;
      std::memset(&r, 0, sizeof(r));
      r.slots = slots[0];
      r.n_slots = 1;
      r.slot_stride = (int64_t)D.n_out[0] * (D.e + 1 + p.ng);
      r.n_out = D.n_out[0];
      r.e = D.e;
      r.periodic_mask = net->periodic_mask;
      r.period_train_mask = net->period_train_mask;
      r.d_in = D.d_in;
      r.w64 = a.w[0];
      r.omega64 = a.omega;
      r.grad = grad;
      r.off_p = D.off_p;
      r.accumulate = accumulate;
      rc = launch_reduce_period(r, stream);
      if (rc) return rc;
    }
  }
  {
    LossArgs l;
    std::memset(&l, 0, sizeof(l));
    l.slots = a.loss_slots;
    l.n_slots = p.blocks;
    l.n_res = p.n_res;
    l.n_anchor = n_anchor;
    for (int k = 0; k < kMaxOut; ++k) l.w_res[k] = N > 0 ? pde->lambda_res[k] / N : 0.0;
    for (int k = 0; k < n_anchor; ++k) l.w_anchor[k] = anchors[k].n > 0 ? anchors[k].lambda / (double)anchors[k].n : 0.0;
    l.loss = loss;
    l.wscale = wscale;
    l.accumulate = accumulate;
    rc = launch_reduce_loss(l, stream);
    if (rc) return rc;
  }
  return hip_rc(hipGetLastError());
}

// Workspace bytes of either kind of plan.
int plan_bytes(const pinn_net* net, const pinn_pde* pde, int64_t n_points, const pinn_anchor* anchors, int n_anchor,
               int prec, int with_grad, const pinn_tune* tune, int64_t* bytes) {
  if (prec == PINN_PREC_FP64) {
    Plan64 p;
    int rc = make_plan64(net, pde, n_points, anchors, n_anchor, with_grad, &p);
    if (rc) return rc;
    *bytes = p.bytes;
    return PINN_OK;
  }
  Plan p;
  int rc = make_plan(net, pde, n_points, anchors, n_anchor, prec, with_grad, tune, &p);
  if (rc) return rc;
  *bytes = p.bytes;
  return PINN_OK;
}

int run(const pinn_net* net, const pinn_pde* pde, const float* params, const float* B, const float* points,
        int64_t n_points, const pinn_anchor* anchors, int n_anchor, int prec, uint32_t flags,
        const pinn_tune* tune, float* residual, double* loss, double* grad, void* workspace,
        size_t ws_bytes, pinn_stream_t stream_, bool with_grad, bool allow_timing = true,
        const double* wscale = nullptr, bool accumulate = false) {
  if (prec == PINN_PREC_FP64)
    return run_fp64(net, pde, params, B, points, n_points, anchors, n_anchor, flags, residual, loss, grad, workspace,
                    ws_bytes, reinterpret_cast<hipStream_t>(stream_), with_grad, wscale, accumulate);
  Plan p;
  int rc = make_plan(net, pde, n_points, anchors, n_anchor, prec, with_grad, tune, &p);
  if (rc) return rc;
  if (!params || !loss || !workspace || (n_points > 0 && !points)) return PINN_E_INVALID;
  if (with_grad && !grad) return PINN_E_INVALID;
  if (net->n_freq > 0 && !B) return PINN_E_INVALID;
  for (int a = 0; a < n_anchor; ++a)
    if (anchors[a].n > 0 && (!anchors[a].points || !anchors[a].targets)) return PINN_E_INVALID;
  if ((int64_t)ws_bytes < p.bytes) return PINN_E_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return PINN_E_INVALID;
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  char* ws = static_cast<char*>(workspace);
  const Dims& D = p.D;

  if (flags & PINN_FLAG_CHECK_FINITE) {
    int* flag = reinterpret_cast<int*>(ws + p.o_flag);
    rc = timed(allow_timing, "k_check_finite", stream, [&] { return launch_check_finite(params, D.n_params, flag, stream); });
    if (rc) return rc;
    int h = 0;
    if (hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess) return PINN_E_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return PINN_E_HIP;
    if (h) return PINN_E_NONFINITE;
  }

  // points and weights (one launch)
  {
    PointsArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.d_in = D.d_in;
    pa.n_seg = p.n_seg;
    for (int s = 0; s < p.n_seg; ++s) {
      pa.start[s] = p.seg_start[s];
      pa.n[s] = p.seg_n[s];
      pa.src[s] = s == 0 ? points : anchors[s - 1].points;
    }
    pa.n_pad = p.n_pad;
    pa.dst = reinterpret_cast<float4*>(ws + p.o_pts);
    pa.zero = reinterpret_cast<unsigned int*>(ws + p.o_amax);
    pa.n_zero = kMaxHidden;
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n_layers = D.n_layers;
    a.rwf = net->rwf;
    a.has_bias = net->has_bias;
    a.periodic_mask = net->periodic_mask;
    a.period_train_mask = net->period_train_mask;
    for (int k = 0; k < 3; ++k) a.period[k] = net->period[k];
    a.off_p = D.off_p;
    a.omega = reinterpret_cast<float*>(ws + p.o_omega);
    a.params = params;
    int64_t cum = 0;
    for (int l = 0; l < D.n_layers; ++l) {
      a.off_w[l] = D.off_w[l];
      a.off_s[l] = D.off_s[l];
      a.off_b[l] = D.off_b[l];
      a.n_in[l] = D.n_in[l];
      a.n_out[l] = D.n_out[l];
      a.wf[l] = ws + p.o_wf[l];
      a.wb[l] = ws + p.o_wb[l];
      a.w[l] = reinterpret_cast<float*>(ws + p.o_w[l]);
      a.b[l] = reinterpret_cast<float*>(ws + p.o_b[l]);
      const int64_t nbo = (D.n_out[l] + 15) / 16, kci = (D.n_in[l] + 31) / 32;
      const int64_t nbi = (D.n_in[l] + 15) / 16, kco = (D.n_out[l] + 31) / 32;
      a.cum[l] = cum;
      cum += nbo * kci * 64 + nbi * kco * 64 + (int64_t)D.n_out[l] * D.n_in[l] + D.n_out[l];
    }
    a.cum[D.n_layers] = cum;
    rc = timed(allow_timing, "k_prepare", stream, [&] { return launch_prepare(p.prec, pa, a, stream); });
    if (rc) return rc;
  }

  const NetDev nd = make_netdev(net, pde, p, ws, B);
  Work wk;
  std::memset(&wk, 0, sizeof(wk));
  wk.n_pad = p.n_pad;
  wk.pts = reinterpret_cast<const float4*>(ws + p.o_pts);
  wk.loss_slots = reinterpret_cast<double*>(ws + p.o_loss);
  wk.amax = reinterpret_cast<unsigned int*>(ws + p.o_amax);
  if (p.with_grad) {
    wk.zs0 = reinterpret_cast<float*>(ws + p.o_zs[0]);
    wk.zs_stride = p.zs_stride;
    wk.zb[0] = reinterpret_cast<float*>(ws + p.o_zb[0]);
    wk.zb[1] = reinterpret_cast<float*>(ws + p.o_zb[1]);
    wk.out_slots = reinterpret_cast<double*>(ws + p.o_out);
    for (int l = 0; l < D.L; ++l) wk.layer_slots[l] = reinterpret_cast<double*>(ws + p.o_layer[l]);
  }
  const double N = pde->norm_N > 0 ? pde->norm_N : (double)n_points;
  {
    FwdArgs a;
    std::memset(&a, 0, sizeof(a));
    a.net = nd;
    a.pde.pde_id = pde->pde_id;
    a.pde.n_res = p.n_res;
    for (int k = 0; k < 4; ++k) a.pde.coef[k] = (float)pde->coef[k];
    for (int k = 0; k < kMaxOut; ++k) a.pde.seed_scale[k] = N > 0 ? (float)(2.0 * pde->lambda_res[k] / N) : 0.0f;
    a.seg.n_seg = p.n_seg;
    for (int s = 0; s < p.n_seg; ++s) {
      a.seg.start[s] = p.seg_start[s];
      a.seg.n[s] = p.seg_n[s];
    }
    for (int k = 0; k < n_anchor; ++k) {
      a.seg.targets[k] = anchors[k].targets;
      a.seg.out_mask[k] = anchors[k].out_mask;
      a.seg.lam_anchor[k] = anchors[k].n > 0 ? (float)(2.0 * anchors[k].lambda / (double)anchors[k].n) : 0.0f;
    }
    a.work = wk;
    a.n_tiles = p.n_tiles;
    a.kmax = p.kmax;
    a.with_grad = p.with_grad;
    a.residual = residual;
    a.wscale = wscale;
    rc = timed(allow_timing, "k_forward", stream, [&] { return launch_forward(p.prec, act_code(net, pde), D.H, p.pf, a, p.grid_f, p.lds_f, stream); });
    if (rc) return rc;
  }
  int cur = 0;
  // every layer's slot reduction and the loss terms: one launch after the backward
  ReduceAllArgs ra;
  std::memset(&ra, 0, sizeof(ra));
  if (p.with_grad) {
    for (int j = D.L - 1; j >= 1; --j) {
      BwdArgs a;
      std::memset(&a, 0, sizeof(a));
      a.net = nd;
      a.work = wk;
      a.layer = j;
      a.n_sub = p.n_sub;
      a.zb_in = wk.zb[cur];
      a.zb_out = wk.zb[cur ^ 1];
      a.z_prev = wk.zs0 + (j - 1) * wk.zs_stride;
      a.slots = wk.layer_slots[j];
      a.wide = p.split ? 2 : p.wide;
      a.pb = p.pb;
      if (j == 1 && p.fuse0) a.g0_slots = wk.layer_slots[0];
      a.pace = reinterpret_cast<unsigned long long*>(ws + p.o_pace);
      a.launch = next_launch_id();
      rc = timed(allow_timing, "k_backward", stream, [&] { return launch_backward(p.prec, act_code(net, pde), D.H, false, a, p.grid_b, p.lds_b, stream); });
      if (rc) return rc;
      cur ^= 1;
    }
    if (net->n_freq > 0) {
      BwdArgs a;
      std::memset(&a, 0, sizeof(a));
      a.net = nd;
      a.work = wk;
      a.layer = 0;
      a.n_sub = p.n_sub0;
      a.zb_in = wk.zb[cur];
      a.zb_out = nullptr;
      a.z_prev = nullptr;
      a.slots = wk.layer_slots[0];
      a.wide = p.wide0 ? (D.n_out[0] == D.H && D.H >= 64 ? 3 : 1) : 0;
      rc = timed(allow_timing, "k_backward_embed", stream, [&] { return launch_backward(p.prec, act_code(net, pde), D.H, true, a, p.grid_b0, p.lds_b0, stream); });
      if (rc) return rc;
    } else if (!p.fuse0) {
      Grad0Args a;
      std::memset(&a, 0, sizeof(a));
      a.zb = wk.zb[cur];
      a.pts = wk.pts;
      a.n_out = D.n_out[0];
      a.d_in = D.d_in;
      a.n_cb = p.n_pad / 4;
      a.slots = wk.layer_slots[0];
      a.periodic_mask = net->periodic_mask;
      a.period_train_mask = net->period_train_mask;
      a.lap_mask = pde->lap_mask;
      a.e = D.e;
      a.omega = reinterpret_cast<const float*>(ws + p.o_omega);
      rc = timed(allow_timing, "k_grad0", stream, [&] { return launch_grad0(a, p.grid_g0, stream); });
      if (rc) return rc;
    }
    for (int l = 0; l < D.n_layers; ++l) {
      ReduceArgs& a = ra.layer[l];
      a.accumulate = accumulate;
      a.n_out = D.n_out[l];
      a.n_in = D.n_in[l];
      a.rwf = net->rwf;
      a.has_bias = net->has_bias;
      a.params = params;
      a.off_w = D.off_w[l];
      a.off_s = D.off_s[l];
      a.off_b = D.off_b[l];
      a.grad = grad;
      a.slot_stride = (int64_t)D.n_out[l] * (D.n_in[l] + 1 + (l == 0 ? p.ng0 : 0));
      if (l == D.L) {
        a.slots = wk.out_slots;
        a.n_slots = p.grid_f;
      } else {
        a.slots = wk.layer_slots[l];
        a.n_slots = l == 0 ? (net->n_freq > 0 ? p.grid_b0 : (p.fuse0 ? fused0_slots(p) : p.grid_g0))
                           : (p.split ? p.grid_b / 2 : p.grid_b);
      }
      ra.row0[l + 1] = ra.row0[l] + D.n_out[l];
    }
    ra.n_layers = D.n_layers;
  }
  {
    LossArgs& a = ra.loss;
    a.slots = wk.loss_slots;
    a.n_slots = p.grid_f;
    a.n_res = p.n_res;
    a.n_anchor = n_anchor;
    for (int k = 0; k < kMaxOut; ++k) a.w_res[k] = N > 0 ? pde->lambda_res[k] / N : 0.0;
    for (int k = 0; k < n_anchor; ++k)
      a.w_anchor[k] = anchors[k].n > 0 ? anchors[k].lambda / (double)anchors[k].n : 0.0;
    a.loss = loss;
    a.wscale = wscale;
    a.accumulate = accumulate;
    rc = timed(allow_timing, "k_reduce", stream, [&] { return launch_reduce_all(ra, stream); });
    if (rc) return rc;
  }
  if (p.with_grad) {
    if (D.n_tp > 0) {  // trained periods of the periodic embedding (from layer 0's slots)
      PeriodReduceArgs a;
      std::memset(&a, 0, sizeof(a));
      a.slots = wk.layer_slots[0];
      a.n_slots = p.grid_g0;
      a.slot_stride = (int64_t)D.n_out[0] * (D.e + 1 + p.ng0);
      a.n_out = D.n_out[0];
      a.e = D.e;
      a.periodic_mask = net->periodic_mask;
      a.period_train_mask = net->period_train_mask;
      a.d_in = D.d_in;
      a.w = reinterpret_cast<const float*>(ws + p.o_w[0]);
      a.omega = reinterpret_cast<const float*>(ws + p.o_omega);
      a.grad = grad;
      a.off_p = D.off_p;
      a.accumulate = accumulate;
      rc = timed(allow_timing, "k_reduce_period", stream, [&] { return launch_reduce_period(a, stream); });
      if (rc) return rc;
    }
  }
  return hip_rc(hipGetLastError());
}


// ---------------------------------------------------------------- many networks, one launch

struct BatchPlan {
  int n_inst, prec, act, n_res, n_items, grid;
  std::vector<Dims> D;
  std::vector<int64_t> chunk, pts_off, n_pad, item0, n_items_of, n_eff, slot_base;
  std::vector<int> kmax;
  std::vector<char> sep;   // instance runs as a fused step of its own (chunk_points == -1)
  int64_t o_sep, sep_bytes;
  std::vector<BatchItem> items;
  std::vector<int64_t> order;
  int64_t n_pad_all, scratch_per_wg, n_slot_doubles;
  size_t lds;
  // workspace offsets
  int64_t o_pts, o_tables, tables_bytes, o_counter, o_loss, o_grad, o_scratch;
  std::vector<int64_t> o_wf[kMaxLayers], o_wb[kMaxLayers], o_w[kMaxLayers], o_b[kMaxLayers];
  int64_t bytes;
};

int default_chunk(int H) { return H == 256 ? 1024 : H == 128 ? 2048 : 4096; }

int make_batch_plan(const pinn_net* nets, const pinn_pde* pde, const int64_t* n_points, int n_inst, int prec,
                    const pinn_tune* tune, BatchPlan* out) {
  BatchPlan& b = *out;
  if (!nets || !pde || !n_points || n_inst <= 0 || n_inst > 65536) return PINN_E_INVALID;
  int kp = 0;
  const int prc = kernel_prec(prec, &kp);
  if (prc) return prc;
  b.n_inst = n_inst;
  b.prec = kp;
  b.act = nets[0].act;
  b.D.resize(n_inst);
  b.chunk.resize(n_inst);
  b.kmax.resize(n_inst);
  b.sep.assign(n_inst, 0);
  b.sep_bytes = 0;
  for (int i = 0; i < n_inst; ++i) {
    int rc = check_net(&nets[i], &b.D[i]);
    if (rc) return rc;
    rc = check_pde(&nets[i], pde);
    if (rc) return rc;
    rc = check_supported(&nets[i], b.D[i], pde->lap_mask);
    if (rc) return rc;
    if (nets[i].n_freq != 0 || nets[i].periodic_mask != 0 || nets[i].act != b.act || nets[i].d_in != nets[0].d_in ||
        nets[i].d_out != nets[0].d_out)
      return PINN_E_UNSUPPORTED;
    if (n_points[i] <= 0) return PINN_E_INVALID;
    int c = default_chunk(b.D[i].H);
    if (tune && tune[i].chunk_points == -1) {
      b.sep[i] = 1;
      pinn_pde pd = *pde;
      pd.norm_N = 0.0;  // the mean over the instance's own points
      int64_t sb = 0;
      rc = plan_bytes(&nets[i], &pd, n_points[i], nullptr, 0, prec, 1, nullptr, &sb);
      if (rc) return rc;
      b.sep_bytes = std::max(b.sep_bytes, sb);
    } else if (tune && tune[i].chunk_points != 0) {
      if (tune[i].chunk_points < 0 || tune[i].chunk_points % kSegAlign) return PINN_E_INVALID;
      c = tune[i].chunk_points;
    }
    if (tune && tune[i].tile_points > 0 && tune[i].tile_points != default_fwd_p(b.D[i].H)) return PINN_E_UNSUPPORTED;
    b.chunk[i] = c;
    b.kmax[i] = (int)align_up(std::max(b.D[i].e, b.D[i].hmax), 32);
  }
  b.n_res = n_res_of(pde->pde_id);
  // points, items, slots
  b.pts_off.resize(n_inst);
  b.n_pad.resize(n_inst);
  b.item0.resize(n_inst);
  b.n_items_of.resize(n_inst);
  b.n_eff.resize(n_inst);
  b.slot_base.resize(n_inst);
  int64_t pts = 0, slots = 0;
  b.items.clear();
  b.scratch_per_wg = 0;
  b.lds = 0;
  std::vector<double> cost;
  for (int i = 0; i < n_inst; ++i) {
    const Dims& D = b.D[i];
    b.pts_off[i] = pts;
    b.n_pad[i] = align_up(n_points[i], kSegAlign);
    pts += b.n_pad[i];
    int64_t ne = 0, flops = 0;
    for (int l = 0; l < D.n_layers; ++l) {
      ne += (int64_t)D.n_out[l] * (D.n_in[l] + 1);
      flops += (int64_t)D.n_out[l] * D.n_in[l];
    }
    b.n_eff[i] = ne;
    b.item0[i] = (int64_t)b.items.size();
    b.slot_base[i] = slots;
    b.n_items_of[i] = 0;
    if (b.sep[i]) continue;
    for (int64_t p0 = 0; p0 < b.n_pad[i]; p0 += b.chunk[i]) {
      BatchItem it;
      it.inst = i;
      it.p0 = p0;
      it.p1 = std::min<int64_t>(p0 + b.chunk[i], b.n_pad[i]);
      it.slot_off = slots;
      slots += ne;
      b.items.push_back(it);
      cost.push_back((double)(it.p1 - it.p0) * (double)flops);
    }
    b.n_items_of[i] = (int64_t)b.items.size() - b.item0[i];
    const int64_t stride = b.chunk[i] * 4 * D.hmax;
    b.scratch_per_wg = std::max<int64_t>(b.scratch_per_wg, stride * (D.L + 2));
    b.lds = std::max(b.lds, batched_lds(b.kmax[i], D.H));
  }
  if (b.lds > kLdsBudget) return PINN_E_UNSUPPORTED;
  b.n_pad_all = pts;
  b.n_slot_doubles = slots;
  b.n_items = (int)b.items.size();
  b.order.resize(b.n_items);
  for (int q = 0; q < b.n_items; ++q) b.order[q] = q;
  std::stable_sort(b.order.begin(), b.order.end(), [&](int64_t x, int64_t y) { return cost[x] > cost[y]; });
  b.grid = std::min(b.n_items, (tune && tune[0].grid > 0) ? tune[0].grid : kGridCap);
  // workspace
  int64_t o = 0;
  auto take = [&](int64_t bytes) { int64_t r = o; o = align_up(o + bytes, kAlign); return r; };
  b.o_pts = take(b.n_pad_all * 16);
  for (int l = 0; l < kMaxLayers; ++l) {
    b.o_wf[l].assign(n_inst, 0);
    b.o_wb[l].assign(n_inst, 0);
    b.o_w[l].assign(n_inst, 0);
    b.o_b[l].assign(n_inst, 0);
  }
  for (int i = 0; i < n_inst; ++i) {
    const Dims& D = b.D[i];
    for (int l = 0; l < D.n_layers; ++l) {
      const int64_t nbo = (D.n_out[l] + 15) / 16, kci = (D.n_in[l] + 31) / 32;
      const int64_t nbi = (D.n_in[l] + 15) / 16, kco = (D.n_out[l] + 31) / 32;
      b.o_wf[l][i] = take(nbo * kci * 64 * 32);
      b.o_wb[l][i] = take(nbi * kco * 64 * 32);
      b.o_w[l][i] = take((int64_t)D.n_out[l] * D.n_in[l] * 4);
      b.o_b[l][i] = take((int64_t)D.n_out[l] * 4);
    }
  }
  int64_t n_rows_entries = 0;
  for (int i = 0; i < n_inst; ++i) n_rows_entries += b.D[i].n_layers;
  b.tables_bytes = (int64_t)sizeof(BatchInst) * n_inst + (int64_t)sizeof(BatchItem) * b.n_items +
                   (int64_t)sizeof(int64_t) * b.n_items + (int64_t)sizeof(BatchRow) * n_rows_entries +
                   (int64_t)n_inst * (sizeof(int64_t) + sizeof(int) + kMaxOut * sizeof(double)) + 64 * 8;
  b.o_tables = take(b.tables_bytes);
  b.o_counter = take(16);
  b.o_loss = take((int64_t)b.n_items * kMaxTerms * 8);
  b.o_grad = take(b.n_slot_doubles * 8);
  b.o_scratch = take(b.scratch_per_wg * 4 * b.grid);
  b.o_sep = take(b.sep_bytes);
  b.bytes = o;
  return PINN_OK;
}

int run_batched(const pinn_net* nets, const pinn_pde* pde, const float* const* params, const float* const* points,
                const int64_t* n_points, int n_inst, int prec, const pinn_tune* tune, double* const* grads,
                double* losses, void* workspace, size_t ws_bytes, pinn_stream_t stream_) {
  const bool allow_timing = true;
  BatchPlan b;
  int rc = make_batch_plan(nets, pde, n_points, n_inst, prec, tune, &b);
  if (rc) return rc;
  if (!params || !points || !grads || !losses || !workspace) return PINN_E_INVALID;
  for (int i = 0; i < n_inst; ++i)
    if (!params[i] || !points[i] || !grads[i]) return PINN_E_INVALID;
  if ((int64_t)ws_bytes < b.bytes) return PINN_E_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return PINN_E_INVALID;
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  char* ws = static_cast<char*>(workspace);

  // host tables, uploaded in one copy
  std::vector<char> host((size_t)b.tables_bytes, 0);
  char* hp = host.data();
  BatchInst* hinst = reinterpret_cast<BatchInst*>(hp);
  BatchItem* hitems = reinterpret_cast<BatchItem*>(hinst + n_inst);
  int64_t* horder = reinterpret_cast<int64_t*>(hitems + b.n_items);
  BatchRow* hrows = reinterpret_cast<BatchRow*>(horder + b.n_items);
  int64_t n_entries = 0;
  for (int i = 0; i < n_inst; ++i) n_entries += b.D[i].n_layers;
  int64_t* hitem0 = reinterpret_cast<int64_t*>(hrows + n_entries);
  int* hnitems = reinterpret_cast<int*>(hitem0 + n_inst);
  double* hw = reinterpret_cast<double*>(
      reinterpret_cast<char*>(hnitems) + align_up((int64_t)n_inst * sizeof(int), 8));
  char* dbase = ws + b.o_tables;
  auto dev = [&](const void* hptr) { return dbase + (static_cast<const char*>(hptr) - hp); };

  int64_t row0 = 0;
  int64_t entry = 0;
  for (int i = 0; i < n_inst; ++i) {
    const Dims& D = b.D[i];
    BatchInst& in = hinst[i];
    std::memset(&in, 0, sizeof(in));
    NetDev& nd = in.net;
    nd.L = D.L;
    nd.d_in = D.d_in;
    nd.d_out = D.d_out;
    nd.e = D.e;
    nd.n_freq = 0;
    nd.lap_mask = pde->lap_mask;
    nd.lapch = pde->lap_mask ? 1 + D.d_in : -1;
    nd.w0 = nets[i].w0;
    nd.B = nullptr;
    for (int l = 0; l < D.n_layers; ++l) {
      LayerDev& L = nd.layer[l];
      L.n_in = D.n_in[l];
      L.n_out = D.n_out[l];
      L.nbo = (D.n_out[l] + 15) / 16;
      L.kci = (D.n_in[l] + 31) / 32;
      L.nbi = (D.n_in[l] + 15) / 16;
      L.kco = (D.n_out[l] + 31) / 32;
      L.wf = ws + b.o_wf[l][i];
      L.wb = ws + b.o_wb[l][i];
      L.w = reinterpret_cast<const float*>(ws + b.o_w[l][i]);
      L.b = reinterpret_cast<const float*>(ws + b.o_b[l][i]);
    }
    in.H = D.H;
    in.kmax = b.kmax[i];
    in.pts_off = b.pts_off[i];
    in.n = n_points[i];
    int64_t eo = 0;
    for (int l = 0; l < D.n_layers; ++l) {
      in.eff_off[l] = eo;
      eo += (int64_t)D.n_out[l] * (D.n_in[l] + 1);
    }
    in.zs_stride = b.chunk[i] * 4 * D.hmax;
    in.zb_off[0] = in.zs_stride * D.L;
    in.zb_off[1] = in.zs_stride * (D.L + 1);
    for (int l = 0; l < D.n_layers; ++l, ++entry) {
      BatchRow& r = hrows[entry];
      r.row0 = row0;
      row0 += D.n_out[l];
      r.slot0 = b.slot_base[i] + in.eff_off[l];
      r.slot_stride = b.n_eff[i];
      r.n_items = (int)b.n_items_of[i];
      r.n_out = D.n_out[l];
      r.n_in = D.n_in[l];
      r.rwf = nets[i].rwf;
      r.has_bias = nets[i].has_bias;
      r.params = params[i];
      r.off_w = D.off_w[l];
      r.off_s = D.off_s[l];
      r.off_b = D.off_b[l];
      r.grad = grads[i];
    }
    hitem0[i] = b.item0[i];
    hnitems[i] = (int)b.n_items_of[i];
    for (int k = 0; k < kMaxOut; ++k) hw[i * kMaxOut + k] = pde->lambda_res[k] / (double)n_points[i];
  }
  for (int q = 0; q < b.n_items; ++q) {
    hitems[q] = b.items[q];
    horder[q] = b.order[q];
  }
  if (hipMemcpyAsync(dbase, hp, host.size(), hipMemcpyHostToDevice, stream) != hipSuccess) return PINN_E_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return PINN_E_HIP;

  for (int i = 0; i < n_inst; ++i) {
    if (b.sep[i]) continue;
    const Dims& D = b.D[i];
    PointsArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.d_in = D.d_in;
    pa.n_seg = 1;
    pa.start[0] = 0;
    pa.n[0] = n_points[i];
    pa.src[0] = points[i];
    pa.n_pad = b.n_pad[i];
    pa.dst = reinterpret_cast<float4*>(ws + b.o_pts) + b.pts_off[i];
    StageArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.n_layers = D.n_layers;
    sa.rwf = nets[i].rwf;
    sa.has_bias = nets[i].has_bias;
    sa.params = params[i];
    int64_t cum = 0;
    for (int l = 0; l < D.n_layers; ++l) {
      sa.off_w[l] = D.off_w[l];
      sa.off_s[l] = D.off_s[l];
      sa.off_b[l] = D.off_b[l];
      sa.n_in[l] = D.n_in[l];
      sa.n_out[l] = D.n_out[l];
      sa.wf[l] = ws + b.o_wf[l][i];
      sa.wb[l] = ws + b.o_wb[l][i];
      sa.w[l] = reinterpret_cast<float*>(ws + b.o_w[l][i]);
      sa.b[l] = reinterpret_cast<float*>(ws + b.o_b[l][i]);
      const int64_t nbo = (D.n_out[l] + 15) / 16, kci = (D.n_in[l] + 31) / 32;
      const int64_t nbi = (D.n_in[l] + 15) / 16, kco = (D.n_out[l] + 31) / 32;
      sa.cum[l] = cum;
      cum += nbo * kci * 64 + nbi * kco * 64 + (int64_t)D.n_out[l] * D.n_in[l] + D.n_out[l];
    }
    sa.cum[D.n_layers] = cum;
    rc = timed(allow_timing, "k_prepare", stream, [&] { return launch_prepare(b.prec, pa, sa, stream); });
    if (rc) return rc;
  }
  int* counter = reinterpret_cast<int*>(ws + b.o_counter);
  BatchArgs ba;
  std::memset(&ba, 0, sizeof(ba));
  ba.inst = reinterpret_cast<const BatchInst*>(dev(hinst));
  ba.items = reinterpret_cast<const BatchItem*>(dev(hitems));
  ba.order = reinterpret_cast<const int64_t*>(dev(horder));
  ba.n_items = b.n_items;
  ba.counter = counter;
  ba.pde.pde_id = pde->pde_id;
  ba.pde.n_res = b.n_res;
  for (int k = 0; k < 4; ++k) ba.pde.coef[k] = (float)pde->coef[k];
  ba.pts = reinterpret_cast<const float4*>(ws + b.o_pts);
  ba.scratch = reinterpret_cast<float*>(ws + b.o_scratch);
  ba.scratch_per_wg = b.scratch_per_wg;
  ba.loss_slots = reinterpret_cast<double*>(ws + b.o_loss);
  ba.grad_slots = reinterpret_cast<double*>(ws + b.o_grad);
  for (int k = 0; k < kMaxOut; ++k) ba.lambda_res[k] = (float)pde->lambda_res[k];
  if (b.n_items > 0) {
    rc = timed(allow_timing, "k_zero_int", stream, [&] { return launch_zero_int(counter, stream); });
    if (rc) return rc;
    rc = timed(allow_timing, "k_batched", stream, [&] { return launch_batched(b.prec, b.act | (pde->lap_mask ? kLapFlag : 0), ba, b.grid, b.lds, stream); });
    if (rc) return rc;
  }
  BatchReduceArgs ra;
  ra.rows = reinterpret_cast<const BatchRow*>(dev(hrows));
  ra.n_entries = (int)n_entries;
  ra.n_rows = row0;
  ra.grad_slots = ba.grad_slots;
  rc = timed(allow_timing, "k_reduce_batched", stream, [&] { return launch_reduce_batched(ra, stream); });
  if (rc) return rc;
  BatchLossArgs la;
  la.loss_slots = ba.loss_slots;
  la.item0 = reinterpret_cast<const int64_t*>(dev(hitem0));
  la.n_items = reinterpret_cast<const int*>(dev(hnitems));
  la.w_res = reinterpret_cast<const double*>(dev(hw));
  la.n_inst = n_inst;
  la.n_res = b.n_res;
  la.losses = losses;
  rc = timed(allow_timing, "k_reduce_loss_batched", stream, [&] { return launch_reduce_loss_batched(la, stream); });
  if (rc) return rc;
  // instances on their own launches: after the batched reductions, which wrote zeros for
  // them, their fused steps write their loss and gradient
  for (int i = 0; i < n_inst; ++i) {
    if (!b.sep[i]) continue;
    pinn_pde pd = *pde;
    pd.norm_N = 0.0;
    rc = run(&nets[i], &pd, params[i], nullptr, points[i], n_points[i], nullptr, 0, prec, 0, nullptr, nullptr,
             losses + (size_t)i * (1 + b.n_res), grads[i], ws + b.o_sep, (size_t)b.sep_bytes, stream_, true,
             allow_timing);
    if (rc) return rc;
  }
  return hip_rc(hipGetLastError());
}

}  // namespace

namespace pinn {
// The fused step on a caller-provided workspace with event timing disabled (used by the
// allocation-free entry point, whose workspace is the library's static device scratch).
int run_bwd_untimed(const pinn_net* net, const pinn_pde* pde, const float* params, const float* B,
                    const float* points, int64_t n_points, const pinn_anchor* anchors, int n_anchor, int prec,
                    uint32_t flags, const pinn_tune* tune, float* residual, double* loss, double* grad,
                    void* workspace, size_t ws_bytes, pinn_stream_t stream) {
  return run(net, pde, params, B, points, n_points, anchors, n_anchor, prec, flags, tune, residual, loss, grad,
             workspace, ws_bytes, stream, true, false);
}
}  // namespace pinn

extern "C" {

int64_t pinn_param_count(const pinn_net* net) {
  Dims D;
  int rc = check_net(net, &D);
  return rc ? rc : D.n_params;
}

int pinn_n_residuals(int pde_id) { return n_res_of(pde_id); }

int pinn_workspace_bytes(const pinn_net* net, const pinn_pde* pde, int64_t n_points, const pinn_anchor* anchors,
                         int n_anchor, int prec, int with_grad, const pinn_tune* tune, size_t* bytes) {
  if (!bytes) return PINN_E_INVALID;
  int64_t b = 0;
  int rc = plan_bytes(net, pde, n_points, anchors, n_anchor, prec, with_grad, tune, &b);
  if (rc) return rc;
  *bytes = (size_t)b;
  return PINN_OK;
}

int pinn_residual_fwd(const pinn_net* net, const pinn_pde* pde, const float* params, const float* fourier_B,
                      const float* points, int64_t n_points, const pinn_anchor* anchors, int n_anchor, int prec,
                      uint32_t flags, const pinn_tune* tune, float* residual, double* loss, void* workspace,
                      size_t ws_bytes, pinn_stream_t stream) {
  return run(net, pde, params, fourier_B, points, n_points, anchors, n_anchor, prec, flags, tune, residual, loss,
             nullptr, workspace, ws_bytes, stream, false);
}

int pinn_residual_bwd(const pinn_net* net, const pinn_pde* pde, const float* params, const float* fourier_B,
                      const float* points, int64_t n_points, const pinn_anchor* anchors, int n_anchor, int prec,
                      uint32_t flags, const pinn_tune* tune, float* residual, double* loss, double* grad,
                      void* workspace, size_t ws_bytes, pinn_stream_t stream) {
  return run(net, pde, params, fourier_B, points, n_points, anchors, n_anchor, prec, flags, tune, residual, loss,
             grad, workspace, ws_bytes, stream, true);
}

int pinn_term_grads_workspace_bytes(const pinn_net* net, const pinn_pde* pde, int64_t n_points,
                                    const pinn_anchor* anchors, int n_anchor, int prec, const pinn_tune* tune,
                                    size_t* bytes) {
  if (!bytes || !pde || n_points < 1 || n_anchor < 0 || n_anchor > kMaxAnchors || (n_anchor > 0 && !anchors))
    return PINN_E_INVALID;
  for (int a = 0; a < n_anchor; ++a)
    if (anchors[a].n < 1) return PINN_E_INVALID;
  int64_t run_bytes = 0, b = 0;
  int rc = plan_bytes(net, pde, n_points, nullptr, 0, prec, 1, tune, &run_bytes);
  if (rc) return rc;
  for (int a = 0; a < n_anchor; ++a) {
    rc = plan_bytes(net, pde, 0, &anchors[a], 1, prec, 1, tune, &b);
    if (rc) return rc;
    run_bytes = std::max(run_bytes, b);
  }
  const int64_t tmp = align_up((int64_t)(1 + n_anchor) * (2 + n_res_of(pde->pde_id)) * 8, kAlign);
  *bytes = (size_t)(tmp + run_bytes);
  return PINN_OK;
}

int pinn_term_grads(const pinn_net* net, const pinn_pde* pde, const float* params, const float* fourier_B,
                    const float* points, int64_t n_points, const pinn_anchor* anchors, int n_anchor, int prec,
                    uint32_t flags, const pinn_tune* tune, double* loss, double* grads, void* workspace,
                    size_t ws_bytes, pinn_stream_t stream) {
  size_t need = 0;
  int rc = pinn_term_grads_workspace_bytes(net, pde, n_points, anchors, n_anchor, prec, tune, &need);
  if (rc) return rc;
  if (!loss || !grads || !workspace) return PINN_E_INVALID;
  if (ws_bytes < need) return PINN_E_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return PINN_E_INVALID;
  const int nres = n_res_of(pde->pde_id);
  const int64_t np = pinn_param_count(net);
  const int64_t tmp_bytes = align_up((int64_t)(1 + n_anchor) * (2 + nres) * 8, kAlign);
  double* tmp = static_cast<double*>(workspace);
  void* run_ws = static_cast<char*>(workspace) + tmp_bytes;
  const size_t run_bytes = ws_bytes - (size_t)tmp_bytes;
  // each term over its own points: together the same point work as one fused call
  rc = run(net, pde, params, fourier_B, points, n_points, nullptr, 0, prec, flags, tune, nullptr, tmp, grads, run_ws,
           run_bytes, stream, true);
  if (rc) return rc;
  for (int a = 0; a < n_anchor; ++a) {
    rc = run(net, pde, params, fourier_B, nullptr, 0, &anchors[a], 1, prec, flags & ~(uint32_t)PINN_FLAG_CHECK_FINITE,
             tune, nullptr, tmp + (size_t)(1 + a) * (2 + nres), grads + (size_t)(1 + a) * np, run_ws, run_bytes,
             stream, true);
    if (rc) return rc;
  }
  rc = launch_assemble_terms(tmp, 1 + n_anchor, nres, loss, reinterpret_cast<hipStream_t>(stream));
  if (rc) return rc;
  return hip_rc(hipGetLastError());
}

int pinn_causal_workspace_bytes(const pinn_net* net, const pinn_pde* pde, int64_t n_points, const pinn_causal* causal,
                                const pinn_anchor* anchors, int n_anchor, int prec, const pinn_tune* tune,
                                size_t* bytes) {
  if (!bytes || !pde || !causal || !causal->bin_n || causal->n_bins < 1 || causal->n_bins > 256) return PINN_E_INVALID;
  if (!(causal->eps >= 0.0) || !std::isfinite(causal->eps)) return PINN_E_INVALID;
  if (pde->norm_N != 0.0) return PINN_E_INVALID;  // every segment is its own mean
  int64_t tot = 0;
  for (int i = 0; i < causal->n_bins; ++i) {
    if (causal->bin_n[i] < 1) return PINN_E_INVALID;
    tot += causal->bin_n[i];
  }
  if (tot != n_points) return PINN_E_INVALID;
  int64_t run_bytes = 0, b = 0;
  for (int i = 0; i < causal->n_bins; ++i) {
    int rc = plan_bytes(net, pde, causal->bin_n[i], nullptr, 0, prec, 1, tune, &b);
    if (rc) return rc;
    run_bytes = std::max(run_bytes, b);
  }
  if (n_anchor > 0) {
    int rc = plan_bytes(net, pde, 0, anchors, n_anchor, prec, 1, tune, &b);
    if (rc) return rc;
    run_bytes = std::max(run_bytes, b);
  }
  const int64_t tmp = align_up((int64_t)causal->n_bins * (1 + n_res_of(pde->pde_id)) * 8 + causal->n_bins * 8, kAlign);
  *bytes = (size_t)(tmp + run_bytes);
  return PINN_OK;
}

int pinn_causal_bwd(const pinn_net* net, const pinn_pde* pde, const float* params, const float* fourier_B,
                    const float* points, int64_t n_points, const pinn_causal* causal, const pinn_anchor* anchors,
                    int n_anchor, int prec, uint32_t flags, const pinn_tune* tune, float* residual, double* loss,
                    double* grad, double* bin_loss, double* bin_w, void* workspace, size_t ws_bytes,
                    pinn_stream_t stream) {
  size_t need = 0;
  int rc = pinn_causal_workspace_bytes(net, pde, n_points, causal, anchors, n_anchor, prec, tune, &need);
  if (rc) return rc;
  if (!loss || !grad || !workspace || !points) return PINN_E_INVALID;
  if (ws_bytes < need) return PINN_E_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return PINN_E_INVALID;
  const int M = causal->n_bins, nres = n_res_of(pde->pde_id), d = net->d_in;
  const int stride = 1 + nres;
  double* tl = static_cast<double*>(workspace);                       // [M][1 + n_res] segment losses
  double* wbin = tl + (size_t)M * stride;                               // [M] w_i / M
  const int64_t tmp = align_up((int64_t)M * stride * 8 + M * 8, kAlign);
  void* run_ws = static_cast<char*>(workspace) + tmp;
  const size_t run_bytes = ws_bytes - (size_t)tmp;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // pass 1: each time segment's residual loss L^i (forward only)
  int64_t off = 0;
  for (int i = 0; i < M; ++i) {
    rc = run(net, pde, params, fourier_B, points + off * d, causal->bin_n[i], nullptr, 0, prec,
             i == 0 ? flags : flags & ~(uint32_t)PINN_FLAG_CHECK_FINITE, tune, nullptr, tl + (size_t)i * stride,
             nullptr, run_ws, run_bytes, stream, false);
    if (rc) return rc;
    off += causal->bin_n[i];
  }
  // the weights (Sec. 2.6.8), on the device
  rc = launch_causal_weights(tl, stride, M, causal->eps, wbin, bin_loss, bin_w, s);
  if (rc) return rc;
  // pass 2: the fused step per segment with its weight w_i / M (held fixed), and the
  // supervision sets, the gradients and loss terms accumulated
  bool acc = false;
  if (n_anchor > 0) {
    rc = run(net, pde, params, fourier_B, nullptr, 0, anchors, n_anchor, prec, flags & ~(uint32_t)PINN_FLAG_CHECK_FINITE,
             tune, nullptr, loss, grad, run_ws, run_bytes, stream, true);
    if (rc) return rc;
    acc = true;
  }
  off = 0;
  for (int i = 0; i < M; ++i) {
    pinn_pde pi = *pde;
    rc = run(net, &pi, params, fourier_B, points + off * d, causal->bin_n[i], nullptr, 0, prec,
             flags & ~(uint32_t)PINN_FLAG_CHECK_FINITE, tune, residual ? residual + off * nres : nullptr, loss, grad,
             run_ws, run_bytes, stream, true, true, wbin + i, acc);
    if (rc) return rc;
    acc = true;
    off += causal->bin_n[i];
  }
  return hip_rc(hipGetLastError());
}

int pinn_balance_update(const double* grads, int n_terms, int64_t n_params, double* lambda, double* lambda_hat,
                        double alpha, double eps, pinn_stream_t stream) {
  if (!grads || !lambda || n_terms < 1 || n_terms > 16 || n_params < 1) return PINN_E_INVALID;
  if (!(alpha >= 0.0 && alpha <= 1.0) || !(eps >= 0.0) || !std::isfinite(eps)) return PINN_E_INVALID;
  int rc = launch_balance(grads, n_terms, n_params, lambda, lambda_hat, alpha, eps,
                          reinterpret_cast<hipStream_t>(stream));
  if (rc) return rc;
  return hip_rc(hipGetLastError());
}

int pinn_batched_workspace_bytes(const pinn_net* nets, const pinn_pde* pde, const int64_t* n_points, int n_inst,
                                 int prec, const pinn_tune* tune_table, size_t* bytes) {
  if (!bytes) return PINN_E_INVALID;
  BatchPlan bp;
  int rc = make_batch_plan(nets, pde, n_points, n_inst, prec, tune_table, &bp);
  if (rc) return rc;
  *bytes = (size_t)bp.bytes;
  return PINN_OK;
}

int pinn_batched_bwd(const pinn_net* nets, const pinn_pde* pde, const float* const* params,
                     const float* const* points, const int64_t* n_points, int n_inst, int prec,
                     const pinn_tune* tune_table, double* const* grads, double* losses, void* workspace,
                     size_t ws_bytes, pinn_stream_t stream) {
  return run_batched(nets, pde, params, points, n_points, n_inst, prec, tune_table, grads, losses, workspace,
                     ws_bytes, stream);
}

int pinn_timing_enable(int on) {
  Timing& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  T.on = on != 0;
  return PINN_OK;
}

int pinn_timing_collect(pinn_kernel_time* out, int max_entries, int* n_entries) {
  if (!n_entries || max_entries < 0 || (max_entries > 0 && !out)) return PINN_E_INVALID;
  Timing& T = timing();
  std::lock_guard<std::mutex> lk(T.mu);
  std::vector<std::string> names;
  std::vector<int64_t> count;
  std::vector<double> ms;
  int rc = PINN_OK;
  for (auto& tl : T.rec) {
    float t = 0.0f;
    if (hipEventSynchronize(tl.stop) != hipSuccess || hipEventElapsedTime(&t, tl.start, tl.stop) != hipSuccess)
      rc = PINN_E_HIP;
    size_t k = 0;
    while (k < names.size() && names[k] != tl.name) ++k;
    if (k == names.size()) {
      names.emplace_back(tl.name);
      count.push_back(0);
      ms.push_back(0.0);
    }
    count[k] += 1;
    ms[k] += t;
    T.pool.push_back(tl.start);
    T.pool.push_back(tl.stop);
  }
  T.rec.clear();
  int n = 0;
  for (size_t k = 0; k < names.size() && n < max_entries; ++k, ++n) {
    std::memset(out[n].name, 0, sizeof(out[n].name));
    std::strncpy(out[n].name, names[k].c_str(), sizeof(out[n].name) - 1);
    out[n].launches = count[k];
    out[n].total_ms = ms[k];
  }
  *n_entries = n;
  return rc;
}

const char* pinn_status_string(int status) {
  switch (status) {
    case PINN_OK: return "ok";
    case PINN_E_INVALID: return "invalid argument";
    case PINN_E_UNSUPPORTED: return "unsupported configuration";
    case PINN_E_WORKSPACE: return "workspace too small";
    case PINN_E_NONFINITE: return "non-finite parameter";
    case PINN_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

}  // extern "C"
