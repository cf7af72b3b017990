// pinn_internal.h -- descriptors shared by the host planner (pinn_api.cpp) and the HIP
// kernels (k_*.hip, pinn_device.h).  Not part of the public C ABI.
#pragma once
#include <stdint.h>
#include <stddef.h>

#include <hip/hip_runtime.h>

namespace pinn {

constexpr int kMaxHidden = 8;
constexpr int kMaxLayers = kMaxHidden + 1;
constexpr int kMaxAnchors = 8;
constexpr int kMaxOut = 4;      // network outputs and residual components (2D Euler: 4)
constexpr int kMaxTerms = kMaxOut + kMaxAnchors;
constexpr int kSegAlign = 128;  // every point segment starts at a multiple of this
constexpr int kWaves = 8;
constexpr int kRedThreads = 1024;  // reduction blocks: kRedGroups slot groups x 256 columns
constexpr int kRedGroups = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kMaxFreq = 128;                     // Fourier frequencies (2 m <= 256)
constexpr int kFourierLds = 3 * kMaxFreq * 4;     // LDS bytes of a staged Fourier matrix
constexpr int kOutLds = 8 * 4 * kMaxOut * 32;     // LDS bytes of the staged output-layer fragments

// Kernel precision codes.  The two split forms run three 16-bit matrix-core products per
// logical product (hi*hi + hi*lo + lo*hi, x = hi + lo); they differ in the 16-bit format.
enum { kFP32 = 0, kBF16X3 = 1, kFP16X3 = 2 };
__host__ __device__ constexpr bool is_split(int prec) { return prec != kFP32; }
enum { kTanh = 0, kSin = 1 };
// Kernel activation code: kTanh or kSin, plus kLapFlag when jet channel 3 is a Laplacian.
enum { kLapFlag = 2 };
enum { kBurgers = 1, kEuler1D = 2, kNS2D = 3, kMaxwell = 4, kAdvection = 5, kAllenCahn = 6, kEuler2D = 7 };

// One linear layer as the kernels see it (all pointers into the workspace).
struct LayerDev {
  int n_in, n_out;     // true sizes
  int nbo, kci;        // forward fragments: n_out/16 blocks (padded) x n_in/32 chunks (padded)
  int nbi, kco;        // backward fragments: n_in/16 blocks x n_out/32 chunks
  const char* wf;      // forward fragments  [nbo][kci][64 lanes][32 B]
  const char* wb;      // backward fragments [nbi][kco][64 lanes][32 B]
  const float* w;      // effective weights, FP32, n_out x n_in row-major
  const float* b;      // bias, FP32, n_out (zeros without bias)
};

struct NetDev {
  int L;               // hidden layers
  int d_in, d_out;
  int e;               // embedding width (d_in, 2 * n_freq, or inputs with periodic ones twice)
  int n_freq;
  int periodic_mask;   // inputs embedded as [cos, sin](omega_k x_k) (0: identity or Fourier)
  const float* omega;  // omega_k = 2 pi / P_k of the periodic inputs (workspace, from k_prepare)
  int lap_mask;        // inputs in the Laplacian set
  int lapch;           // channel of the Laplacian (-1 if none)
  float w0;
  const float* B;      // Fourier matrix d_in x n_freq (device, caller's)
  LayerDev layer[kMaxLayers];
};

struct SegDev {
  int n_seg;                       // 1 + number of anchor sets
  int64_t start[1 + kMaxAnchors];  // first padded point of the segment
  int64_t n[1 + kMaxAnchors];      // valid points
  const float* targets[kMaxAnchors];
  int out_mask[kMaxAnchors];
  float lam_anchor[kMaxAnchors];   // seed scale: 2 lambda / N_s
};

struct PdeDev {
  int pde_id, n_res;
  float coef[4];
  float seed_scale[kMaxOut];       // 2 lambda_c / N
};

// Workspace pieces used by the kernels.
struct Work {
  int64_t n_pad;                   // padded point count (all segments)
  const float4* pts;               // n_pad x (x, y, t, 0)
  float* zs0;                      // pre-activation stash of hidden layer 0, fragment-major;
  int64_t zs_stride;               // layer j starts zs_stride floats after layer j - 1
  float* zb[2];                    // adjoint ping-pong, fragment-major
  double* loss_slots;              // [grid_f][kMaxTerms] sums of squares
  double* out_slots;               // [grid_f][d_out * (n_L + 1)] output-layer W and b sums
  double* layer_slots[kMaxHidden]; // [grid_b][n_out * (n_in + 1)] hidden/embedding layer sums
  // FP16X3: largest magnitude of the adjoint of each hidden layer's pre-activation jets
  // (FP32 bit patterns, combined by integer maximum), written by the kernel that produces
  // the adjoint and read by the kernel that consumes it; zeroed at the start of a call
  unsigned int* amax;              // [kMaxHidden]
};

// Kernel argument blocks (passed by value).
struct StageArgs {
  int n_layers;
  int rwf, has_bias;
  int periodic_mask, period_train_mask;
  float period[3];
  int64_t off_p;                // first trainable period in params
  float* omega;                 // out: 2 pi / P_k per input (0 for inputs that pass through)
  const float* params;
  int64_t off_w[kMaxLayers], off_s[kMaxLayers], off_b[kMaxLayers];
  int n_in[kMaxLayers], n_out[kMaxLayers];
  char* wf[kMaxLayers];
  char* wb[kMaxLayers];
  float* w[kMaxLayers];
  float* b[kMaxLayers];
  int64_t cum[kMaxLayers + 1];  // cumulative thread counts per layer
};

struct PointsArgs {
  int d_in;
  int n_seg;
  int64_t start[1 + kMaxAnchors], n[1 + kMaxAnchors];
  const float* src[1 + kMaxAnchors];
  int64_t n_pad;
  float4* dst;
  unsigned int* zero;    // words cleared before anything else of the call runs (or null)
  int n_zero;
};

struct FwdArgs {
  NetDev net;
  PdeDev pde;
  SegDev seg;
  Work work;
  int64_t n_tiles;
  int kmax;          // widest GEMM input (R-layout row width, elements)
  int with_grad;
  float* residual;   // caller's n x n_res or null
  const double* wscale;  // device weight multiplying the residual seed (or null)
};

struct BwdArgs {
  NetDev net;
  Work work;
  int layer;          // linear layer j (input side 0)
  int64_t n_sub;      // sub-tiles of the padded point set
  const float* zb_in;   // adjoint of this layer's output (fragment-major, n_out wide)
  float* zb_out;        // adjoint of the previous hidden layer's pre-activation (or null)
  const float* z_prev;  // stash of the previous hidden layer (null for layer 0)
  double* slots;        // [gridDim][n_out * (n_in + 1)]
  int wide;             // use the wide bf16x3 kernel (input width a multiple of 128)
  int pb;               // sub-tile points of the split-role kernel (wide_pb(H) or half)
  // layer 1 over an identity embedding (split-role kernel): the input-adjoint role sums the
  // first layer's weight and bias gradient from the adjoint it computes, into these slots
  // ([grid / 2][n_in * (d_in + 1)]), instead of writing that adjoint to zb_out
  double* g0_slots;
  // split roles: progress of each weight-gradient work-group, (launch << 20) + sub-tile
  // index, read by its input-adjoint partner to stay at most one sub-tile ahead
  unsigned long long* pace;
  unsigned long long launch;
};

struct Grad0Args {
  const float* zb;
  const float4* pts;
  int n_out, d_in;
  int64_t n_cb;       // cp blocks of the padded point set
  double* slots;      // [gridDim][n_out * (e + 1) (+ n_out * 2 * trained periods)]
  // periodic embedding (0: identity): the weight gradient runs over the e embedding
  // features, and for every trained period the sums G[o][j] = sum zbar[o] . d e_j / d omega
  // of its two features follow the bias sums
  int periodic_mask, period_train_mask, lap_mask, e;
  const float* omega;
};

// d(loss)/dP_k of the trained periods: (-omega_k / P_k) sum_o sum_j W[o][j] G[o][j], the G
// sums reduced over the work-group slots in slot order.
struct PeriodReduceArgs {
  const double* slots;
  int n_slots;
  int64_t slot_stride;
  int n_out, e;
  int periodic_mask, period_train_mask, d_in;
  const float* w;       // effective first-layer weights, n_out x e
  const float* omega;
  double* grad;         // the gradient, periods at off_p
  int64_t off_p;
  int accumulate;
  const double* w64;    // FP64 precision: double weights and omega instead of w / omega
  const double* omega64;
};

struct ReduceArgs {
  const double* slots;
  int n_slots;
  int64_t slot_stride;    // doubles between consecutive slots
  int n_out, n_in;
  int rwf, has_bias;
  const float* params;
  int64_t off_w, off_s, off_b;
  double* grad;
  int accumulate;         // add to grad instead of overwriting it
};

struct LossArgs {
  const double* slots;
  int n_slots;
  int n_res, n_anchor;
  double w_res[kMaxOut];  // lambda_c / N
  double w_anchor[kMaxAnchors];  // lambda_s / N_s
  double* loss;
  const double* wscale;   // device weight of the residual terms (or null)
  int accumulate;         // add to loss instead of overwriting it
};

// Every layer's slot reduction and the loss terms in one launch: blocks row0[l] ..
// row0[l + 1] - 1 reduce the rows of layer l, block row0[n_layers] the loss.
struct ReduceAllArgs {
  ReduceArgs layer[kMaxLayers];
  int row0[kMaxLayers + 1];
  int n_layers;
  LossArgs loss;
};


// Many independent networks in one persistent launch.
struct BatchInst {
  NetDev net;
  int H;                     // width bucket
  int kmax;                  // widest product input (R-layout row width)
  int64_t pts_off;           // first padded point of the instance in the shared buffer
  int64_t n;                 // valid points
  int64_t eff_off[kMaxLayers];  // offset of layer l's sums inside an item slot
  int64_t zs_stride;         // floats between hidden layers' stash in the work-group scratch
  int64_t zb_off[2];         // adjoint ping-pong offsets in the work-group scratch (floats)
};

struct BatchItem {
  int inst;
  int64_t p0, p1;            // padded point range of the instance (multiples of 128)
  int64_t slot_off;          // offset of the item's gradient slot (doubles)
};

struct BatchArgs {
  const BatchInst* inst;
  const BatchItem* items;
  const int64_t* order;      // items in the order the queue hands them out
  int n_items;
  int* counter;              // zeroed before the launch
  PdeDev pde;
  const float4* pts;
  float* scratch;            // per work-group jet buffers
  int64_t scratch_per_wg;    // floats
  double* loss_slots;        // [n_items][kMaxTerms]
  double* grad_slots;
  float lambda_res[kMaxOut]; // residual weights; the seed scale is 2 lambda / n per instance
};

struct BatchRow {            // one (instance, layer): rows [row0, row0 + n_out) of the grid
  int64_t row0;
  int64_t slot0;             // first item's slot for this layer (doubles)
  int64_t slot_stride;       // between consecutive items' slots
  int n_items;
  int n_out, n_in, rwf, has_bias;
  const float* params;
  int64_t off_w, off_s, off_b;
  double* grad;
};

struct BatchReduceArgs {
  const BatchRow* rows;
  int n_entries;
  int64_t n_rows;
  const double* grad_slots;
};

struct BatchLossArgs {
  const double* loss_slots;
  const int64_t* item0;      // first item of each instance
  const int* n_items;
  const double* w_res;       // [n_inst][kMaxOut] lambda_c / N_i
  int n_inst, n_res;
  double* losses;            // [n_inst][1 + n_res]
};

// The FP64 precision (k_fp64.hip): one thread per point, double precision throughout.
struct F64StageArgs {
  int n_layers, rwf, has_bias;
  int periodic_mask, period_train_mask;
  float period[3];
  int64_t off_p;
  const float* params;
  int64_t off_w[kMaxLayers], off_s[kMaxLayers], off_b[kMaxLayers];
  int n_in[kMaxLayers], n_out[kMaxLayers];
  double* w[kMaxLayers];
  double* b[kMaxLayers];
  double* omega;                 // [3]
};

struct F64Args {
  int64_t n_pad;
  int L, d_in, d_out, e, n_freq, act;
  int periodic_mask, period_train_mask, lap_mask, lapch;
  int ng;                        // omega rows of the first layer (2 per trained period)
  double w0;
  int n_in[kMaxLayers], n_out[kMaxLayers];
  const double* w[kMaxLayers];
  const double* b[kMaxLayers];
  double* a[kMaxLayers];         // jets feeding linear layer l (a[0]: embedding)
  double* z[kMaxHidden];         // pre-activation jets of hidden layer l
  double* zb[kMaxHidden];        // their adjoints
  double* ab[2];                 // activation adjoints, alternating
  double* yb;                    // output-jet seed
  double* dw;                    // omega-derivatives of the trained periods' features
  const double* omega;
  const float* B;                // Fourier matrix (caller's)
  const float4* pts;
  int pde_id, n_res;
  double coef[4];
  double seed[kMaxOut];          // 2 lambda_c / N
  double lam_anchor[kMaxAnchors];  // 2 lambda_s / N_s
  const double* wscale;          // device weight of the residual seed (or null)
  SegDev seg;
  float* residual;
  double* loss_slots;            // [blocks][kMaxTerms]
};

int launch_fp64(const F64StageArgs& s, const F64Args& a, double* const* slots, hipStream_t st);

// Sub-tile points of the wide bf16x3 layer backward (input width a multiple of 128).
constexpr int wide_pb(int H) { return H >= 256 ? 16 : 32; }
// Forward tile points: the width's default, and the alternatives a caller may choose.
constexpr int fwd_default_p(int H) { return H == 256 ? 32 : H == 128 ? 64 : H == 64 ? 64 : 128; }
constexpr int fwd_half_p(int H) { return fwd_default_p(H) / 2 >= 32 ? fwd_default_p(H) / 2 : 0; }

// Waves per work-group of the forward kernel for hidden width H and tile points P.
constexpr int fwd_waves(int H, int P) { return kWaves; }
// Resident forward work-groups per compute unit.
constexpr int fwd_wg_per_cu(int H, int P) { return kWaves / fwd_waves(H, P); }
// 16-point forward tiles keep two layer-input tiles in LDS: layer j's activations go to one
// while layer j's product may still read the other, so a wave that finishes its product
// starts its activations without waiting for the slower waves.
constexpr bool fwd_double_x(int P) { return P <= 16; }

// Launchers (k_*.hip).  Each returns a pinn_status value.
int launch_check_finite(const float* p, int64_t n, int* flag, hipStream_t s);
int launch_points(const PointsArgs& a, hipStream_t s);
int launch_forward(int prec, int act, int H, int P, const FwdArgs& a, int grid, size_t lds, hipStream_t s);
int launch_backward(int prec, int act, int H, bool embed, const BwdArgs& a, int grid, size_t lds, hipStream_t s);
int launch_grad0(const Grad0Args& a, int grid, hipStream_t s);
int launch_reduce_layer(const ReduceArgs& a, hipStream_t s);
int launch_reduce_period(const PeriodReduceArgs& a, hipStream_t s);
int launch_assemble_terms(const double* tmp, int n_terms, int n_res, double* loss, hipStream_t s);
int launch_causal_weights(const double* bin_loss, int stride, int n_bins, double eps, double* wbin, double* bin_loss_out,
                          double* w_out, hipStream_t s);
int launch_balance(const double* grads, int n_terms, int64_t n_params, double* lambda, double* hat, double alpha,
                   double eps, hipStream_t s);
int launch_reduce_loss(const LossArgs& a, hipStream_t s);
int launch_reduce_all(const ReduceAllArgs& a, hipStream_t s);
int launch_prepare(int prec, const PointsArgs& pa, const StageArgs& sa, hipStream_t s);
int launch_batched(int prec, int act, const BatchArgs& a, int grid, size_t lds, hipStream_t s);
int launch_reduce_batched(const BatchReduceArgs& a, hipStream_t s);
int launch_reduce_loss_batched(const BatchLossArgs& a, hipStream_t s);
int launch_zero_int(int* p, hipStream_t s);
size_t batched_lds(int kmax_max, int H_max);

}  // namespace pinn
