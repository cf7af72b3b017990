/*
 * pinn.h -- C ABI of the fused PINN residual + parameter-gradient library (libpinn.so,
 * gfx950 / MI355X).
 *
 * The operation (paper: QPINNACLE, arXiv 2604.15645):
 *   network   Sec. 2.2: z = W a + b per layer, a = sigma(z), linear output layer;
 *             sigma = tanh (Sec. 2.2) or sin(w0 z) (App. A.5).  Optional input embedding
 *             by random Fourier features [cos(xB), sin(xB)] (Sec. 2.6.1, App. A.2) and
 *             optional weight factorisation W = diag(exp s) V on every linear layer
 *             (Sec. 2.6.2).
 *   residual  per PDE, "left side minus right side" of the printed equation:
 *             Burgers (Sec. 4.3, with viscosity nu u_xx), 1D Euler in conservative form
 *             (Sec. 4.6), steady incompressible Navier-Stokes (Sec. 4.4), 2D Maxwell
 *             (Sec. 4.8), linear advection (Sec. 4.1), Allen-Cahn (Sec. 4.2).
 *   loss      Sec. 2.3: L = sum_c lambda_c (1/N) sum_i r_c(x_i)^2
 *                         + sum_s lambda_s (1/N_s) sum_i sum_{o in mask_s} (y_o(x_i) - t_{o,i})^2
 *   gradient  dL/dtheta for every parameter theta (the quantity the optimiser of Sec. 2.3
 *             consumes).  The Fourier matrix B is fixed (no gradient); inputs are not
 *             differentiated.
 *
 * Conventions shared by every entry point.
 *   Pointers are DEVICE pointers unless marked (host).  The caller owns every buffer,
 *   including the workspace; the compute calls keep nothing between calls and allocate
 *   no device memory (the only process-wide state is the optional per-kernel timing
 *   record declared at the end).  Calls are asynchronous on `stream` (a hipStream_t; NULL = the null stream);
 *   the return code reports argument errors (checked on the host, before any HIP call)
 *   and launch errors.  Calls sharing a workspace must not overlap.
 *   Points: n x d_in, row-major, FP32, inputs ordered (x,t) Burgers/Euler/advection/
 *   Allen-Cahn, (x,y) NS, (x,y,t) Maxwell and 2D Euler.  Parameters: FP32, flat, per linear layer l = 0..n_hidden (input
 *   side first): [W_l or V_l (n_out x n_in, row-major)] [s_l (n_out) if rwf]
 *   [b_l (n_out) if has_bias], then the trainable periods of a periodic embedding.
 *   Gradient: FP64 in the same layout.
 *   Device limits: d_in <= 3, d_out <= 4, 1 + d_in + (Laplacian needed) <= 4 derivative
 *   channels, hidden widths multiples of 32 and <= 256, n_freq a multiple of 16 with
 *   2*n_freq <= 256, n_hidden in 1..8 (PINN_PREC_FP64: any width <= 256, any n_freq,
 *   n_hidden in 0..8).
 */
#ifndef PINN_H
#define PINN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* pinn_stream_t; /* == hipStream_t */

typedef enum {
  PINN_OK = 0,
  PINN_E_INVALID = -1,     /* malformed descriptor, null pointer, bad size          */
  PINN_E_UNSUPPORTED = -2, /* valid request outside what the kernels implement      */
  PINN_E_WORKSPACE = -3,   /* ws_bytes smaller than pinn_workspace_bytes() reports  */
  PINN_E_NONFINITE = -4,   /* PINN_FLAG_CHECK_FINITE found NaN/Inf in the parameters */
  PINN_E_HIP = -5          /* a HIP runtime call or kernel launch failed            */
} pinn_status;

typedef enum {
  PINN_PDE_BURGERS = 1,       /* in (x,t), out u:          u_t + u u_x - nu u_xx       */
  PINN_PDE_EULER1D = 2,       /* in (x,t), out (rho,u,p):  conservative 1D Euler       */
  PINN_PDE_NS2D_STEADY = 3,   /* in (x,y), out (u,v,p):    continuity + 2 momentum     */
  PINN_PDE_MAXWELL_TE2D = 4,  /* in (x,y,t), out (E_z,H_x,H_y)                          */
  PINN_PDE_ADVECTION = 5,     /* in (x,t), out u:          u_t + c u_x (Sec. 4.1)      */
  PINN_PDE_ALLEN_CAHN = 6,    /* in (x,t), out u:          u_t - D u_xx + k (u^3 - u)
                                 (Sec. 4.2; the paper's D = 1e-4, k = 5)              */
  PINN_PDE_EULER2D = 7        /* in (x,y,t), out (rho,u,v,p): conservative 2D Euler,
                                 mass, two momentum and energy residuals (Sec. 4.7)   */
} pinn_pde_id;

typedef enum { PINN_ACT_TANH = 0, PINN_ACT_SIN = 1 } pinn_act;

typedef enum {
  PINN_PREC_FP32 = 0,   /* FP32 matrix cores (v_mfma_f32_16x16x4_f32), FP32 accumulate   */
  PINN_PREC_BF16X3 = 1, /* each product a*b as hi*hi + hi*lo + lo*hi with a = hi + lo,
                           hi = bf16(a), lo = bf16(a - hi), BF16 matrix cores, FP32
                           accumulate.  hi + lo holds 16 significant bits, so each
                           operand is represented to about 2^-16 relative; a residual
                           much smaller than the terms it is formed from (strong
                           cancellation) loses accuracy in proportion.                  */
  PINN_PREC_BF16 = 2,   /* one BF16 product per product (8 significant bits): not
                           implemented -- the derivative jets of a residual need more;
                           returns PINN_E_UNSUPPORTED                                   */
  PINN_PREC_FP64 = 3,   /* double precision throughout on the vector ALU, one thread per
                           point: a checking mode (finite differences at small steps,
                           parity with an FP64 reference to rounding), not a fast path.
                           Also takes any hidden width <= 256 and n_hidden = 0 (a linear
                           read-out of the embedding).  Not available to the batched call. */
  PINN_PREC_FP16X3 = 4  /* as BF16X3 with IEEE half parts, hi = fp16(a), lo = fp16(a - hi),
                           FP16 matrix cores (the same rate as BF16): 22 significant bits,
                           operands represented to about 2^-22.  Half precision has a
                           narrow range: every adjoint is scaled by a power of two from its
                           largest magnitude before it is split (exact, undone on the
                           result); activation jets and weights are split unscaled and must
                           stay below 65504 in magnitude (the result is otherwise not
                           finite); parts below 2^-14 keep an absolute resolution of 2^-24. */
} pinn_prec;

/* Opt-in flags (bitwise or). */
#define PINN_FLAG_CHECK_FINITE 1 /* scan the parameters for NaN/Inf first; this call then
                                    synchronises `stream` (the check mirrors the NaN test
                                    on the network input in App. B)                   */

/* (host) Network descriptor. */
typedef struct {
  int32_t d_in, d_out;   /* d_in 1..3, d_out 1..4                                        */
  int32_t n_hidden;      /* hidden layers L                                              */
  int32_t width[8];      /* hidden widths                                                */
  int32_t act;           /* pinn_act                                                     */
  float w0;              /* sine frequency, sigma(z) = sin(w0 z)                          */
  int32_t n_freq;        /* 0: identity embedding; m > 0: Fourier features, B is d_in x m */
  int32_t rwf;           /* 1: every linear layer stored as (V, s), W = diag(exp s) V    */
  int32_t has_bias;      /* 1: every linear layer has a bias                             */
  /* Strict periodic input embedding (Sec. 2.6.3; requires n_freq == 0): input k with bit k
   * of periodic_mask enters the network as the pair [cos(2 pi x_k / P_k), sin(2 pi x_k / P_k)],
   * the other inputs as themselves, in input order; the output is then periodic in x_k
   * with period P_k, derivatives included.  P_k is period[k], or, with bit k of
   * period_train_mask, a trainable parameter stored after every layer's parameters (one
   * FP32 value per trained input, in input order) whose gradient is returned there.      */
  int32_t periodic_mask;
  int32_t period_train_mask; /* subset of periodic_mask                                   */
  float period[3];
} pinn_net;

/* (host) PDE descriptor. */
typedef struct {
  int32_t pde_id;        /* pinn_pde_id                                                  */
  int32_t lap_mask;      /* bit k: input k belongs to the Laplacian set S (Burgers: x,
                            NS: x and y; Euler and Maxwell need none)                     */
  double coef[4];        /* Burgers: nu | Euler: gamma | NS: Re | Maxwell: eps, mu |
                            advection: c | Allen-Cahn: D, k | 2D Euler: gamma             */
  double lambda_res[4];  /* weight of each residual component's mean square             */
  double norm_N;         /* divisor of the residual means; 0 = n_points of this call.
                            A caller that shards the points passes the global count.     */
} pinn_pde;

/* (host) Value-only supervision set (initial / boundary data).  Device arrays. */
typedef struct {
  const float* points;   /* n x d_in                                                     */
  const float* targets;  /* n x d_out (only outputs in out_mask are read)               */
  int64_t n;
  int32_t out_mask;      /* bit o: output o is supervised                               */
  double lambda;
} pinn_anchor;

/* (host) Optional launch shape; NULL selects the built-in plan.  Fields <= 0 = default. */
typedef struct {
  int32_t tile_points;   /* forward tile points: the width's default (32 for width 256,
                            64 for 64..128, 128 for 32), half of it when that is at least
                            32, or 16                                                     */
  int32_t grid;          /* work-groups of the persistent launches (default 256)          */
  int32_t bwd_points;    /* sub-tile points of the split-role hidden-layer backward
                            (uniform hidden width 128 or 256, split precisions): the
                            default (32 at width 128, 16 at 256) or half of it            */
  int32_t chunk_points;  /* batched call: points per work item, a multiple of 128
                            (default 1024 for width 256, 2048 for 128, 4096 below), or
                            -1: the instance runs as a fused step of its own (the
                            single-network kernels) after the persistent launch          */
} pinn_tune;

/* Number of FP32 parameters of the network (layout above).  < 0 on a bad descriptor. */
int64_t pinn_param_count(const pinn_net* net);

/* Number of residual components of a PDE (1, 3 or 4); < 0 if unknown. */
int pinn_n_residuals(int pde_id);

/* Workspace bytes needed by pinn_residual_fwd / _bwd for this problem and plan.
 * `with_grad` = 1 for _bwd.  Writes *bytes (host).  Errors as for the compute calls. */
int pinn_workspace_bytes(const pinn_net* net, const pinn_pde* pde, int64_t n_points,
                         const pinn_anchor* anchors, int n_anchor, int prec, int with_grad,
                         const pinn_tune* tune, size_t* bytes);

/* Residual and loss (no gradient).
 *   params     FP32 [pinn_param_count]
 *   fourier_B  FP32 d_in x n_freq row-major, or NULL when n_freq == 0
 *   points     FP32 n_points x d_in
 *   anchors    (host) array of n_anchor value-supervision sets (device arrays inside)
 *   residual   FP32 n_points x n_res, or NULL
 *   loss       FP64 [1 + n_res + n_anchor]: total, each residual component's weighted
 *              mean square, each anchor set's weighted mean square
 *   workspace  device buffer of ws_bytes >= pinn_workspace_bytes(..., with_grad = 0) */
int pinn_residual_fwd(const pinn_net* net, const pinn_pde* pde, const float* params,
                      const float* fourier_B, const float* points, int64_t n_points,
                      const pinn_anchor* anchors, int n_anchor, int prec, uint32_t flags,
                      const pinn_tune* tune, float* residual, double* loss, void* workspace,
                      size_t ws_bytes, pinn_stream_t stream);

/* The fused step: residual, loss and dL/dtheta in one call.
 *   grad       FP64 [pinn_param_count], overwritten (parameter layout)
 *   other arguments as pinn_residual_fwd; workspace sized with with_grad = 1.
 * The parameter-gradient sum over points is accumulated in FP64; the result does not
 * depend on the order of the points beyond FP64 rounding. */
int pinn_residual_bwd(const pinn_net* net, const pinn_pde* pde, const float* params,
                      const float* fourier_B, const float* points, int64_t n_points,
                      const pinn_anchor* anchors, int n_anchor, int prec, uint32_t flags,
                      const pinn_tune* tune, float* residual, double* loss, double* grad,
                      void* workspace, size_t ws_bytes, pinn_stream_t stream);

/* The fused step without a caller workspace, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that forbid
 * allocation).  Arguments and results as pinn_residual_bwd.  The workspace is the
 * library's own static device array of PINN_NOALLOC_MAX_BYTES, one per GPU, held until
 * the process ends; this call allocates nothing.  A problem whose pinn_workspace_bytes(...,
 * with_grad = 1, ...) exceeds that size is refused with PINN_E_WORKSPACE before any HIP
 * call.  Every call on one GPU uses that GPU's array and leaves its contents behind (each
 * call clears what it needs cleared): calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  The per-kernel timing record is
 * not kept for these calls (it would create events). */
#define PINN_NOALLOC_MAX_BYTES (64u << 20)
int pinn_residual_bwd_noalloc(const pinn_net* net, const pinn_pde* pde, const float* params,
                              const float* fourier_B, const float* points, int64_t n_points,
                              const pinn_anchor* anchors, int n_anchor, int prec, uint32_t flags,
                              const pinn_tune* tune, float* residual, double* loss, double* grad,
                              pinn_stream_t stream);

/* Per-term gradients for loss balancing (Sec. 2.6.4).  Term 0 is the residual term (every
 * residual component with its weight lambda_res[c], mean over the n_points residual points
 * or pde->norm_N), term 1 + a the supervision set a (its weight and mean).  Each term
 * involves only its own points, so the call runs the fused step over each term's points
 * in turn (together the point work of one pinn_residual_bwd call):
 *   loss   FP64 [1 + n_res + n_anchor], as pinn_residual_bwd (the total is the sum)
 *   grads  FP64 [(1 + n_anchor) x pinn_param_count], term t's gradient at t * n_params;
 *          their sum is pinn_residual_bwd's gradient
 * n_points >= 1 and every set non-empty.  Workspace from pinn_term_grads_workspace_bytes. */
int pinn_term_grads_workspace_bytes(const pinn_net* net, const pinn_pde* pde, int64_t n_points,
                                    const pinn_anchor* anchors, int n_anchor, int prec,
                                    const pinn_tune* tune, size_t* bytes);
int pinn_term_grads(const pinn_net* net, const pinn_pde* pde, const float* params,
                    const float* fourier_B, const float* points, int64_t n_points,
                    const pinn_anchor* anchors, int n_anchor, int prec, uint32_t flags,
                    const pinn_tune* tune, double* loss, double* grads, void* workspace,
                    size_t ws_bytes, pinn_stream_t stream);

/* Temporal causality (Sec. 2.6.8).  The residual points come sorted into M consecutive
 * time segments (segment i holds bin_n[i] points, in order).  With L^i the residual loss of
 * segment i alone (every component with its weight lambda_res[c], mean over the segment's
 * points) the weights are w_1 = 1, w_i = exp(-eps * (L^1 + ... + L^{i-1})), and the residual
 * term becomes (1/M) sum_i w_i L^i.  The weights are computed from the current losses and
 * held fixed in the gradient (the paper does not differentiate them).                     */
typedef struct {
  int32_t n_bins;        /* M, 1..256                                                    */
  const int64_t* bin_n;  /* (host) [M] points per segment, >= 1 each, summing to n_points */
  double eps;            /* decay rate, >= 0                                             */
} pinn_causal;

/* The fused step with the causality-weighted residual term: a forward pass per segment for
 * the L^i (device), the weights on the device, then the fused step per segment with weight
 * w_i / M, and the supervision sets (unweighted, as pinn_residual_bwd), accumulated.
 *   residual  FP32 n_points x n_res (unweighted residuals), or NULL
 *   loss      FP64 [1 + n_res + n_anchor]: total, weighted residual components, sets
 *   grad      FP64 [pinn_param_count]
 *   bin_loss, bin_w  FP64 [M] each, the L^i and the w_i (device), or NULL
 * pde->norm_N must be 0 (each segment is its own mean).  The call makes 2M + 1 launch
 * sequences; workspace from pinn_causal_workspace_bytes.                                  */
int pinn_causal_workspace_bytes(const pinn_net* net, const pinn_pde* pde, int64_t n_points,
                                const pinn_causal* causal, const pinn_anchor* anchors,
                                int n_anchor, int prec, const pinn_tune* tune, size_t* bytes);
int pinn_causal_bwd(const pinn_net* net, const pinn_pde* pde, const float* params,
                    const float* fourier_B, const float* points, int64_t n_points,
                    const pinn_causal* causal, const pinn_anchor* anchors, int n_anchor, int prec,
                    uint32_t flags, const pinn_tune* tune, float* residual, double* loss,
                    double* grad, double* bin_loss, double* bin_w, void* workspace,
                    size_t ws_bytes, pinn_stream_t stream);

/* Loss-balancing weights from per-term gradients (Sec. 2.6.4), on the device, without a
 * host round trip.  With n_t = ||grads[t]||_2 (FP64, fixed summation order):
 *   lambda_hat[t] = (n_0 + ... + n_{T-1}) / (n_t + eps)
 *   lambda[t]    <- alpha * lambda[t] + (1 - alpha) * lambda_hat[t]     (paper: alpha 0.9)
 * eps (>= 0) guards a vanishing gradient (the paper's code uses 1e-9).  grads: device FP64
 * [n_terms x n_params]; lambda: device FP64 [n_terms], updated in place; lambda_hat:
 * device FP64 [n_terms] or NULL.  1 <= n_terms <= 16, 0 <= alpha <= 1. */
int pinn_balance_update(const double* grads, int n_terms, int64_t n_params, double* lambda,
                        double* lambda_hat, double alpha, double eps, pinn_stream_t stream);

/* Many independent networks in one persistent launch: the hyperparameter searches and
 * repeated random initialisations whose cost Sec. 1.2 counts against PINNs, and the
 * per-method comparisons of Sec. 4, where each network trains as a run of its own.
 * Instance i has its own descriptor nets[i] (host array), the
 * shared PDE `pde`, its own params[i], points[i] (n_points[i] x d_in, device) and grads[i]
 * (device, FP64, parameter layout); losses (device, FP64) receives n_inst x (1 + n_res)
 * values (total, then per residual component; no supervision sets).  Every instance has an
 * identity input embedding (n_freq == 0); widths, depths and point counts may differ.
 * The residual mean of instance i divides by n_points[i] (pde->norm_N is ignored).
 *   params, points, grads: (host) arrays of n_inst device pointers.
 *   tune_table (host, nullable): n_inst pinn_tune entries (chunk_points per instance).
 * Work items are (instance, chunk of points), handed out longest first from an atomic
 * counter; each item runs the forward and the whole backward of its points in one work-
 * group and writes its own FP64 partial sums, which are reduced per instance in item order
 * (the result does not depend on the schedule).  The call uploads its descriptor tables
 * into the workspace and synchronises `stream` once before launching.
 * Workspace from pinn_batched_workspace_bytes. */
int pinn_batched_workspace_bytes(const pinn_net* nets, const pinn_pde* pde,
                                 const int64_t* n_points, int n_inst, int prec,
                                 const pinn_tune* tune_table, size_t* bytes);
/* An instance whose tune entry has chunk_points == -1 takes no part in the persistent
 * launch: after it, on the same stream, it runs the fused step of pinn_residual_bwd (its
 * own launches, a region of the same workspace), with the same loss and gradient layout
 * and the same 1 / n_points[i] mean.  The autotuner uses this where the single-network
 * kernels are faster for a width class. */
int pinn_batched_bwd(const pinn_net* nets, const pinn_pde* pde, const float* const* params,
                     const float* const* points, const int64_t* n_points, int n_inst,
                     int prec, const pinn_tune* tune_table, double* const* grads,
                     double* losses, void* workspace, size_t ws_bytes, pinn_stream_t stream);

/* Per-kernel timing (tracing aid).  While enabled, every kernel launch made by the compute
 * calls of this process is bracketed by HIP events recorded on the call's stream; the
 * events cost a few microseconds per launch and do not synchronise anything.
 * pinn_timing_collect synchronises the recorded events, writes (host) up to max_entries
 * summaries (kernel name, launches, summed milliseconds) in first-seen order, sets
 * *n_entries, and clears the record.  Not for concurrent use from several threads. */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
} pinn_kernel_time;
int pinn_timing_enable(int on);
int pinn_timing_collect(pinn_kernel_time* out, int max_entries, int* n_entries);

/* Static description of an error code. */
const char* pinn_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* PINN_H */
