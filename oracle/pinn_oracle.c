/*
 * pinn_oracle.c -- plain FP64 CPU oracle for the PINN residual loss and its
 * parameter gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares nothing with the
 * HIP path: no header, no helper, no table.  Everything is double precision.
 *
 * What it computes (paper: QPINNACLE, arXiv 2604.15645):
 *   network      -- Sec. 2.2 "Network architecture": z = W a + b per layer, a = sigma(z),
 *                   linear output layer; tanh activation (Sec. 2.2), sine activation
 *                   sin(w0 z) (App. A.5 "Periodic activation function").
 *   embedding    -- Sec. 2.6.1 "Random Fourier features": gamma(x) = [cos(xB), sin(xB)],
 *                   B fixed, cos block first (App. A.2); or Sec. 2.6.3 "strict periodic
 *                   boundary conditions": each periodic input x_k becomes
 *                   [cos(2 pi x_k / P_k), sin(2 pi x_k / P_k)], the other inputs pass
 *                   through, and a period may be a trainable parameter (P_t in Sec. 2.6.3).
 *   factorisation-- Sec. 2.6.2 "Random weight factorization": W = diag(exp s) V for every
 *                   linear layer l = 1..L+1.
 *   residuals    -- Burgers (Sec. 4.3 equation, with a viscosity term nu*u_xx, nu = 0 gives
 *                   the printed inviscid form); 1D Euler in conservative form (Sec. 4.6);
 *                   steady incompressible Navier-Stokes (Sec. 4.4); 2D Maxwell, the
 *                   (E_z, H_x, H_y) system of Sec. 4.8; linear advection (Sec. 4.1,
 *                   u_t + c u_x); Allen-Cahn (Sec. 4.2, u_t - D u_xx + k (u^3 - u)); 2D Euler
 *                   in conservative form, outputs (rho, u, v, p) (Sec. 4.7).  Each
 *                   residual is "left side minus right side" of the printed equation.
 *   loss         -- Sec. 2.3 "Loss function": mean of squared residuals per constraint,
 *                   summed (one mean per residual component, weighted by lambda_c), plus
 *                   value-only supervision terms (initial / boundary data) each with its
 *                   own mean.
 *   gradient     -- d(loss)/d(theta) for every parameter (Sec. 2.3, the quantity the
 *                   optimizer consumes).
 *
 * Method.  The derivatives that enter the residual (first derivatives in every input,
 * and the Laplacian over the inputs in lap_mask) are carried forward through the network
 * as "jets": for every neuron the tuple (value, d/dx_k for each input k, Laplacian).
 * This is the plain chain rule; it gives exactly the quantities the paper obtains with
 * automatic differentiation (Sec. 2.3).  The parameter gradient is then obtained with a
 * reverse sweep through those jets, point by point, accumulating in FP64.  Point blocks
 * of fixed size are summed in block order, so the result does not depend on the number
 * of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_HIDDEN 8
#define OR_MAX_CH 5          /* value + 3 first derivatives + Laplacian */
#define OR_BLOCK 64          /* points per fixed summation block */
static const double OR_PI = 3.14159265358979323846;

enum { OR_OK = 0, OR_E_INVALID = -1, OR_E_UNSUPPORTED = -2, OR_E_NOMEM = -3 };
#define OR_MAX_OUT 4         /* outputs (rho, u, v, p) of the 2D Euler system */
enum { OR_BURGERS = 1, OR_EULER1D = 2, OR_NS2D = 3, OR_MAXWELL = 4, OR_ADVECTION = 5, OR_ALLEN_CAHN = 6,
       OR_EULER2D = 7 };

typedef struct {
  int32_t d_in, d_out, n_hidden;
  int32_t width[OR_MAX_HIDDEN];
  int32_t act;      /* 0: tanh, 1: sin(w0 z) */
  double w0;
  int32_t n_freq;   /* 0: identity embedding, else Fourier features with m = n_freq */
  int32_t rwf;      /* 1: every linear layer stored as (V, s), W = diag(exp s) V */
  int32_t has_bias;
  int32_t periodic_mask;     /* bit k: input k enters as [cos, sin](2 pi x_k / P_k) */
  int32_t period_train_mask; /* bit k: P_k is a trainable parameter (after the layers) */
  double period[3];          /* P_k of the periodic inputs that are not trained */
} or_net;

typedef struct {
  int32_t pde_id;
  int32_t lap_mask;     /* bit k set: input k belongs to the Laplacian set */
  double coef[4];       /* Burgers nu | Euler gamma | NS Re | Maxwell eps, mu | advection c |
                           Allen-Cahn D, k | 2D Euler gamma */
  double lambda_res[OR_MAX_OUT];
  double norm_N;        /* divisor of the residual mean; 0 means "number of points" */
} or_pde;

typedef struct {
  const double* points;   /* n x d_in */
  const double* targets;  /* n x d_out */
  int64_t n;
  int32_t out_mask;       /* bit o set: output o is supervised */
  double lambda;
} or_anchor;

/* ------------------------------------------------------------------ layout */

static int n_layers(const or_net* net) { return net->n_hidden + 1; }

static int embed_width(const or_net* net) {
  if (net->periodic_mask) {
    int e = 0;
    for (int k = 0; k < net->d_in; ++k) e += (net->periodic_mask >> k) & 1 ? 2 : 1;
    return e;
  }
  return net->n_freq > 0 ? 2 * net->n_freq : net->d_in;
}

/* Trainable periods: one parameter each, after every layer's parameters, in input order. */
static int n_train_periods(const or_net* net) {
  int n = 0;
  for (int k = 0; k < net->d_in; ++k) n += (net->period_train_mask >> k) & 1;
  return n;
}

static int layer_in(const or_net* net, int l) {
  return l == 0 ? embed_width(net) : net->width[l - 1];
}

static int layer_out(const or_net* net, int l) {
  return l == net->n_hidden ? net->d_out : net->width[l];
}

/* Offsets of W (or V), s and b of layer l in the flat parameter vector.
 * Per layer: [W or V (n_out x n_in, row-major)] [s (n_out) if rwf] [b (n_out) if bias]. */
static int64_t layer_offsets(const or_net* net, int l, int64_t* off_w, int64_t* off_s,
                             int64_t* off_b) {
  int64_t off = 0;
  for (int j = 0; j <= l; ++j) {
    int64_t ni = layer_in(net, j), no = layer_out(net, j);
    int64_t ow = off;
    off += no * ni;
    int64_t os = -1, ob = -1;
    if (net->rwf) { os = off; off += no; }
    if (net->has_bias) { ob = off; off += no; }
    if (j == l) {
      if (off_w) *off_w = ow;
      if (off_s) *off_s = os;
      if (off_b) *off_b = ob;
    }
  }
  return off;
}

int64_t or_param_count(const or_net* net) {
  return layer_offsets(net, n_layers(net) - 1, 0, 0, 0) + n_train_periods(net);
}

/* Period of every input (0 for inputs that pass through). */
static void input_periods(const or_net* net, const double* params, double* per) {
  int64_t t = layer_offsets(net, n_layers(net) - 1, 0, 0, 0);
  for (int k = 0; k < 3; ++k) per[k] = 0.0;
  for (int k = 0; k < net->d_in; ++k) {
    if (!((net->periodic_mask >> k) & 1)) continue;
    per[k] = (net->period_train_mask >> k) & 1 ? params[t++] : net->period[k];
  }
}

static int n_channels(const or_net* net, int lap_mask) {
  return 1 + net->d_in + (lap_mask != 0 ? 1 : 0);
}

static int n_residuals(int pde_id) {
  if (pde_id == OR_EULER2D) return 4;
  return pde_id == OR_EULER1D || pde_id == OR_NS2D || pde_id == OR_MAXWELL ? 3 : 1;
}

static int check_net(const or_net* net, int lap_mask) {
  if (!net) return OR_E_INVALID;
  if (net->d_in < 1 || net->d_in > 3 || net->d_out < 1 || net->d_out > OR_MAX_OUT) return OR_E_INVALID;
  if (net->n_hidden < 0 || net->n_hidden > OR_MAX_HIDDEN) return OR_E_INVALID;
  for (int l = 0; l < net->n_hidden; ++l)
    if (net->width[l] < 1 || net->width[l] > 4096) return OR_E_INVALID;
  if (net->act != 0 && net->act != 1) return OR_E_INVALID;
  if (net->n_freq < 0 || net->n_freq > 4096) return OR_E_INVALID;
  if (lap_mask & ~((1 << net->d_in) - 1)) return OR_E_INVALID;
  const int all = (1 << net->d_in) - 1;
  if ((net->periodic_mask & ~all) || (net->period_train_mask & ~net->periodic_mask)) return OR_E_INVALID;
  if (net->periodic_mask && net->n_freq > 0) return OR_E_UNSUPPORTED;
  for (int k = 0; k < net->d_in; ++k)
    if ((net->periodic_mask >> k) & 1 && !((net->period_train_mask >> k) & 1) && !(net->period[k] != 0.0))
      return OR_E_INVALID;
  return OR_OK;
}

/* -------------------------------------------------------- effective weights */

/* W_l = diag(exp s_l) V_l (Sec. 2.6.2) or W_l itself; b_l or 0. */
typedef struct {
  double* w[OR_MAX_HIDDEN + 1];
  double* b[OR_MAX_HIDDEN + 1];
} or_weights;

static int build_weights(const or_net* net, const double* params, or_weights* ow) {
  memset(ow, 0, sizeof(*ow));
  for (int l = 0; l < n_layers(net); ++l) {
    int64_t ni = layer_in(net, l), no = layer_out(net, l);
    int64_t offw, offs, offb;
    layer_offsets(net, l, &offw, &offs, &offb);
    ow->w[l] = (double*)malloc(sizeof(double) * no * ni);
    ow->b[l] = (double*)calloc((size_t)no, sizeof(double));
    if (!ow->w[l] || !ow->b[l]) return OR_E_NOMEM;
    for (int64_t i = 0; i < no; ++i) {
      double scale = net->rwf ? exp(params[offs + i]) : 1.0;
      for (int64_t j = 0; j < ni; ++j) ow->w[l][i * ni + j] = scale * params[offw + i * ni + j];
      if (net->has_bias) ow->b[l][i] = params[offb + i];
    }
  }
  return OR_OK;
}

static void free_weights(const or_net* net, or_weights* ow) {
  for (int l = 0; l < n_layers(net); ++l) {
    free(ow->w[l]);
    free(ow->b[l]);
  }
}

/* ------------------------------------------------------------- activation */

/* sigma and its first three derivatives at z. */
static void act_derivs(const or_net* net, double z, double* s0, double* s1, double* s2,
                       double* s3) {
  if (net->act == 0) {
    double t = tanh(z);
    double d1 = 1.0 - t * t;
    *s0 = t;
    *s1 = d1;
    *s2 = -2.0 * t * d1;
    *s3 = d1 * (6.0 * t * t - 2.0);
  } else {
    double w = net->w0, sn = sin(w * z), cs = cos(w * z);
    *s0 = sn;
    *s1 = w * cs;
    *s2 = -w * w * sn;
    *s3 = -w * w * w * cs;
  }
}

/* --------------------------------------------------------------- jets */

/* Embedding jets of one point: A0[j*C + c].  Identity: value x_j, d/dx_k = [j == k],
 * Laplacian 0.  Fourier features (Sec. 2.6.1): v_j = sum_k x_k B[k][j];
 * feature j < m is cos(v_j), feature m + j is sin(v_j); their derivatives follow from
 * the chain rule.  Periodic inputs (Sec. 2.6.3): per[k] is the period P_k. */
static void embed_point(const or_net* net, int lap_mask, const double* B, const double* per,
                        const double* x, double* A0, int C) {
  int d = net->d_in, e = embed_width(net);
  memset(A0, 0, sizeof(double) * (size_t)e * C);
  if (net->periodic_mask) {
    /* Sec. 2.6.3: omega = 2 pi / P_k; cos(omega x_k) and sin(omega x_k) depend on x_k
     * alone, so their only derivative channel is k (and the Laplacian if k is in S). */
    int f = 0;
    for (int k = 0; k < d; ++k) {
      if (!((net->periodic_mask >> k) & 1)) {
        A0[f * C + 0] = x[k];
        A0[f * C + 1 + k] = 1.0;
        ++f;
        continue;
      }
      double w = 2.0 * OR_PI / per[k], cv = cos(w * x[k]), sv = sin(w * x[k]);
      double* ac = A0 + (size_t)f * C;
      double* as = A0 + (size_t)(f + 1) * C;
      ac[0] = cv;
      as[0] = sv;
      ac[1 + k] = -w * sv;
      as[1 + k] = w * cv;
      if (lap_mask & (1 << k)) {
        ac[1 + d] = -w * w * cv;
        as[1 + d] = -w * w * sv;
      }
      f += 2;
    }
    return;
  }
  if (net->n_freq == 0) {
    for (int j = 0; j < d; ++j) {
      A0[j * C + 0] = x[j];
      A0[j * C + 1 + j] = 1.0;
    }
    return;
  }
  int m = net->n_freq;
  for (int j = 0; j < m; ++j) {
    double v = 0.0, bl = 0.0;
    for (int k = 0; k < d; ++k) {
      v += x[k] * B[k * m + j];
      if (lap_mask & (1 << k)) bl += B[k * m + j] * B[k * m + j];
    }
    double cv = cos(v), sv = sin(v);
    double* ac = A0 + (size_t)j * C;
    double* as = A0 + (size_t)(m + j) * C;
    ac[0] = cv;
    as[0] = sv;
    for (int k = 0; k < d; ++k) {
      ac[1 + k] = -sv * B[k * m + j];
      as[1 + k] = cv * B[k * m + j];
    }
    if (lap_mask) {
      ac[1 + d] = -cv * bl;
      as[1 + d] = -sv * bl;
    }
  }
}

/* Linear layer on jets: z[i][c] = sum_j W[i][j] a[j][c] (+ b[i] on the value channel). */
static void linear_jets(const double* W, const double* b, int no, int ni, const double* a,
                        double* z, int C) {
  for (int i = 0; i < no; ++i) {
    for (int c = 0; c < C; ++c) {
      double acc = 0.0;
      for (int j = 0; j < ni; ++j) acc += W[(size_t)i * ni + j] * a[(size_t)j * C + c];
      z[(size_t)i * C + c] = acc;
    }
    z[(size_t)i * C + 0] += b[i];
  }
}

/* Activation on jets: a = sigma(z); d_k a = sigma'(z) d_k z;
 * Lap a = sigma''(z) sum_{k in S} (d_k z)^2 + sigma'(z) Lap z. */
static void act_jets(const or_net* net, int lap_mask, int n, const double* z, double* a, int C) {
  int d = net->d_in;
  for (int i = 0; i < n; ++i) {
    const double* zi = z + (size_t)i * C;
    double* ai = a + (size_t)i * C;
    double s0, s1, s2, s3;
    act_derivs(net, zi[0], &s0, &s1, &s2, &s3);
    ai[0] = s0;
    for (int k = 0; k < d; ++k) ai[1 + k] = s1 * zi[1 + k];
    if (lap_mask) {
      double q = 0.0;
      for (int k = 0; k < d; ++k)
        if (lap_mask & (1 << k)) q += zi[1 + k] * zi[1 + k];
      ai[1 + d] = s2 * q + s1 * zi[1 + d];
    }
  }
}

/* Forward pass of one point.  zbuf[l] holds the pre-activation jets of hidden layer l,
 * abuf[l] the activation jets feeding linear layer l (abuf[0] = embedding). */
static void forward_point(const or_net* net, int lap_mask, const or_weights* ow, const double* B,
                          const double* per, const double* x, double** abuf, double** zbuf, double* y,
                          int C) {
  embed_point(net, lap_mask, B, per, x, abuf[0], C);
  int L = net->n_hidden;
  for (int l = 0; l < L; ++l) {
    linear_jets(ow->w[l], ow->b[l], layer_out(net, l), layer_in(net, l), abuf[l], zbuf[l], C);
    act_jets(net, lap_mask, layer_out(net, l), zbuf[l], abuf[l + 1], C);
  }
  linear_jets(ow->w[L], ow->b[L], net->d_out, layer_in(net, L), abuf[L], y, C);
}

/* ------------------------------------------------------------ residuals */

/* Residuals of one point from its output jets y[o*C + c].  Channel c = 1 + k is d/dx_k,
 * channel 1 + d_in the Laplacian.  If rbar is non-null, also the adjoint: the output-jet
 * seed ybar[o*C + c] = sum_r rbar[r] * d r / d y[o][c]. */
static void residual_point(const or_pde* pde, int d_in, const double* y, int C, double* r,
                           const double* rbar, double* ybar) {
  const int LAP = 1 + d_in;
#define Y(o, c) y[(o) * C + (c)]
#define YB(o, c) ybar[(o) * C + (c)]
  switch (pde->pde_id) {
    case OR_BURGERS: { /* inputs (x, t): u_t + u u_x - nu u_xx */
      double nu = pde->coef[0];
      double u = Y(0, 0), ux = Y(0, 1), ut = Y(0, 2), uxx = Y(0, LAP);
      r[0] = ut + u * ux - nu * uxx;
      if (rbar) {
        YB(0, 0) += rbar[0] * ux;
        YB(0, 1) += rbar[0] * u;
        YB(0, 2) += rbar[0];
        YB(0, LAP) += rbar[0] * (-nu);
      }
      break;
    }
    case OR_EULER1D: { /* inputs (x, t), outputs (rho, u, p); conservative form */
      double g = 1.0 / (pde->coef[0] - 1.0);
      double rho = Y(0, 0), rx = Y(0, 1), rt = Y(0, 2);
      double u = Y(1, 0), ux = Y(1, 1), ut = Y(1, 2);
      double p = Y(2, 0), px = Y(2, 1), pt = Y(2, 2);
      /* d/dt(rho) + d/dx(rho u) */
      r[0] = rt + u * rx + rho * ux;
      /* d/dt(rho u) + d/dx(rho u^2 + p) */
      r[1] = u * rt + rho * ut + u * u * rx + 2.0 * rho * u * ux + px;
      /* d/dt(rho E) + d/dx(u (rho E + p)), rho E = g p + rho u^2 / 2 */
      r[2] = g * pt + 0.5 * u * u * rt + rho * u * ut + (g + 1.0) * (u * px + p * ux) +
             0.5 * u * u * u * rx + 1.5 * rho * u * u * ux;
      if (rbar) {
        double b0 = rbar[0], b1 = rbar[1], b2 = rbar[2];
        YB(0, 0) += b0 * ux + b1 * (ut + 2.0 * u * ux) + b2 * (u * ut + 1.5 * u * u * ux);
        YB(0, 1) += b0 * u + b1 * u * u + b2 * 0.5 * u * u * u;
        YB(0, 2) += b0 + b1 * u + b2 * 0.5 * u * u;
        YB(1, 0) += b0 * rx + b1 * (rt + 2.0 * u * rx + 2.0 * rho * ux) +
                    b2 * (u * rt + rho * ut + (g + 1.0) * px + 1.5 * u * u * rx + 3.0 * rho * u * ux);
        YB(1, 1) += b0 * rho + b1 * 2.0 * rho * u + b2 * ((g + 1.0) * p + 1.5 * rho * u * u);
        YB(1, 2) += b1 * rho + b2 * rho * u;
        YB(2, 0) += b2 * (g + 1.0) * ux;
        YB(2, 1) += b1 + b2 * (g + 1.0) * u;
        YB(2, 2) += b2 * g;
      }
      break;
    }
    case OR_NS2D: { /* inputs (x, y), outputs (u, v, p); steady incompressible */
      double inv = 1.0 / pde->coef[0];
      double u = Y(0, 0), ux = Y(0, 1), uy = Y(0, 2), lu = Y(0, LAP);
      double v = Y(1, 0), vx = Y(1, 1), vy = Y(1, 2), lv = Y(1, LAP);
      double px = Y(2, 1), py = Y(2, 2);
      r[0] = ux + vy;
      r[1] = u * ux + v * uy + px - inv * lu;
      r[2] = u * vx + v * vy + py - inv * lv;
      if (rbar) {
        double b0 = rbar[0], b1 = rbar[1], b2 = rbar[2];
        YB(0, 0) += b1 * ux + b2 * vx;
        YB(0, 1) += b0 + b1 * u;
        YB(0, 2) += b1 * v;
        YB(0, LAP) += -b1 * inv;
        YB(1, 0) += b1 * uy + b2 * vy;
        YB(1, 1) += b2 * u;
        YB(1, 2) += b0 + b2 * v;
        YB(1, LAP) += -b2 * inv;
        YB(2, 1) += b1;
        YB(2, 2) += b2;
      }
      break;
    }
    case OR_MAXWELL: { /* inputs (x, y, t), outputs (E_z, H_x, H_y) */
      double ie = 1.0 / pde->coef[0], im = 1.0 / pde->coef[1];
      double ez_x = Y(0, 1), ez_y = Y(0, 2), ez_t = Y(0, 3);
      double hx_y = Y(1, 2), hx_t = Y(1, 3);
      double hy_x = Y(2, 1), hy_t = Y(2, 3);
      r[0] = ez_t - ie * (hy_x - hx_y);
      r[1] = hx_t + im * ez_y;
      r[2] = hy_t - im * ez_x;
      if (rbar) {
        double b0 = rbar[0], b1 = rbar[1], b2 = rbar[2];
        YB(0, 3) += b0;
        YB(2, 1) += -b0 * ie;
        YB(1, 2) += b0 * ie;
        YB(1, 3) += b1;
        YB(0, 2) += b1 * im;
        YB(2, 3) += b2;
        YB(0, 1) += -b2 * im;
      }
      break;
    }
    case OR_ADVECTION: { /* inputs (x, t): u_t + c u_x (Sec. 4.1) */
      double c = pde->coef[0];
      double ux = Y(0, 1), ut = Y(0, 2);
      r[0] = ut + c * ux;
      if (rbar) {
        YB(0, 1) += rbar[0] * c;
        YB(0, 2) += rbar[0];
      }
      break;
    }
    case OR_ALLEN_CAHN: { /* inputs (x, t): u_t - D u_xx + k u^3 - k u (Sec. 4.2) */
      double D = pde->coef[0], k = pde->coef[1];
      double u = Y(0, 0), ut = Y(0, 2), uxx = Y(0, LAP);
      r[0] = ut - D * uxx + k * u * u * u - k * u;
      if (rbar) {
        YB(0, 0) += rbar[0] * (3.0 * k * u * u - k);
        YB(0, 2) += rbar[0];
        YB(0, LAP) += rbar[0] * (-D);
      }
      break;
    }
    case OR_EULER2D: { /* inputs (x, y, t), outputs (rho, u, v, p); conservative form (Sec. 4.7) */
      /* With q = u^2 + v^2 and g = 1 / (gamma - 1): rho E = g p + rho q / 2 and
       * rho E + p = H = (g + 1) p + rho q / 2.  Every conservative derivative is expanded
       * by the product rule into the output jets. */
      double g = 1.0 / (pde->coef[0] - 1.0);
      double rho = Y(0, 0), rx = Y(0, 1), ry = Y(0, 2), rt = Y(0, 3);
      double u = Y(1, 0), ux = Y(1, 1), uy = Y(1, 2), ut = Y(1, 3);
      double v = Y(2, 0), vx = Y(2, 1), vy = Y(2, 2), vt = Y(2, 3);
      double p = Y(3, 0), px = Y(3, 1), py = Y(3, 2), pt = Y(3, 3);
      double q = u * u + v * v;
      double H = (g + 1.0) * p + 0.5 * rho * q;
      double Hx = (g + 1.0) * px + 0.5 * q * rx + rho * (u * ux + v * vx);  /* d/dx of H */
      double Hy = (g + 1.0) * py + 0.5 * q * ry + rho * (u * uy + v * vy);  /* d/dy of H */
      double Et = g * pt + 0.5 * q * rt + rho * (u * ut + v * vt);        /* d/dt of rho E */
      /* d/dt(rho) + d/dx(rho u) + d/dy(rho v) */
      r[0] = rt + (u * rx + rho * ux) + (v * ry + rho * vy);
      /* d/dt(rho u) + d/dx(rho u^2 + p) + d/dy(rho u v) */
      r[1] = (u * rt + rho * ut) + (u * u * rx + 2.0 * rho * u * ux + px) + (u * v * ry + rho * v * uy + rho * u * vy);
      /* d/dt(rho v) + d/dx(rho u v) + d/dy(rho v^2 + p) */
      r[2] = (v * rt + rho * vt) + (u * v * rx + rho * v * ux + rho * u * vx) + (v * v * ry + 2.0 * rho * v * vy + py);
      /* d/dt(rho E) + d/dx(u H) + d/dy(v H) */
      r[3] = Et + (ux * H + u * Hx) + (vy * H + v * Hy);
      if (rbar) {
        double b0 = rbar[0], b1 = rbar[1], b2 = rbar[2], b3 = rbar[3];
        /* adjoints of rho, u, v, p and their derivatives, then of the intermediates */
        double a_r = 0, a_rx = 0, a_ry = 0, a_rt = 0, a_u = 0, a_ux = 0, a_uy = 0, a_ut = 0;
        double a_v = 0, a_vx = 0, a_vy = 0, a_vt = 0, a_p = 0, a_px = 0, a_py = 0, a_pt = 0;
        /* r[0] */
        a_rt += b0; a_u += b0 * rx; a_rx += b0 * u; a_r += b0 * (ux + vy); a_ux += b0 * rho;
        a_v += b0 * ry; a_ry += b0 * v; a_vy += b0 * rho;
        /* r[1] */
        a_u += b1 * (rt + 2.0 * u * rx + 2.0 * rho * ux + v * ry + rho * vy);
        a_r += b1 * (ut + 2.0 * u * ux + v * uy + u * vy);
        a_v += b1 * (u * ry + rho * uy);
        a_rt += b1 * u; a_ut += b1 * rho; a_rx += b1 * u * u; a_ux += b1 * 2.0 * rho * u; a_px += b1;
        a_ry += b1 * u * v; a_uy += b1 * rho * v; a_vy += b1 * rho * u;
        /* r[2] */
        a_v += b2 * (rt + u * rx + rho * ux + 2.0 * v * ry + 2.0 * rho * vy);
        a_r += b2 * (vt + v * ux + u * vx + 2.0 * v * vy);
        a_u += b2 * (v * rx + rho * vx);
        a_rt += b2 * v; a_vt += b2 * rho; a_rx += b2 * u * v; a_ux += b2 * rho * v; a_vx += b2 * rho * u;
        a_ry += b2 * v * v; a_vy += b2 * 2.0 * rho * v; a_py += b2;
        /* r[3] = Et + ux H + u Hx + vy H + v Hy */
        double a_Et = b3, a_H = b3 * (ux + vy), a_Hx = b3 * u, a_Hy = b3 * v, a_q = 0.0;
        a_ux += b3 * H; a_vy += b3 * H; a_u += b3 * Hx; a_v += b3 * Hy;
        /* Et */
        a_pt += g * a_Et; a_q += 0.5 * rt * a_Et; a_rt += 0.5 * q * a_Et; a_r += (u * ut + v * vt) * a_Et;
        a_u += rho * ut * a_Et; a_ut += rho * u * a_Et; a_v += rho * vt * a_Et; a_vt += rho * v * a_Et;
        /* Hx */
        a_px += (g + 1.0) * a_Hx; a_q += 0.5 * rx * a_Hx; a_rx += 0.5 * q * a_Hx; a_r += (u * ux + v * vx) * a_Hx;
        a_u += rho * ux * a_Hx; a_ux += rho * u * a_Hx; a_v += rho * vx * a_Hx; a_vx += rho * v * a_Hx;
        /* Hy */
        a_py += (g + 1.0) * a_Hy; a_q += 0.5 * ry * a_Hy; a_ry += 0.5 * q * a_Hy; a_r += (u * uy + v * vy) * a_Hy;
        a_u += rho * uy * a_Hy; a_uy += rho * u * a_Hy; a_v += rho * vy * a_Hy; a_vy += rho * v * a_Hy;
        /* H */
        a_p += (g + 1.0) * a_H; a_r += 0.5 * q * a_H; a_q += 0.5 * rho * a_H;
        /* q */
        a_u += 2.0 * u * a_q; a_v += 2.0 * v * a_q;
        YB(0, 0) += a_r; YB(0, 1) += a_rx; YB(0, 2) += a_ry; YB(0, 3) += a_rt;
        YB(1, 0) += a_u; YB(1, 1) += a_ux; YB(1, 2) += a_uy; YB(1, 3) += a_ut;
        YB(2, 0) += a_v; YB(2, 1) += a_vx; YB(2, 2) += a_vy; YB(2, 3) += a_vt;
        YB(3, 0) += a_p; YB(3, 1) += a_px; YB(3, 2) += a_py; YB(3, 3) += a_pt;
      }
      break;
    }
    default:
      break;
  }
#undef Y
#undef YB
}

static int check_pde(const or_net* net, const or_pde* pde) {
  if (!pde) return OR_E_INVALID;
  switch (pde->pde_id) {
    case OR_BURGERS:
      if (net->d_in != 2 || net->d_out < 1 || !(pde->lap_mask & 1)) return OR_E_UNSUPPORTED;
      return OR_OK;
    case OR_EULER1D:
      if (net->d_in != 2 || net->d_out != 3 || !(pde->coef[0] > 1.0)) return OR_E_UNSUPPORTED;
      return OR_OK;
    case OR_NS2D:
      if (net->d_in != 2 || net->d_out != 3 || (pde->lap_mask & 3) != 3 || pde->coef[0] == 0.0)
        return OR_E_UNSUPPORTED;
      return OR_OK;
    case OR_MAXWELL:
      if (net->d_in != 3 || net->d_out != 3 || pde->coef[0] == 0.0 || pde->coef[1] == 0.0)
        return OR_E_UNSUPPORTED;
      return OR_OK;
    case OR_ADVECTION:
      if (net->d_in != 2 || net->d_out < 1) return OR_E_UNSUPPORTED;
      return OR_OK;
    case OR_ALLEN_CAHN:
      if (net->d_in != 2 || net->d_out < 1 || pde->lap_mask != 1) return OR_E_UNSUPPORTED;
      return OR_OK;
    case OR_EULER2D:
      if (net->d_in != 3 || net->d_out != 4 || pde->lap_mask != 0 || !(pde->coef[0] > 1.0)) return OR_E_UNSUPPORTED;
      return OR_OK;
    default:
      return OR_E_UNSUPPORTED;
  }
}

/* ------------------------------------------------------------ reverse sweep */

/* Activation adjoint: given the adjoints (abar) of the activation jets and the
 * pre-activation jets z, accumulate the adjoints of z (the transpose of act_jets). */
static void act_jets_adjoint(const or_net* net, int lap_mask, int n, const double* z,
                             const double* abar, double* zbar, int C) {
  int d = net->d_in;
  for (int i = 0; i < n; ++i) {
    const double* zi = z + (size_t)i * C;
    const double* ab = abar + (size_t)i * C;
    double* zb = zbar + (size_t)i * C;
    double s0, s1, s2, s3;
    act_derivs(net, zi[0], &s0, &s1, &s2, &s3);
    /* a0 = s0 */
    double z0b = ab[0] * s1;
    /* a_k = s1 * z_k */
    for (int k = 0; k < d; ++k) {
      z0b += ab[1 + k] * s2 * zi[1 + k];
      zb[1 + k] = ab[1 + k] * s1;
    }
    if (lap_mask) {
      /* aL = s2 * sum_S z_k^2 + s1 * zL */
      double lb = ab[1 + d];
      double q = 0.0;
      for (int k = 0; k < d; ++k)
        if (lap_mask & (1 << k)) {
          q += zi[1 + k] * zi[1 + k];
          zb[1 + k] += lb * s2 * 2.0 * zi[1 + k];
        }
      z0b += lb * (s3 * q + s2 * zi[1 + d]);
      zb[1 + d] = lb * s1;
    }
    zb[0] = z0b;
  }
}

/* Linear-layer adjoint: W_bar[i][j] += sum_c zbar[i][c] a[j][c]; b_bar[i] += zbar[i][0];
 * abar[j][c] = sum_i W[i][j] zbar[i][c] (if abar non-null). */
static void linear_jets_adjoint(const double* W, int no, int ni, const double* a,
                                const double* zbar, double* Wbar, double* bbar, double* abar,
                                int C) {
  for (int i = 0; i < no; ++i) {
    const double* zb = zbar + (size_t)i * C;
    for (int j = 0; j < ni; ++j) {
      const double* aj = a + (size_t)j * C;
      double acc = 0.0;
      for (int c = 0; c < C; ++c) acc += zb[c] * aj[c];
      Wbar[(size_t)i * ni + j] += acc;
    }
    bbar[i] += zb[0];
  }
  if (abar) {
    for (int j = 0; j < ni; ++j)
      for (int c = 0; c < C; ++c) {
        double acc = 0.0;
        for (int i = 0; i < no; ++i) acc += W[(size_t)i * ni + j] * zbar[(size_t)i * C + c];
        abar[(size_t)j * C + c] = acc;
      }
  }
}

/* Work buffers for one thread. */
typedef struct {
  double* a[OR_MAX_HIDDEN + 1];
  double* z[OR_MAX_HIDDEN];
  double* ab;   /* adjoint of activation jets, max width */
  double* zb;   /* adjoint of pre-activation jets, max width */
  double y[OR_MAX_OUT * OR_MAX_CH];
  double yb[OR_MAX_OUT * OR_MAX_CH];
} or_scratch;

static int max_width(const or_net* net) {
  int w = embed_width(net);
  for (int l = 0; l < net->n_hidden; ++l) w = net->width[l] > w ? net->width[l] : w;
  return w > OR_MAX_OUT ? w : OR_MAX_OUT;
}

static int alloc_scratch(const or_net* net, int C, or_scratch* s) {
  memset(s, 0, sizeof(*s));
  size_t mw = (size_t)max_width(net) * C;
  for (int l = 0; l <= net->n_hidden; ++l) {
    s->a[l] = (double*)calloc(mw, sizeof(double));
    if (!s->a[l]) return OR_E_NOMEM;
  }
  for (int l = 0; l < net->n_hidden; ++l) {
    s->z[l] = (double*)calloc(mw, sizeof(double));
    if (!s->z[l]) return OR_E_NOMEM;
  }
  s->ab = (double*)calloc(mw, sizeof(double));
  s->zb = (double*)calloc(mw, sizeof(double));
  return (s->ab && s->zb) ? OR_OK : OR_E_NOMEM;
}

static void free_scratch(const or_net* net, or_scratch* s) {
  for (int l = 0; l <= net->n_hidden; ++l) free(s->a[l]);
  for (int l = 0; l < net->n_hidden; ++l) free(s->z[l]);
  free(s->ab);
  free(s->zb);
}

/* Gradient in "effective" space: per layer W (n_out x n_in) then b (n_out). */
static int64_t eff_offset(const or_net* net, int l) {
  int64_t off = 0;
  for (int j = 0; j < l; ++j) off += (int64_t)layer_out(net, j) * (layer_in(net, j) + 1);
  return off;
}

/* d(loss)/dP_k of the trainable periods (Sec. 2.6.3) from the adjoint abar0 of the
 * embedding jets: omega = 2 pi / P_k, d omega / dP_k = -omega / P_k, and each jet entry of
 * the pair [cos, sin](omega x_k) differentiated in omega.  gper: one slot per trainable
 * period, in input order. */
static void period_grad(const or_net* net, int lap_mask, const double* per, const double* x,
                        const double* abar0, int C, double* gper) {
  int d = net->d_in, f = 0, t = 0;
  for (int k = 0; k < d; ++k) {
    if (!((net->periodic_mask >> k) & 1)) {
      ++f;
      continue;
    }
    if ((net->period_train_mask >> k) & 1) {
      double w = 2.0 * OR_PI / per[k], xk = x[k];
      double cv = cos(w * xk), sv = sin(w * xk);
      const double* bc = abar0 + (size_t)f * C;
      const double* bs = abar0 + (size_t)(f + 1) * C;
      double dw = bc[0] * (-xk * sv) + bs[0] * (xk * cv);
      dw += bc[1 + k] * (-sv - w * xk * cv) + bs[1 + k] * (cv - w * xk * sv);
      if (lap_mask & (1 << k))
        dw += bc[1 + d] * (-2.0 * w * cv + w * w * xk * sv) + bs[1 + d] * (-2.0 * w * sv - w * w * xk * cv);
      gper[t] += dw * (-w / per[k]);
      ++t;
    }
    f += 2;
  }
}

/* Reverse sweep of one point given the output-jet seed in s->yb (forward already done).
 * With trainable periods the adjoint of the embedding jets is formed as well, and the
 * period gradient goes to geff[eff_offset(L + 1) + t]. */
static void backward_point(const or_net* net, int lap_mask, const or_weights* ow, const double* per,
                           const double* x, or_scratch* s, double* geff, int C) {
  int L = net->n_hidden;
  const int ntp = n_train_periods(net);
  /* output layer */
  {
    int ni = layer_in(net, L), no = net->d_out;
    double* g = geff + eff_offset(net, L);
    linear_jets_adjoint(ow->w[L], no, ni, s->a[L], s->yb, g, g + (int64_t)no * ni,
                        L > 0 ? s->ab : 0, C);
  }
  for (int l = L - 1; l >= 0; --l) {
    int ni = layer_in(net, l), no = layer_out(net, l);
    act_jets_adjoint(net, lap_mask, no, s->z[l], s->ab, s->zb, C);
    double* g = geff + eff_offset(net, l);
    linear_jets_adjoint(ow->w[l], no, ni, s->a[l], s->zb, g, g + (int64_t)no * ni,
                        l > 0 || ntp > 0 ? s->ab : 0, C);
  }
  if (ntp > 0) period_grad(net, lap_mask, per, x, s->ab, C, geff + eff_offset(net, L + 1));
}

/* --------------------------------------------------------------- public API */

/* Output jets of the network at n points: jets[(i*d_out + o)*C + c]. */
int or_forward_jets(const or_net* net, int lap_mask, const double* params, const double* B,
                    const double* pts, int64_t n, double* jets) {
  int rc = check_net(net, lap_mask);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!params || !pts || !jets))) return OR_E_INVALID;
  if (net->n_freq > 0 && !B) return OR_E_INVALID;
  int C = n_channels(net, lap_mask);
  double per[3];
  input_periods(net, params, per);
  or_weights ow;
  rc = build_weights(net, params, &ow);
  if (rc) { free_weights(net, &ow); return rc; }
  int err = 0;
#pragma omp parallel
  {
    or_scratch s;
    if (alloc_scratch(net, C, &s)) {
#pragma omp atomic write
      err = 1;
    } else {
#pragma omp for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        forward_point(net, lap_mask, &ow, B, per, pts + i * net->d_in, s.a, s.z, s.y, C);
        memcpy(jets + i * net->d_out * C, s.y, sizeof(double) * net->d_out * C);
      }
    }
    free_scratch(net, &s);
  }
  free_weights(net, &ow);
  return err ? OR_E_NOMEM : OR_OK;
}

/* Residuals from given output jets (the PDE stage alone, used with analytic jets). */
int or_pde_residual(const or_pde* pde, int d_in, int d_out, const double* jets, int64_t n,
                    double* r) {
  if (!pde || !jets || !r || n < 0) return OR_E_INVALID;
  or_net tmp;
  memset(&tmp, 0, sizeof(tmp));
  tmp.d_in = d_in;
  tmp.d_out = d_out;
  int rc = check_pde(&tmp, pde);
  if (rc) return rc;
  int C = 1 + d_in + (pde->lap_mask != 0 ? 1 : 0);
  int nr = n_residuals(pde->pde_id);
  for (int64_t i = 0; i < n; ++i) residual_point(pde, d_in, jets + i * d_out * C, C, r + i * nr, 0, 0);
  return OR_OK;
}

int or_n_residuals(int pde_id) { return n_residuals(pde_id); }

/* Full loss, per-term losses, residuals and the gradient with respect to every parameter.
 * loss_terms: [total, residual component 0..n_res-1, anchor set 0..n_anchor-1].
 * grad: parameter layout (may be null).  residual: n x n_res (may be null). */
int or_loss_grad(const or_net* net, const or_pde* pde, const double* params, const double* B,
                 const double* pts, int64_t n, const or_anchor* anchors, int n_anchor,
                 double* residual, double* loss_terms, double* grad, int n_threads) {
  int rc = check_net(net, pde ? pde->lap_mask : 0);
  if (rc) return rc;
  rc = check_pde(net, pde);
  if (rc) return rc;
  if (n < 0 || n_anchor < 0 || n_anchor > 8 || !loss_terms || !params) return OR_E_INVALID;
  if (n > 0 && !pts) return OR_E_INVALID;
  if (net->n_freq > 0 && !B) return OR_E_INVALID;
  for (int a = 0; a < n_anchor; ++a)
    if (anchors[a].n < 0 || (anchors[a].n > 0 && (!anchors[a].points || !anchors[a].targets)))
      return OR_E_INVALID;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
  const int lap = pde->lap_mask;
  const int C = n_channels(net, lap);
  const int nr = n_residuals(pde->pde_id);
  const int d = net->d_in, dout = net->d_out;
  const double N = pde->norm_N > 0 ? pde->norm_N : (double)n;
  const int ntp = n_train_periods(net);
  const int64_t neff = eff_offset(net, net->n_hidden + 1) + ntp;
  double per[3];
  input_periods(net, params, per);

  or_weights ow;
  rc = build_weights(net, params, &ow);
  if (rc) { free_weights(net, &ow); return rc; }

  /* Segments: 0 = residual points, 1 + a = anchor set a.  Every segment is cut into
   * fixed blocks; blocks are processed in parallel in batches and summed in order. */
  int nseg = 1 + n_anchor;
  int64_t seg_n[9], seg_blocks[9], seg_first[9];
  int64_t nblocks = 0;
  for (int s = 0; s < nseg; ++s) {
    seg_n[s] = s == 0 ? n : anchors[s - 1].n;
    seg_blocks[s] = (seg_n[s] + OR_BLOCK - 1) / OR_BLOCK;
    seg_first[s] = nblocks;
    nblocks += seg_blocks[s];
  }
  int nterm = 1 + nr + n_anchor;
  double term[1 + OR_MAX_OUT + 8];
  memset(term, 0, sizeof(term));
  double* geff = grad ? (double*)calloc((size_t)neff, sizeof(double)) : 0;

  int threads = 1;
#ifdef _OPENMP
  threads = omp_get_max_threads();
#endif
  int64_t batch = 4 * (int64_t)threads;
  double* bgrad = grad ? (double*)malloc(sizeof(double) * (size_t)(batch * neff)) : 0;
  double* bterm = (double*)malloc(sizeof(double) * (size_t)(batch * nterm));
  int err = (grad && (!geff || !bgrad)) || !bterm;

  for (int64_t b0 = 0; b0 < nblocks && !err; b0 += batch) {
    int64_t b1 = b0 + batch < nblocks ? b0 + batch : nblocks;
#pragma omp parallel
    {
      or_scratch s;
      int ok = alloc_scratch(net, C, &s) == OR_OK;
      if (!ok) {
#pragma omp atomic write
        err = 1;
      }
#pragma omp for schedule(dynamic, 1)
      for (int64_t b = b0; b < b1; ++b) {
        if (!ok) continue;
        double* g = bgrad ? bgrad + (b - b0) * neff : 0;
        double* t = bterm + (b - b0) * nterm;
        if (g) memset(g, 0, sizeof(double) * (size_t)neff);
        memset(t, 0, sizeof(double) * (size_t)nterm);
        int seg = 0;
        while (seg + 1 < nseg && b >= seg_first[seg + 1]) ++seg;
        int64_t i0 = (b - seg_first[seg]) * OR_BLOCK;
        int64_t i1 = i0 + OR_BLOCK < seg_n[seg] ? i0 + OR_BLOCK : seg_n[seg];
        for (int64_t i = i0; i < i1; ++i) {
          const double* x = seg == 0 ? pts + i * d : anchors[seg - 1].points + i * d;
          forward_point(net, lap, &ow, B, per, x, s.a, s.z, s.y, C);
          memset(s.yb, 0, sizeof(s.yb));
          if (seg == 0) {
            double r[OR_MAX_OUT], rb[OR_MAX_OUT];
            residual_point(pde, d, s.y, C, r, 0, 0);
            for (int c = 0; c < nr; ++c) {
              t[1 + c] += pde->lambda_res[c] * r[c] * r[c] / N;
              rb[c] = 2.0 * pde->lambda_res[c] * r[c] / N;
              if (residual) residual[i * nr + c] = r[c];
            }
            if (g) residual_point(pde, d, s.y, C, r, rb, s.yb);
          } else {
            const or_anchor* an = &anchors[seg - 1];
            double Ns = (double)an->n;
            for (int o = 0; o < dout; ++o) {
              if (!(an->out_mask & (1 << o))) continue;
              double diff = s.y[o * C + 0] - an->targets[i * dout + o];
              t[1 + nr + seg - 1] += an->lambda * diff * diff / Ns;
              s.yb[o * C + 0] = 2.0 * an->lambda * diff / Ns;
            }
          }
          if (g) backward_point(net, lap, &ow, per, x, &s, g, C);
        }
      }
      free_scratch(net, &s);
    }
    if (err) break;
    for (int64_t b = b0; b < b1; ++b) {
      const double* t = bterm + (b - b0) * nterm;
      for (int k = 1; k < nterm; ++k) term[k] += t[k];
      if (geff) {
        const double* g = bgrad + (b - b0) * neff;
        for (int64_t k = 0; k < neff; ++k) geff[k] += g[k];
      }
    }
  }

  if (!err) {
    term[0] = 0.0;
    for (int k = 1; k < nterm; ++k) term[0] += term[k];
    memcpy(loss_terms, term, sizeof(double) * (size_t)nterm);
    if (grad) {
      /* Map effective-space gradient to the parameter layout.  With weight factorisation
       * (Sec. 2.6.2) W_ij = exp(s_i) V_ij, so dL/dV_ij = exp(s_i) dL/dW_ij and
       * dL/ds_i = sum_j dL/dW_ij * W_ij. */
      for (int l = 0; l <= net->n_hidden; ++l) {
        int64_t ni = layer_in(net, l), no = layer_out(net, l);
        int64_t offw, offs, offb;
        layer_offsets(net, l, &offw, &offs, &offb);
        const double* gw = geff + eff_offset(net, l);
        const double* gb = gw + no * ni;
        for (int64_t i = 0; i < no; ++i) {
          double es = net->rwf ? exp(params[offs + i]) : 1.0;
          double ssum = 0.0;
          for (int64_t j = 0; j < ni; ++j) {
            grad[offw + i * ni + j] = es * gw[i * ni + j];
            ssum += gw[i * ni + j] * ow.w[l][i * ni + j];
          }
          if (net->rwf) grad[offs + i] = ssum;
          if (net->has_bias) grad[offb + i] = gb[i];
        }
      }
      const int64_t np_layers = layer_offsets(net, n_layers(net) - 1, 0, 0, 0);
      for (int t = 0; t < ntp; ++t) grad[np_layers + t] = geff[eff_offset(net, net->n_hidden + 1) + t];
    }
  }
  free(geff);
  free(bgrad);
  free(bterm);
  free_weights(net, &ow);
  return err ? OR_E_NOMEM : OR_OK;
}
