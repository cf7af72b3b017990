"""Seeded synthetic inputs for the PINN residual + gradient path.

This module only draws numbers: network and PDE descriptions (plain dicts), FP32
parameters, the fixed Fourier matrix, collocation points and value-supervision
(anchor) sets.  It holds none of the method's arithmetic, so that the HIP path and
the FP64 oracle can both consume the same inputs without sharing code.

Workload recipes (the paper's datasets and reference solutions are not available;
these synthetic sets stand in for its benchmark problems with their shapes):
  burgers  1D viscous Burgers (Sec. 4.3 form plus nu = 0.01/pi), MLP 2 -> 3x32 tanh -> 1,
           4,096 uniform points on [-1,1]x[0,1] plus 128 initial points (target -sin(pi x))
           and 128 boundary points (x = +-1, target 0).
  euler    1D Euler (Sec. 4.6), Fourier features m = 64, sigma = 1, MLP 4x64 tanh -> 3,
           65,536 uniform points on [0,1]x[0,0.2], gamma = 1.4.
  ns       steady Navier-Stokes (Sec. 4.4), Re = 100, MLP 2 -> 5x128 tanh -> 3 with weight
           factorisation (Sec. 2.6.2, s ~ N(1, 0.1)), 262,144 uniform points on [0,1]^2.
  maxwell  2D Maxwell (Sec. 4.8), Fourier features m = 128, sigma = 2, MLP 6x256 sin -> 3,
           1,048,576 uniform points on [0,1]^3, eps = mu = 1.
  sweep    64 independent Burgers networks, widths {32,64,128,256}, depths 3..6,
           4k..128k points each.
  advection  linear advection u_t + c u_x (Sec. 4.1, c = 10), MLP 2 -> 4x64 tanh -> 1,
           16,384 uniform points on [0,2pi]x[0,1] plus 128 initial points (target sin x).
  allen_cahn Allen-Cahn u_t - 1e-4 u_xx + 5 u^3 - 5 u (Sec. 4.2), MLP 2 -> 4x128 tanh -> 1,
           16,384 uniform points on [-1,1]x[0,1] plus 128 initial points (target x^2 cos(pi x)).
  euler2d  2D Euler in conservative form (Sec. 4.7, the four-quadrant Riemann problem of its
           configuration 6, gamma = 1.4), x and y through the strict periodic pair with
           P = 1 (Sec. 2.6.3), weight factorisation, MLP 5 -> 4x128 tanh -> 4 (the paper
           prints no width or depth for it), 262,144 = 64^3 uniform points on
           [0,1]^2 x [0,0.3] plus 256 initial points carrying the four quadrant states
           (rho, u, v, p) as targets of all four outputs.
Weights are Xavier-normal (std = sqrt(2 / (fan_in + fan_out))), biases zero; with
perturb=True biases (and factorisation scales) get random non-zero values so that
parity tests exercise every parameter path.
"""
import math

import numpy as np

SEED_BASE = 15645

CONFIGS = {
    "burgers": dict(
        net=dict(d_in=2, d_out=1, widths=[32, 32, 32], act="tanh", w0=1.0, n_freq=0,
                 rwf=False, has_bias=True),
        pde=dict(pde="burgers", lap_mask=1, coef=[0.01 / math.pi, 0, 0, 0],
                 lambda_res=[1.0, 1.0, 1.0], norm_N=0.0),
        box=[(-1.0, 1.0), (0.0, 1.0)], n_points=4096, rff_sigma=0.0, index=0),
    "euler": dict(
        net=dict(d_in=2, d_out=3, widths=[64, 64, 64, 64], act="tanh", w0=1.0, n_freq=64,
                 rwf=False, has_bias=True),
        pde=dict(pde="euler1d", lap_mask=0, coef=[1.4, 0, 0, 0], lambda_res=[1.0, 1.0, 1.0],
                 norm_N=0.0),
        box=[(0.0, 1.0), (0.0, 0.2)], n_points=65536, rff_sigma=1.0, index=1),
    "ns": dict(
        net=dict(d_in=2, d_out=3, widths=[128] * 5, act="tanh", w0=1.0, n_freq=0, rwf=True,
                 has_bias=True),
        pde=dict(pde="ns2d", lap_mask=3, coef=[100.0, 0, 0, 0], lambda_res=[1.0, 1.0, 1.0],
                 norm_N=0.0),
        box=[(0.0, 1.0), (0.0, 1.0)], n_points=262144, rff_sigma=0.0, index=2),
    "maxwell": dict(
        net=dict(d_in=3, d_out=3, widths=[256] * 6, act="sin", w0=1.0, n_freq=128, rwf=False,
                 has_bias=True),
        pde=dict(pde="maxwell", lap_mask=0, coef=[1.0, 1.0, 0, 0], lambda_res=[1.0, 1.0, 1.0],
                 norm_N=0.0),
        box=[(0.0, 1.0), (0.0, 1.0), (0.0, 1.0)], n_points=1048576, rff_sigma=2.0, index=3),
    "advection": dict(
        net=dict(d_in=2, d_out=1, widths=[64, 64, 64, 64], act="tanh", w0=1.0, n_freq=0,
                 rwf=False, has_bias=True),
        pde=dict(pde="advection", lap_mask=0, coef=[10.0, 0, 0, 0], lambda_res=[1.0, 1.0, 1.0],
                 norm_N=0.0),
        box=[(0.0, 2.0 * math.pi), (0.0, 1.0)], n_points=16384, rff_sigma=0.0, index=5),
    "allen_cahn": dict(
        net=dict(d_in=2, d_out=1, widths=[128, 128, 128, 128], act="tanh", w0=1.0, n_freq=0,
                 rwf=False, has_bias=True),
        pde=dict(pde="allen_cahn", lap_mask=1, coef=[1e-4, 5.0, 0, 0], lambda_res=[1.0, 1.0, 1.0],
                 norm_N=0.0),
        box=[(-1.0, 1.0), (0.0, 1.0)], n_points=16384, rff_sigma=0.0, index=6),
    "euler2d": dict(
        net=dict(d_in=3, d_out=4, widths=[128, 128, 128, 128], act="tanh", w0=1.0, n_freq=0,
                 rwf=True, has_bias=True, periodic_mask=3, period_train_mask=0,
                 period=[1.0, 1.0, 0.0]),
        pde=dict(pde="euler2d", lap_mask=0, coef=[1.4, 0, 0, 0],
                 lambda_res=[1.0, 1.0, 1.0, 1.0], norm_N=0.0),
        box=[(0.0, 1.0), (0.0, 1.0), (0.0, 0.3)], n_points=262144, rff_sigma=0.0, index=7),
}

# Sec. 4.7, configuration 6: (rho, u, v, p) in the quadrants x > 0.5 / y > 0.5 and so on
RIEMANN6 = {(1, 1): (1.0, 0.75, -0.5, 1.0), (0, 1): (2.0, 0.75, 0.5, 1.0),
            (0, 0): (1.0, -0.75, 0.5, 1.0), (1, 0): (3.0, -0.75, -0.5, 1.0)}


def embed_width(net):
    """Width of the network input: 2 m Fourier features, or each input once (twice when it
    enters through the periodic [cos, sin] pair)."""
    pm = int(net.get("periodic_mask", 0))
    if pm:
        return sum(2 if (pm >> k) & 1 else 1 for k in range(net["d_in"]))
    return 2 * net["n_freq"] if net.get("n_freq", 0) else net["d_in"]


def n_train_periods(net):
    return bin(int(net.get("period_train_mask", 0))).count("1")


def layer_dims(net):
    """(n_out, n_in) of every linear layer, input side first."""
    e = embed_width(net)
    dims = []
    prev = e
    for w in net["widths"]:
        dims.append((w, prev))
        prev = w
    dims.append((net["d_out"], prev))
    return dims


def param_count(net):
    n = 0
    for no, ni in layer_dims(net):
        n += no * ni + (no if net.get("rwf") else 0) + (no if net.get("has_bias", True) else 0)
    return n + n_train_periods(net)


def init_params(net, rng, perturb=False, rwf_mean=1.0, rwf_std=0.1):
    """Flat FP32 parameters, per layer [W or V (row-major n_out x n_in)] [s] [b], then the
    trainable periods (initial value net["period"][k], in input order)."""
    out = []
    for no, ni in layer_dims(net):
        std = math.sqrt(2.0 / (ni + no))
        out.append(rng.normal(0.0, std, size=no * ni))
        if net.get("rwf"):
            out.append(rng.normal(rwf_mean, rwf_std, size=no))
        if net.get("has_bias", True):
            out.append(rng.normal(0.0, 0.1, size=no) if perturb else np.zeros(no))
    tm = int(net.get("period_train_mask", 0))
    out.append(np.array([net["period"][k] for k in range(net["d_in"]) if (tm >> k) & 1], dtype=np.float64))
    return np.concatenate(out).astype(np.float32)


def uniform_points(rng, box, n):
    cols = [rng.uniform(lo, hi, size=n) for lo, hi in box]
    return np.stack(cols, axis=1).astype(np.float32)


def fourier_matrix(rng, net, sigma):
    if not net.get("n_freq"):
        return None
    return rng.normal(0.0, sigma, size=(net["d_in"], net["n_freq"])).astype(np.float32)


def burgers_anchors(rng, n_ic=128, n_bc=128):
    """Initial data u(x,0) = -sin(pi x) and Dirichlet data u(+-1,t) = 0."""
    x = rng.uniform(-1.0, 1.0, size=n_ic)
    ic_pts = np.stack([x, np.zeros(n_ic)], axis=1).astype(np.float32)
    ic_tgt = (-np.sin(np.pi * ic_pts[:, 0].astype(np.float64))).astype(np.float32)[:, None]
    half = n_bc // 2
    xb = np.concatenate([-np.ones(half), np.ones(n_bc - half)])
    tb = rng.uniform(0.0, 1.0, size=n_bc)
    bc_pts = np.stack([xb, tb], axis=1).astype(np.float32)
    bc_tgt = np.zeros((n_bc, 1), dtype=np.float32)
    return [dict(points=ic_pts, targets=ic_tgt, out_mask=1, **{"lambda": 1.0}),
            dict(points=bc_pts, targets=bc_tgt, out_mask=1, **{"lambda": 1.0})]


def initial_anchors(rng, name, n=128):
    """Initial data u(x, 0) of the advection (sin x) and Allen-Cahn (x^2 cos(pi x)) problems."""
    lo, hi = CONFIGS[name]["box"][0]
    x = rng.uniform(lo, hi, size=n)
    pts = np.stack([x, np.zeros(n)], axis=1).astype(np.float32)
    xd = pts[:, 0].astype(np.float64)
    tgt = np.sin(xd) if name == "advection" else xd * xd * np.cos(np.pi * xd)
    return [dict(points=pts, targets=tgt.astype(np.float32)[:, None], out_mask=1, **{"lambda": 1.0})]


def riemann_anchors(rng, n=256):
    """Initial data of the four-quadrant problem at t = 0, every output supervised."""
    xy = rng.uniform(0.0, 1.0, size=(n, 2))
    pts = np.c_[xy, np.zeros(n)].astype(np.float32)
    tgt = np.array([RIEMANN6[(int(a > 0.5), int(b > 0.5))] for a, b in pts[:, :2]], dtype=np.float32)
    return [dict(points=pts, targets=tgt, out_mask=15, **{"lambda": 1.0})]


def make_case(name, n_points=None, seed=None, perturb=False, anchors=None):
    """One workload: dict(net, pde, params, B, points, anchors)."""
    cfg = CONFIGS[name]
    seed = SEED_BASE + cfg["index"] if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    net = dict(cfg["net"])
    net["widths"] = list(net["widths"])
    pde = dict(cfg["pde"])
    params = init_params(net, rng, perturb=perturb)
    B = fourier_matrix(rng, net, cfg["rff_sigma"])
    n = cfg["n_points"] if n_points is None else n_points
    pts = uniform_points(rng, cfg["box"], n)
    if anchors is None:
        anchors = name in ("burgers", "advection", "allen_cahn", "euler2d")
    anc = []
    if anchors:
        if name == "burgers":
            anc = burgers_anchors(rng)
        elif name == "euler2d":
            anc = riemann_anchors(rng)
        else:
            anc = initial_anchors(rng, name)
    return dict(name=name, net=net, pde=pde, params=params, B=B, points=pts, anchors=anc)


def make_custom(net, pde, box, n_points, seed, sigma=1.0, perturb=True, anchors=()):
    """A workload with an arbitrary network (parity cases of unusual shape)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = init_params(net, rng, perturb=perturb)
    B = fourier_matrix(rng, net, sigma)
    pts = uniform_points(rng, box, n_points)
    return dict(name="custom", net=net, pde=pde, params=params, B=B, points=pts,
                anchors=list(anchors))


SWEEP_SEED = 15650 * 1000
SWEEP_WIDTHS = [32, 64, 128, 256]


def make_sweep(n_inst=64, n_min=4096, n_max=131072, seed_base=SWEEP_SEED, perturb=False,
               scale=1.0):
    """Independent Burgers networks of uneven width, depth and point count.

    Instance i: width SWEEP_WIDTHS[i % 4], depth 3 + (i // 4) % 4, point count uniform in
    [n_min, n_max] rounded to a multiple of 64 (times `scale`, for small test sweeps)."""
    base = CONFIGS["burgers"]
    out = []
    for i in range(n_inst):
        rng = np.random.Generator(np.random.PCG64(seed_base + i))
        width = SWEEP_WIDTHS[i % 4]
        depth = 3 + (i // 4) % 4
        net = dict(base["net"])
        net["widths"] = [width] * depth
        n = int(rng.integers(n_min, n_max + 1))
        n = max(64, int(round(n * scale / 64.0)) * 64)
        params = init_params(net, rng, perturb=perturb)
        pts = uniform_points(rng, base["box"], n)
        out.append(dict(name="sweep%d" % i, net=net, pde=dict(base["pde"]), params=params,
                        B=None, points=pts, anchors=[]))
    return out
