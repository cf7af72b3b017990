"""ctypes shim over the FP64 CPU oracle (pinn_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path never imports this module,
and this module never imports the product package.

Network and PDE descriptions are plain dicts (the same dicts the seeded input
generator produces), so that nothing but data is shared with the HIP path:

  net = {"d_in", "d_out", "widths": [..], "act": "tanh"|"sin", "w0", "n_freq",
         "rwf", "has_bias", "periodic_mask", "period_train_mask", "period": [..3]}
  pde = {"pde": "burgers"|"euler1d"|"ns2d"|"maxwell"|"advection"|"allen_cahn"|"euler2d",
         "lap_mask", "coef": [..4], "lambda_res": [..4], "norm_N"}
Arrays may be float32; they are promoted to float64 before the call.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pinn_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CLANG = "/opt/rocm/llvm/bin/clang"

PDE_IDS = {"burgers": 1, "euler1d": 2, "ns2d": 3, "maxwell": 4, "advection": 5, "allen_cahn": 6,
           "euler2d": 7}
MAX_RES = 4
ACTS = {"tanh": 0, "sin": 1}


class _Net(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_int32), ("d_out", ctypes.c_int32),
                ("n_hidden", ctypes.c_int32), ("width", ctypes.c_int32 * 8),
                ("act", ctypes.c_int32), ("w0", ctypes.c_double),
                ("n_freq", ctypes.c_int32), ("rwf", ctypes.c_int32),
                ("has_bias", ctypes.c_int32), ("periodic_mask", ctypes.c_int32),
                ("period_train_mask", ctypes.c_int32), ("period", ctypes.c_double * 3)]


class _Pde(ctypes.Structure):
    _fields_ = [("pde_id", ctypes.c_int32), ("lap_mask", ctypes.c_int32),
                ("coef", ctypes.c_double * 4), ("lambda_res", ctypes.c_double * MAX_RES),
                ("norm_N", ctypes.c_double)]


class _Anchor(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("targets", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("out_mask", ctypes.c_int32),
                ("lambda_", ctypes.c_double)]


def build_sanitized(out_dir):
    """The oracle with AddressSanitizer and UndefinedBehaviorSanitizer (clang, no OpenMP),
    for running the CPU tests under the sanitizers; returns the library path."""
    out = os.path.join(out_dir, "liboracle_asan.so")
    subprocess.check_call([CLANG, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-std=c99", "-o", out,
                           SRC, "-lm"])
    return out


def build(force=False):
    """Compile the oracle with gcc (plain -O2, IEEE semantics, OpenMP)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("PINN_ORACLE_LIB")   # a prebuilt variant (the sanitizer build)
        if not path:
            path = build()
        L = ctypes.CDLL(path)
        L.or_param_count.restype = ctypes.c_int64
        L.or_param_count.argtypes = [ctypes.POINTER(_Net)]
        L.or_forward_jets.restype = ctypes.c_int
        L.or_forward_jets.argtypes = [ctypes.POINTER(_Net), ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p]
        L.or_pde_residual.restype = ctypes.c_int
        L.or_pde_residual.argtypes = [ctypes.POINTER(_Pde), ctypes.c_int, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        L.or_n_residuals.restype = ctypes.c_int
        L.or_n_residuals.argtypes = [ctypes.c_int]
        L.or_loss_grad.restype = ctypes.c_int
        L.or_loss_grad.argtypes = [ctypes.POINTER(_Net), ctypes.POINTER(_Pde),
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int64, ctypes.POINTER(_Anchor), ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int]
        _lib = L
    return _lib


def _net(spec):
    n = _Net()
    n.d_in = int(spec["d_in"])
    n.d_out = int(spec["d_out"])
    widths = list(spec["widths"])
    n.n_hidden = len(widths)
    for i, w in enumerate(widths):
        n.width[i] = int(w)
    n.act = ACTS[spec.get("act", "tanh")]
    n.w0 = float(spec.get("w0", 1.0))
    n.n_freq = int(spec.get("n_freq", 0))
    n.rwf = int(bool(spec.get("rwf", False)))
    n.has_bias = int(bool(spec.get("has_bias", True)))
    n.periodic_mask = int(spec.get("periodic_mask", 0))
    n.period_train_mask = int(spec.get("period_train_mask", 0))
    per = list(spec.get("period", [])) + [0.0] * 3
    for k in range(3):
        n.period[k] = float(per[k])
    return n


def _pde(spec):
    p = _Pde()
    p.pde_id = PDE_IDS[spec["pde"]]
    p.lap_mask = int(spec.get("lap_mask", 0))
    coef = list(spec.get("coef", [])) + [0.0] * 4
    for i in range(4):
        p.coef[i] = float(coef[i])
    lam = list(spec.get("lambda_res", [])) + [1.0] * MAX_RES
    for i in range(MAX_RES):
        p.lambda_res[i] = float(lam[i])
    p.norm_N = float(spec.get("norm_N", 0.0))
    return p


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data


def n_channels(net_spec, lap_mask):
    return 1 + int(net_spec["d_in"]) + (1 if lap_mask else 0)


def n_residuals(pde_name):
    return int(lib().or_n_residuals(PDE_IDS[pde_name]))


def param_count(net_spec):
    n = _net(net_spec)
    return int(lib().or_param_count(ctypes.byref(n)))


def forward_jets(net_spec, lap_mask, params, B, pts):
    """Output jets, shape (n, d_out, C): channel 0 value, 1+k d/dx_k, 1+d_in Laplacian."""
    n = _net(net_spec)
    params = _f64(params)
    pts = _f64(pts).reshape(-1, n.d_in)
    Bv = None if B is None else _f64(B)
    C = n_channels(net_spec, lap_mask)
    out = np.zeros((pts.shape[0], n.d_out, C))
    rc = lib().or_forward_jets(ctypes.byref(n), int(lap_mask), _ptr(params), _ptr(Bv), _ptr(pts),
                               pts.shape[0], _ptr(out))
    if rc != 0:
        raise ValueError("or_forward_jets failed: %d" % rc)
    return out


def pde_residual(pde_spec, d_in, d_out, jets):
    """Residuals (n, n_res) of the PDE stage alone, from given output jets (n, d_out, C)."""
    p = _pde(pde_spec)
    jets = _f64(jets)
    nres = n_residuals(pde_spec["pde"])
    out = np.zeros((jets.shape[0], nres))
    rc = lib().or_pde_residual(ctypes.byref(p), int(d_in), int(d_out), _ptr(jets), jets.shape[0],
                               _ptr(out))
    if rc != 0:
        raise ValueError("or_pde_residual failed: %d" % rc)
    return out


def loss_grad(net_spec, pde_spec, params, B, pts, anchors=(), want_grad=True,
              want_residual=True, n_threads=0):
    """Loss terms, residuals and the parameter gradient in FP64.

    anchors: sequence of dicts {"points" (n x d_in), "targets" (n x d_out), "out_mask",
    "lambda"}.  Returns dict(loss=[total, res_0.., anchor_0..], residual, grad)."""
    n = _net(net_spec)
    p = _pde(pde_spec)
    params = _f64(params)
    pts = _f64(pts).reshape(-1, n.d_in)
    Bv = None if B is None else _f64(B)
    nres = n_residuals(pde_spec["pde"])
    keep = []
    arr = (_Anchor * max(1, len(anchors)))()
    for i, a in enumerate(anchors):
        ap = _f64(a["points"]).reshape(-1, n.d_in)
        at = _f64(a["targets"]).reshape(-1, n.d_out)
        keep += [ap, at]
        arr[i].points = ap.ctypes.data
        arr[i].targets = at.ctypes.data
        arr[i].n = ap.shape[0]
        arr[i].out_mask = int(a.get("out_mask", 1))
        arr[i].lambda_ = float(a.get("lambda", 1.0))
    loss = np.zeros(1 + nres + len(anchors))
    res = np.zeros((pts.shape[0], nres)) if want_residual else None
    grad = np.zeros(param_count(net_spec)) if want_grad else None
    rc = lib().or_loss_grad(ctypes.byref(n), ctypes.byref(p), _ptr(params), _ptr(Bv), _ptr(pts),
                            pts.shape[0], arr, len(anchors), _ptr(res), _ptr(loss), _ptr(grad),
                            int(n_threads))
    if rc != 0:
        raise ValueError("or_loss_grad failed: %d" % rc)
    return {"loss": loss, "residual": res, "grad": grad}


def term_grads(net_spec, pde_spec, params, B, pts, anchors=()):
    """Gradient of each loss term on its own (Sec. 2.6.4 balances the terms by the norms
    of these): term 0 is the residual term (every residual component with its weight
    lambda_c), term 1 + a the supervision set a (with its weight).  Each term involves
    only its own points, so its gradient is the gradient of the loss evaluated on those
    points alone.  Returns (loss terms as loss_grad does, list of gradients)."""
    d_in = int(net_spec["d_in"])
    full = loss_grad(net_spec, pde_spec, params, B, pts, anchors, want_residual=False)
    grads = [loss_grad(net_spec, pde_spec, params, B, pts, (), want_residual=False)["grad"]]
    for a in anchors:
        grads.append(loss_grad(net_spec, pde_spec, params, B, np.zeros((0, d_in)), [a],
                               want_residual=False)["grad"])
    return full["loss"], grads


def balance_update(grads, lam, alpha=0.9, eps=1e-9):
    """Loss-balancing weights of Sec. 2.6.4: with n_t the 2-norm of term t's gradient,
    lambda_hat_t = (sum_s n_s) / (n_t + eps) (eps guards a vanishing gradient, as the code
    listing of the paper does), and the weights move by an exponential moving average,
    lambda_t <- alpha lambda_t + (1 - alpha) lambda_hat_t.  Returns (lambda, lambda_hat)."""
    norms = np.array([np.sqrt(np.sum(np.asarray(g, dtype=np.float64) ** 2)) for g in grads])
    hat = norms.sum() / (norms + eps)
    return alpha * np.asarray(lam, dtype=np.float64) + (1.0 - alpha) * hat, hat


def causal_weights(bin_losses, eps):
    """Temporal-causality weights of Sec. 2.6.8: w_1 = 1 and
    w_i = exp(-eps * sum_{k < i} L^k) for the later time segments."""
    L = np.asarray(bin_losses, dtype=np.float64)
    return np.exp(-eps * np.concatenate([[0.0], np.cumsum(L)[:-1]]))


def causal_loss_grad(net_spec, pde_spec, params, B, pts, bin_n, eps, anchors=()):
    """The causality-weighted residual loss of Sec. 2.6.8 and its gradient.  The residual
    points come in M consecutive time segments of bin_n[i] points; L^i is the residual loss
    of segment i alone (every component with its weight, mean over the segment's points),
    w_i the causality weights, and L_pde = (1/M) sum_i w_i L^i.  The weights are held fixed
    in the gradient (the paper computes them from the losses and does not differentiate
    them).  Supervision sets add their own terms as in loss_grad.
    Returns dict(loss=[total, residual component 0.., set 0..], grad, bin_loss, w)."""
    M = len(bin_n)
    nres = n_residuals(pde_spec["pde"])
    d_in = int(net_spec["d_in"])
    starts = np.concatenate([[0], np.cumsum(bin_n)])
    per = [loss_grad(net_spec, pde_spec, params, B, pts[starts[i]:starts[i + 1]], (), want_residual=False)
           for i in range(M)]
    Lbin = np.array([r["loss"][0] for r in per])
    w = causal_weights(Lbin, eps)
    loss = np.zeros(1 + nres + len(anchors))
    grad = np.zeros(param_count(net_spec))
    for i in range(M):
        loss[1:1 + nres] += w[i] / M * per[i]["loss"][1:1 + nres]
        grad += w[i] / M * per[i]["grad"]
    for a_i, a in enumerate(anchors):
        r = loss_grad(net_spec, pde_spec, params, B, np.zeros((0, d_in)), [a], want_residual=False)
        loss[1 + nres + a_i] = r["loss"][1 + nres]
        grad += r["grad"]
    loss[0] = loss[1:].sum()
    return {"loss": loss, "grad": grad, "bin_loss": Lbin, "w": w}
