"""ctypes binding of libpinn.so (include/pinn.h), with torch providing device memory and
the current stream.  Argument marshalling only: every step of the computation runs in
the library's HIP kernels.  Raises if the library is missing: there is no fallback."""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# PINN_LIB names another build of the same library (the host-sanitizer build of build.py)
LIB_PATH = os.environ.get("PINN_LIB") or os.path.join(HERE, "libpinn.so")

PDE_IDS = {"burgers": 1, "euler1d": 2, "ns2d": 3, "maxwell": 4, "advection": 5, "allen_cahn": 6,
           "euler2d": 7}
MAX_RES = 4  # residual components (and outputs) a PDE descriptor can carry
ACTS = {"tanh": 0, "sin": 1}
PRECS = {"fp32": 0, "bf16x3": 1, "bf16": 2, "fp64": 3, "fp16x3": 4}
FLAG_CHECK_FINITE = 1

STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported configuration",
          -3: "workspace too small", -4: "non-finite parameter", -5: "HIP runtime error"}


class PinnNet(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_int32), ("d_out", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("width", ctypes.c_int32 * 8), ("act", ctypes.c_int32), ("w0", ctypes.c_float),
                ("n_freq", ctypes.c_int32), ("rwf", ctypes.c_int32), ("has_bias", ctypes.c_int32),
                ("periodic_mask", ctypes.c_int32), ("period_train_mask", ctypes.c_int32),
                ("period", ctypes.c_float * 3)]


class PinnPde(ctypes.Structure):
    _fields_ = [("pde_id", ctypes.c_int32), ("lap_mask", ctypes.c_int32),
                ("coef", ctypes.c_double * 4), ("lambda_res", ctypes.c_double * MAX_RES),
                ("norm_N", ctypes.c_double)]


class PinnAnchor(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("targets", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("out_mask", ctypes.c_int32), ("lambda_", ctypes.c_double)]


class PinnTune(ctypes.Structure):
    _fields_ = [("tile_points", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("bwd_points", ctypes.c_int32), ("chunk_points", ctypes.c_int32)]


class PinnCausal(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("bin_n", ctypes.POINTER(ctypes.c_int64)), ("eps", ctypes.c_double)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class PinnError(RuntimeError):
    def __init__(self, where, code):
        super().__init__("%s: %s (%d)" % (where, STATUS.get(code, "unknown"), code))
        self.code = code


_lib = None

# Symbols the header declares (checked by the CPU tests).
EXPORTS = ["pinn_param_count", "pinn_n_residuals", "pinn_workspace_bytes", "pinn_residual_fwd",
           "pinn_residual_bwd", "pinn_residual_bwd_noalloc", "pinn_batched_workspace_bytes",
           "pinn_batched_bwd", "pinn_term_grads_workspace_bytes", "pinn_term_grads",
           "pinn_balance_update", "pinn_causal_workspace_bytes", "pinn_causal_bwd",
           "pinn_timing_enable", "pinn_timing_collect", "pinn_status_string"]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpinn.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.pinn_param_count.restype = ctypes.c_int64
        L.pinn_param_count.argtypes = [P(PinnNet)]
        L.pinn_n_residuals.restype = ctypes.c_int
        L.pinn_n_residuals.argtypes = [ctypes.c_int]
        L.pinn_workspace_bytes.restype = ctypes.c_int
        L.pinn_workspace_bytes.argtypes = [P(PinnNet), P(PinnPde), ctypes.c_int64, P(PinnAnchor),
                                           ctypes.c_int, ctypes.c_int, ctypes.c_int, P(PinnTune),
                                           P(ctypes.c_size_t)]
        common = [P(PinnNet), P(PinnPde), vp, vp, vp, ctypes.c_int64, P(PinnAnchor), ctypes.c_int,
                  ctypes.c_int, ctypes.c_uint32, P(PinnTune), vp, vp]
        L.pinn_residual_fwd.restype = ctypes.c_int
        L.pinn_residual_fwd.argtypes = common + [vp, ctypes.c_size_t, vp]
        L.pinn_residual_bwd.restype = ctypes.c_int
        L.pinn_residual_bwd.argtypes = common + [vp, vp, ctypes.c_size_t, vp]
        L.pinn_residual_bwd_noalloc.restype = ctypes.c_int
        L.pinn_residual_bwd_noalloc.argtypes = common + [vp, vp]
        L.pinn_batched_workspace_bytes.restype = ctypes.c_int
        L.pinn_batched_workspace_bytes.argtypes = [P(PinnNet), P(PinnPde), P(ctypes.c_int64), ctypes.c_int,
                                                   ctypes.c_int, P(PinnTune), P(ctypes.c_size_t)]
        L.pinn_batched_bwd.restype = ctypes.c_int
        L.pinn_batched_bwd.argtypes = [P(PinnNet), P(PinnPde), P(vp), P(vp), P(ctypes.c_int64), ctypes.c_int,
                                       ctypes.c_int, P(PinnTune), P(vp), vp, vp, ctypes.c_size_t, vp]
        L.pinn_term_grads_workspace_bytes.restype = ctypes.c_int
        L.pinn_term_grads_workspace_bytes.argtypes = [P(PinnNet), P(PinnPde), ctypes.c_int64, P(PinnAnchor),
                                                      ctypes.c_int, ctypes.c_int, P(PinnTune), P(ctypes.c_size_t)]
        L.pinn_term_grads.restype = ctypes.c_int
        L.pinn_term_grads.argtypes = common[:-2] + [vp, vp, vp, ctypes.c_size_t, vp]
        L.pinn_causal_workspace_bytes.restype = ctypes.c_int
        L.pinn_causal_workspace_bytes.argtypes = [P(PinnNet), P(PinnPde), ctypes.c_int64, P(PinnCausal),
                                                  P(PinnAnchor), ctypes.c_int, ctypes.c_int, P(PinnTune),
                                                  P(ctypes.c_size_t)]
        L.pinn_causal_bwd.restype = ctypes.c_int
        L.pinn_causal_bwd.argtypes = [P(PinnNet), P(PinnPde), vp, vp, vp, ctypes.c_int64, P(PinnCausal),
                                      P(PinnAnchor), ctypes.c_int, ctypes.c_int, ctypes.c_uint32, P(PinnTune),
                                      vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.pinn_balance_update.restype = ctypes.c_int
        L.pinn_balance_update.argtypes = [vp, ctypes.c_int, ctypes.c_int64, vp, vp, ctypes.c_double,
                                          ctypes.c_double, vp]
        L.pinn_timing_enable.restype = ctypes.c_int
        L.pinn_timing_enable.argtypes = [ctypes.c_int]
        L.pinn_timing_collect.restype = ctypes.c_int
        L.pinn_timing_collect.argtypes = [P(KernelTime), ctypes.c_int, P(ctypes.c_int)]
        L.pinn_status_string.restype = ctypes.c_char_p
        L.pinn_status_string.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def net_struct(spec):
    n = PinnNet()
    n.d_in = int(spec["d_in"])
    n.d_out = int(spec["d_out"])
    widths = list(spec["widths"])
    if len(widths) > 8:
        raise ValueError("at most 8 hidden layers")
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


def pde_struct(spec):
    p = PinnPde()
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


def tune_struct(tune):
    if tune is None:
        return None
    t = PinnTune()
    t.tile_points = int(tune.get("tile_points", 0))
    t.grid = int(tune.get("grid", 0))
    t.bwd_points = int(tune.get("bwd_points", 0))
    t.chunk_points = int(tune.get("chunk_points", 0))
    return t


def n_residuals(pde_name):
    return lib().pinn_n_residuals(PDE_IDS[pde_name])


def param_count(net_spec):
    n = net_struct(net_spec)
    r = lib().pinn_param_count(ctypes.byref(n))
    if r < 0:
        raise PinnError("pinn_param_count", int(r))
    return int(r)


def _anchor_array(anchors):
    arr = (PinnAnchor * max(1, len(anchors)))()
    for i, a in enumerate(anchors):
        pts, tgt = a["points"], a["targets"]
        arr[i].points = pts.data_ptr() if isinstance(pts, torch.Tensor) else 0
        arr[i].targets = tgt.data_ptr() if isinstance(tgt, torch.Tensor) else 0
        arr[i].n = int(pts.shape[0])
        arr[i].out_mask = int(a.get("out_mask", 1))
        arr[i].lambda_ = float(a.get("lambda", 1.0))
    return arr


def workspace_bytes(net_spec, pde_spec, n_points, anchors=(), prec="bf16x3", with_grad=True,
                    tune=None):
    n, p = net_struct(net_spec), pde_struct(pde_spec)
    arr = _anchor_array(anchors)
    t = tune_struct(tune)
    out = ctypes.c_size_t(0)
    rc = lib().pinn_workspace_bytes(ctypes.byref(n), ctypes.byref(p), int(n_points), arr, len(anchors),
                                    PRECS[prec], int(bool(with_grad)),
                                    ctypes.byref(t) if t is not None else None, ctypes.byref(out))
    if rc != 0:
        raise PinnError("pinn_workspace_bytes", rc)
    return int(out.value)


class Workspace:
    """A reusable device buffer (grown on demand) for the library's scratch."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws = {}


def _ws(device):
    key = str(device)
    if key not in _default_ws:
        _default_ws[key] = Workspace(device)
    return _default_ws[key]


def _check_dev(t, name, dtype=torch.float32):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s tensor" % (name, dtype))


def _check_shapes(net_spec, params, B, points, anchors=()):
    """Sizes the C ABI cannot see: a mis-sized buffer would be read out of bounds on the
    device, so every size is checked here before any library call (ValueError)."""
    d_in, d_out = int(net_spec["d_in"]), int(net_spec["d_out"])
    n_freq = int(net_spec.get("n_freq", 0))
    want = param_count(net_spec)
    if params.dim() != 1 or params.numel() != want:
        raise ValueError("params must be a flat tensor of %d values, got shape %s"
                         % (want, tuple(params.shape)))
    if points.dim() != 2 or points.shape[1] != d_in:
        raise ValueError("points must have shape (n, %d), got %s" % (d_in, tuple(points.shape)))
    if n_freq > 0:
        if B is None or B.numel() != d_in * n_freq:
            raise ValueError("fourier_B must hold d_in x n_freq = %d values" % (d_in * n_freq))
    elif B is not None:
        raise ValueError("fourier_B given for a network without Fourier features")
    for i, a in enumerate(anchors):
        ap, at = a["points"], a["targets"]
        if ap.dim() != 2 or ap.shape[1] != d_in:
            raise ValueError("anchor %d points must have shape (n, %d)" % (i, d_in))
        if at.numel() != ap.shape[0] * d_out:
            raise ValueError("anchor %d targets must hold n x d_out = %d values"
                             % (i, ap.shape[0] * d_out))


def residual_step(net_spec, pde_spec, params, B, points, anchors=(), prec="bf16x3", grad=True,
                  residual=True, tune=None, flags=0, workspace=None, out=None):
    """One call of pinn_residual_bwd (grad=True) or pinn_residual_fwd.

    params, B, points and the anchors' points/targets are FP32 device tensors.  Returns
    dict(loss = FP64 [1 + n_res + n_anchor], grad = FP64 [n_params] or None,
    residual = FP32 [n, n_res] or None).  `out` may hold preallocated result tensors."""
    _check_dev(params, "params")
    _check_dev(points, "points")
    if B is not None:
        _check_dev(B, "fourier_B")
    for a in anchors:
        _check_dev(a["points"], "anchor points")
        _check_dev(a["targets"], "anchor targets")
    _check_shapes(net_spec, params, B, points, anchors)
    dev = points.device
    n, p = net_struct(net_spec), pde_struct(pde_spec)
    arr = _anchor_array(anchors)
    t = tune_struct(tune)
    tref = ctypes.byref(t) if t is not None else None
    npts = int(points.shape[0])
    nres = n_residuals(pde_spec["pde"])
    size = ctypes.c_size_t(0)
    rc = lib().pinn_workspace_bytes(ctypes.byref(n), ctypes.byref(p), npts, arr, len(anchors),
                                    PRECS[prec], int(bool(grad)), tref, ctypes.byref(size))
    if rc != 0:
        raise PinnError("pinn_workspace_bytes", rc)
    ws = (workspace or _ws(dev)).get(int(size.value))
    out = out or {}
    loss = out.get("loss")
    if loss is None:
        loss = torch.empty(1 + nres + len(anchors), dtype=torch.float64, device=dev)
    res = out.get("residual")
    if residual and res is None:
        res = torch.empty((npts, nres), dtype=torch.float32, device=dev)
    g = out.get("grad")
    if grad and g is None:
        g = torch.empty(param_count(net_spec), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    args = [ctypes.byref(n), ctypes.byref(p), params.data_ptr(),
            B.data_ptr() if B is not None else None, points.data_ptr(), npts, arr, len(anchors),
            PRECS[prec], int(flags), tref, res.data_ptr() if residual else None, loss.data_ptr()]
    if grad:
        rc = lib().pinn_residual_bwd(*args, g.data_ptr(), ws.data_ptr(), ws.numel(), stream)
        where = "pinn_residual_bwd"
    else:
        rc = lib().pinn_residual_fwd(*args, ws.data_ptr(), ws.numel(), stream)
        where = "pinn_residual_fwd"
    if rc != 0:
        raise PinnError(where, rc)
    return {"loss": loss, "grad": g if grad else None, "residual": res if residual else None}


class StepGraph:
    """One residual_step captured in a HIP graph (torch.cuda.CUDAGraph) and replayed.

    The capture records the library's kernel launches with their buffers fixed: the
    parameters, Fourier matrix, points and anchors given here, a private workspace, and the
    output tensors in `out`.  Every replay re-reads those inputs (update them in place, e.g.
    an optimiser step on `params`) and overwrites the outputs, at the cost of one graph
    launch instead of one launch per kernel, which is what small steps are bound by.  The
    library issues only kernels on the stream for a step without the finiteness check
    (no memset or copy nodes).  Per-kernel timing (timing_enable) must be off while it is
    built."""

    def __init__(self, net_spec, pde_spec, params, B, points, anchors=(), prec="bf16x3", grad=True,
                 residual=True, tune=None):
        dev = points.device
        self.workspace = Workspace(dev)
        kw = dict(prec=prec, grad=grad, residual=residual, tune=tune, workspace=self.workspace)
        self._args = (net_spec, pde_spec, params, B, points, tuple(anchors))
        # outputs and workspace allocated, kernel attributes set, before the capture
        self.out = residual_step(*self._args, **kw)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        # relaxed: the launchers set kernel attributes (dynamic LDS) while being captured
        with torch.cuda.graph(self.graph, capture_error_mode="relaxed"):
            residual_step(*self._args, out=dict(self.out), **kw)
        torch.cuda.synchronize(dev)

    def replay(self):
        """Launch the captured step on the current stream; returns the output dict."""
        self.graph.replay()
        return self.out


NOALLOC_MAX_BYTES = 64 << 20   # PINN_NOALLOC_MAX_BYTES


def residual_step_noalloc(net_spec, pde_spec, params, B, points, anchors=(), prec="bf16x3",
                          tune=None, flags=0, out=None):
    """One call of pinn_residual_bwd_noalloc: the fused step on the library's own static
    device scratch (no workspace).  Arguments and results as residual_step(grad=True,
    residual=True); result tensors come from `out` when given."""
    _check_dev(params, "params")
    _check_dev(points, "points")
    if B is not None:
        _check_dev(B, "fourier_B")
    for a in anchors:
        _check_dev(a["points"], "anchor points")
        _check_dev(a["targets"], "anchor targets")
    _check_shapes(net_spec, params, B, points, anchors)
    dev = points.device
    n, p = net_struct(net_spec), pde_struct(pde_spec)
    arr = _anchor_array(anchors)
    t = tune_struct(tune)
    tref = ctypes.byref(t) if t is not None else None
    npts = int(points.shape[0])
    nres = n_residuals(pde_spec["pde"])
    out = out or {}
    loss = out.get("loss")
    if loss is None:
        loss = torch.empty(1 + nres + len(anchors), dtype=torch.float64, device=dev)
    res = out.get("residual")
    if res is None:
        res = torch.empty((npts, nres), dtype=torch.float32, device=dev)
    g = out.get("grad")
    if g is None:
        g = torch.empty(param_count(net_spec), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = lib().pinn_residual_bwd_noalloc(ctypes.byref(n), ctypes.byref(p), params.data_ptr(),
                                         B.data_ptr() if B is not None else None, points.data_ptr(),
                                         npts, arr, len(anchors), PRECS[prec], int(flags), tref,
                                         res.data_ptr(), loss.data_ptr(), g.data_ptr(), stream)
    if rc != 0:
        raise PinnError("pinn_residual_bwd_noalloc", rc)
    return {"loss": loss, "grad": g, "residual": res}


def term_grads(net_spec, pde_spec, params, B, points, anchors=(), prec="bf16x3", tune=None,
               flags=0, workspace=None):
    """One call of pinn_term_grads: dict(loss = FP64 [1 + n_res + n_anchor],
    grads = FP64 [1 + n_anchor, n_params]) -- the residual term's gradient, then each
    supervision set's."""
    _check_dev(params, "params")
    _check_dev(points, "points")
    if B is not None:
        _check_dev(B, "fourier_B")
    for a in anchors:
        _check_dev(a["points"], "anchor points")
        _check_dev(a["targets"], "anchor targets")
    _check_shapes(net_spec, params, B, points, anchors)
    dev = points.device
    n, p = net_struct(net_spec), pde_struct(pde_spec)
    arr = _anchor_array(anchors)
    t = tune_struct(tune)
    tref = ctypes.byref(t) if t is not None else None
    npts = int(points.shape[0])
    size = ctypes.c_size_t(0)
    rc = lib().pinn_term_grads_workspace_bytes(ctypes.byref(n), ctypes.byref(p), npts, arr, len(anchors),
                                               PRECS[prec], tref, ctypes.byref(size))
    if rc != 0:
        raise PinnError("pinn_term_grads_workspace_bytes", rc)
    ws = (workspace or _ws(dev)).get(int(size.value))
    nres = n_residuals(pde_spec["pde"])
    loss = torch.empty(1 + nres + len(anchors), dtype=torch.float64, device=dev)
    grads = torch.empty((1 + len(anchors), param_count(net_spec)), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = lib().pinn_term_grads(ctypes.byref(n), ctypes.byref(p), params.data_ptr(),
                               B.data_ptr() if B is not None else None, points.data_ptr(), npts, arr,
                               len(anchors), PRECS[prec], int(flags), tref, loss.data_ptr(), grads.data_ptr(),
                               ws.data_ptr(), ws.numel(), stream)
    if rc != 0:
        raise PinnError("pinn_term_grads", rc)
    return {"loss": loss, "grads": grads}


def causal_step(net_spec, pde_spec, params, B, points, bin_n, eps, anchors=(), prec="bf16x3", tune=None,
                flags=0, workspace=None):
    """One call of pinn_causal_bwd (Sec. 2.6.8): points sorted into len(bin_n) consecutive
    time segments.  Returns dict(loss, grad, residual, bin_loss, w)."""
    _check_dev(params, "params")
    _check_dev(points, "points")
    if B is not None:
        _check_dev(B, "fourier_B")
    for a in anchors:
        _check_dev(a["points"], "anchor points")
        _check_dev(a["targets"], "anchor targets")
    _check_shapes(net_spec, params, B, points, anchors)
    dev = points.device
    n, p = net_struct(net_spec), pde_struct(pde_spec)
    arr = _anchor_array(anchors)
    t = tune_struct(tune)
    tref = ctypes.byref(t) if t is not None else None
    bins = (ctypes.c_int64 * len(bin_n))(*[int(b) for b in bin_n])
    cz = PinnCausal(len(bin_n), ctypes.cast(bins, ctypes.POINTER(ctypes.c_int64)), float(eps))
    npts = int(points.shape[0])
    size = ctypes.c_size_t(0)
    rc = lib().pinn_causal_workspace_bytes(ctypes.byref(n), ctypes.byref(p), npts, ctypes.byref(cz), arr,
                                           len(anchors), PRECS[prec], tref, ctypes.byref(size))
    if rc != 0:
        raise PinnError("pinn_causal_workspace_bytes", rc)
    ws = (workspace or _ws(dev)).get(int(size.value))
    nres = n_residuals(pde_spec["pde"])
    loss = torch.empty(1 + nres + len(anchors), dtype=torch.float64, device=dev)
    grad = torch.empty(param_count(net_spec), dtype=torch.float64, device=dev)
    res = torch.empty((npts, nres), dtype=torch.float32, device=dev)
    bl = torch.empty(len(bin_n), dtype=torch.float64, device=dev)
    bw = torch.empty(len(bin_n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = lib().pinn_causal_bwd(ctypes.byref(n), ctypes.byref(p), params.data_ptr(),
                               B.data_ptr() if B is not None else None, points.data_ptr(), npts, ctypes.byref(cz),
                               arr, len(anchors), PRECS[prec], int(flags), tref, res.data_ptr(), loss.data_ptr(),
                               grad.data_ptr(), bl.data_ptr(), bw.data_ptr(), ws.data_ptr(), ws.numel(), stream)
    if rc != 0:
        raise PinnError("pinn_causal_bwd", rc)
    return {"loss": loss, "grad": grad, "residual": res, "bin_loss": bl, "w": bw}


def balance_update(grads, lam, alpha=0.9, eps=1e-9, want_hat=True):
    """pinn_balance_update on device tensors: grads FP64 [T, n_params], lam FP64 [T]
    (updated in place).  Returns lambda_hat (FP64 [T]) or None."""
    _check_dev(grads, "grads", torch.float64)
    _check_dev(lam, "lambda", torch.float64)
    if grads.dim() != 2 or lam.numel() != grads.shape[0]:
        raise ValueError("grads must be (T, n_params) and lambda (T,)")
    hat = torch.empty_like(lam) if want_hat else None
    stream = torch.cuda.current_stream(grads.device).cuda_stream
    rc = lib().pinn_balance_update(grads.data_ptr(), int(grads.shape[0]), int(grads.shape[1]), lam.data_ptr(),
                                   hat.data_ptr() if hat is not None else None, float(alpha), float(eps), stream)
    if rc != 0:
        raise PinnError("pinn_balance_update", rc)
    return hat


def timing_enable(on=True):
    lib().pinn_timing_enable(int(bool(on)))


def timing_collect():
    """{kernel name: (launches, total ms)} recorded since the last collect."""
    arr = (KernelTime * 64)()
    n = ctypes.c_int(0)
    rc = lib().pinn_timing_collect(arr, 64, ctypes.byref(n))
    if rc != 0:
        raise PinnError("pinn_timing_collect", rc)
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n.value)}


def _batch_structs(net_specs, n_points, tune_table):
    n = len(net_specs)
    nets = (PinnNet * n)(*[net_struct(s) for s in net_specs])
    npts = (ctypes.c_int64 * n)(*[int(x) for x in n_points])
    tt = None
    if tune_table is not None:
        tt = (PinnTune * n)(*[tune_struct(t or {}) for t in tune_table])
    return nets, npts, tt


def batched_workspace_bytes(net_specs, pde_spec, n_points, prec="bf16x3", tune_table=None):
    nets, npts, tt = _batch_structs(net_specs, n_points, tune_table)
    p = pde_struct(pde_spec)
    out = ctypes.c_size_t(0)
    rc = lib().pinn_batched_workspace_bytes(nets, ctypes.byref(p), npts, len(net_specs), PRECS[prec], tt,
                                            ctypes.byref(out))
    if rc != 0:
        raise PinnError("pinn_batched_workspace_bytes", rc)
    return int(out.value)


def batched_step(net_specs, pde_spec, params, points, prec="bf16x3", tune_table=None, workspace=None,
                 out=None):
    """One pinn_batched_bwd call over independent networks.

    params[i], points[i]: FP32 device tensors.  Returns dict(losses = FP64 [n_inst, 1 + n_res],
    grads = list of FP64 [n_params_i])."""
    n = len(net_specs)
    if len(params) != n or len(points) != n:
        raise ValueError("one params and one points tensor per network")
    for i in range(n):
        _check_dev(params[i], "params[%d]" % i)
        _check_dev(points[i], "points[%d]" % i)
        _check_shapes(net_specs[i], params[i], None, points[i])
    dev = points[0].device
    nets, npts, tt = _batch_structs(net_specs, [p.shape[0] for p in points], tune_table)
    p = pde_struct(pde_spec)
    size = ctypes.c_size_t(0)
    rc = lib().pinn_batched_workspace_bytes(nets, ctypes.byref(p), npts, n, PRECS[prec], tt, ctypes.byref(size))
    if rc != 0:
        raise PinnError("pinn_batched_workspace_bytes", rc)
    ws = (workspace or _ws(dev)).get(int(size.value))
    out = out or {}
    nres = n_residuals(pde_spec["pde"])
    losses = out.get("losses")
    if losses is None:
        losses = torch.empty((n, 1 + nres), dtype=torch.float64, device=dev)
    grads = out.get("grads")
    if grads is None:
        grads = [torch.empty(param_count(s), dtype=torch.float64, device=dev) for s in net_specs]
    pp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in params])
    xp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in points])
    gp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in grads])
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = lib().pinn_batched_bwd(nets, ctypes.byref(p), pp, xp, npts, n, PRECS[prec], tt, gp, losses.data_ptr(),
                                ws.data_ptr(), ws.numel(), stream)
    if rc != 0:
        raise PinnError("pinn_batched_bwd", rc)
    return {"losses": losses, "grads": grads}
