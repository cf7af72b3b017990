"""Host-only checks of the C ABI: the library loads, exports every declared symbol, and
rejects malformed requests with the documented status before touching the GPU."""
import ctypes
import math
import os
import re

import pytest

from paper_2604_15645_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libpinn.so not built")
    return binding.lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pinn.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(pinn_\w+)\s*\(", src, re.M)))


def test_header_declares_what_the_binding_expects():
    assert declared_functions() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_param_count_matches_layout():
    for name in synth.CONFIGS:
        net = synth.CONFIGS[name]["net"]
        assert binding.param_count(net) == synth.param_count(net)
    # the published shapes: 2 -> 3x32 -> 1 Burgers has 2,241 parameters
    assert binding.param_count(synth.CONFIGS["burgers"]["net"]) == 2241
    assert binding.param_count(synth.CONFIGS["maxwell"]["net"]) == 395523


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.pinn_status_string(code).decode() == binding.STATUS[code]


def ws(net, pde, n=100, anchors=(), prec="fp32", grad=True, tune=None):
    return binding.workspace_bytes(net, pde, n, anchors, prec, grad, tune)


def code_of(fn):
    with pytest.raises(binding.PinnError) as e:
        fn()
    return e.value.code


def test_validation_errors(lib):
    c = synth.CONFIGS
    net, pde = dict(c["burgers"]["net"]), dict(c["burgers"]["pde"])
    assert ws(net, pde) > 0
    assert code_of(lambda: ws(dict(net, d_in=0), pde)) == -1
    assert code_of(lambda: ws(dict(net, widths=[0, 32]), pde)) == -1
    assert code_of(lambda: ws(net, dict(pde, pde="ns2d"))) == -2          # ns needs 3 outputs
    assert code_of(lambda: ws(net, dict(pde, lap_mask=0))) == -2          # burgers needs u_xx
    assert code_of(lambda: ws(net, dict(pde, lap_mask=3))) == -2          # ... and u_xx alone
    assert code_of(lambda: ws(net, dict(pde, lap_mask=2))) == -2
    assert code_of(lambda: ws(net, dict(pde, lap_mask=8))) == -1          # input 3 does not exist
    assert code_of(lambda: ws(dict(net, widths=[48, 48]), pde)) == -2     # widths: multiples of 32
    assert code_of(lambda: ws(dict(net, widths=[512]), pde)) == -2        # at most 256 wide
    assert code_of(lambda: ws(dict(net, widths=[]), pde)) == -2           # at least one hidden layer
    assert code_of(lambda: ws(net, pde, n=-1)) == -1
    assert code_of(lambda: ws(net, pde, n=0)) == -1                       # nothing to evaluate
    assert code_of(lambda: ws(net, dict(pde, lambda_res=[-1, 1, 1]))) == -1
    assert code_of(lambda: ws(net, dict(pde, coef=[math.nan, 0, 0, 0]))) == -1
    mx, mp = c["maxwell"]["net"], c["maxwell"]["pde"]
    assert code_of(lambda: ws(mx, dict(mp, lap_mask=1))) == -2            # 5 jet channels
    assert code_of(lambda: ws(dict(mx, n_freq=20), mp)) == -2             # m multiple of 16
    eu, ep = c["euler"]["net"], c["euler"]["pde"]
    assert code_of(lambda: ws(eu, dict(ep, coef=[1.0, 0, 0, 0]))) == -2   # gamma > 1
    an, ap = c["advection"]["net"], c["advection"]["pde"]
    assert ws(an, ap) > 0
    assert code_of(lambda: ws(an, dict(ap, lap_mask=1))) == -2            # first derivatives only
    ac, acp = c["allen_cahn"]["net"], c["allen_cahn"]["pde"]
    assert ws(ac, acp) > 0
    assert code_of(lambda: ws(ac, dict(acp, lap_mask=0))) == -2           # needs u_xx
    assert code_of(lambda: ws(mx, dict(mp, pde="advection"))) == -2       # inputs (x, t)
    assert binding.n_residuals("advection") == binding.n_residuals("allen_cahn") == 1
    e2, e2p = c["euler2d"]["net"], c["euler2d"]["pde"]
    assert ws(e2, e2p) > 0
    assert binding.n_residuals("euler2d") == 4
    assert code_of(lambda: ws(e2, dict(e2p, lap_mask=1))) == -2           # first derivatives only
    assert code_of(lambda: ws(dict(e2, d_out=3), e2p)) == -2              # (rho, u, v, p)
    assert code_of(lambda: ws(mx, dict(mp, pde="euler2d"))) == -2         # four outputs
    assert code_of(lambda: ws(dict(e2, d_out=5), e2p)) == -1              # at most four outputs
    assert code_of(lambda: ws(e2, dict(e2p, lambda_res=[1, 1, 1, -1]))) == -1


def test_term_grads_validation(lib):
    """Per-term gradients need at least one residual point and non-empty supervision sets;
    the balance update rejects bad sizes and weights on the host."""
    import ctypes
    c = synth.CONFIGS["burgers"]
    n, p = binding.net_struct(c["net"]), binding.pde_struct(c["pde"])
    size = ctypes.c_size_t(0)
    arr = binding._anchor_array(())
    assert lib.pinn_term_grads_workspace_bytes(ctypes.byref(n), ctypes.byref(p), 100, arr, 0, 1, None,
                                               ctypes.byref(size)) == 0
    assert size.value >= binding.workspace_bytes(c["net"], c["pde"], 100, (), "bf16x3", True)
    assert lib.pinn_term_grads_workspace_bytes(ctypes.byref(n), ctypes.byref(p), 0, arr, 0, 1, None,
                                               ctypes.byref(size)) == -1
    assert lib.pinn_balance_update(16, 0, 10, 16, None, 0.9, 1e-9, None) == -1
    assert lib.pinn_balance_update(16, 3, 10, 16, None, 1.5, 1e-9, None) == -1
    assert lib.pinn_balance_update(16, 3, 10, 16, None, 0.9, -1.0, None) == -1


def test_causal_validation(lib):
    """The causality call checks the segment sizes against the point count before any HIP
    call."""
    import ctypes
    c = synth.CONFIGS["burgers"]
    n, p = binding.net_struct(c["net"]), binding.pde_struct(c["pde"])
    arr = binding._anchor_array(())
    size = ctypes.c_size_t(0)

    def ws_of(bins, npts, eps=1.0):
        b = (ctypes.c_int64 * len(bins))(*bins)
        cz = binding.PinnCausal(len(bins), ctypes.cast(b, ctypes.POINTER(ctypes.c_int64)), eps)
        return lib.pinn_causal_workspace_bytes(ctypes.byref(n), ctypes.byref(p), npts, ctypes.byref(cz), arr, 0, 1,
                                               None, ctypes.byref(size))
    assert ws_of([100, 50], 150) == 0 and size.value > 0
    assert ws_of([100, 50], 151) == -1        # segments must cover the points
    assert ws_of([100, 0], 100) == -1         # no empty segment
    assert ws_of([100, 50], 150, eps=-1.0) == -1


def test_precision_codes(lib):
    """FP32, BF16X3 and FP16X3 are implemented; single-product BF16 is refused as
    unsupported, an unknown code as invalid; the split forms need the same workspace."""
    c = synth.CONFIGS
    for name in ("burgers", "maxwell"):
        net, pde = c[name]["net"], c[name]["pde"]
        assert ws(net, pde, prec="bf16x3") == ws(net, pde, prec="fp16x3") > 0
        assert ws(net, pde, prec="fp32") > 0
        assert code_of(lambda: ws(net, pde, prec="bf16")) == -2
    with pytest.raises(KeyError):
        ws(c["burgers"]["net"], c["burgers"]["pde"], prec="fp8")
    assert lib.pinn_workspace_bytes is not None


def test_compute_calls_reject_before_any_hip_call(lib):
    """Null pointers and a short workspace fail on the host (no GPU in this container)."""
    c = synth.CONFIGS["burgers"]
    n, p = binding.net_struct(c["net"]), binding.pde_struct(c["pde"])
    loss = ctypes.c_double * 4
    buf = loss()
    arr = (binding.PinnAnchor * 1)()
    size = ctypes.c_size_t(0)
    rc = lib.pinn_workspace_bytes(ctypes.byref(n), ctypes.byref(p), 100, arr, 0, 0, 1, None,
                                  ctypes.byref(size))
    assert rc == 0 and size.value > 0
    fake = 1 << 20  # never dereferenced: the calls below must fail on argument checks
    common = [ctypes.byref(n), ctypes.byref(p)]
    # params missing
    rc = lib.pinn_residual_bwd(*common, None, None, fake, 100, arr, 0, 0, 0, None, None,
                               ctypes.addressof(buf), fake, fake, size.value, None)
    assert rc == -1
    # grad missing
    rc = lib.pinn_residual_bwd(*common, fake, None, fake, 100, arr, 0, 0, 0, None, None,
                               ctypes.addressof(buf), None, fake, size.value, None)
    assert rc == -1
    # workspace too small
    rc = lib.pinn_residual_bwd(*common, fake, None, fake, 100, arr, 0, 0, 0, None, None,
                               ctypes.addressof(buf), fake, fake, size.value - 1, None)
    assert rc == -3
    # fourier matrix missing for an RFF network
    e = synth.CONFIGS["euler"]
    ne, pe = binding.net_struct(e["net"]), binding.pde_struct(e["pde"])
    rc = lib.pinn_workspace_bytes(ctypes.byref(ne), ctypes.byref(pe), 100, arr, 0, 0, 0, None,
                                  ctypes.byref(size))
    assert rc == 0
    rc = lib.pinn_residual_fwd(ctypes.byref(ne), ctypes.byref(pe), fake, None, fake, 100, arr, 0, 0,
                               0, None, None, ctypes.addressof(buf), fake, size.value, None)
    assert rc == -1


def test_workspace_grows_with_points_and_gradient():
    c = synth.CONFIGS["ns"]
    a = ws(c["net"], c["pde"], n=1000)
    b = ws(c["net"], c["pde"], n=100000)
    f = ws(c["net"], c["pde"], n=100000, grad=False)
    assert b > a and f < b
    # the stash of every hidden layer dominates: 5 layers x 4 channels x 128 x 4 B per point
    assert b >= 100000 * 5 * 4 * 128 * 4


def test_binding_rejects_mis_sized_buffers():
    """The C ABI cannot see buffer sizes: the binding checks every one before a call."""
    import torch
    for name in ("burgers", "euler", "maxwell"):
        c = synth.make_case(name, n_points=10)
        net = c["net"]
        p = torch.from_numpy(c["params"])
        x = torch.from_numpy(c["points"])
        B = None if c["B"] is None else torch.from_numpy(c["B"])
        binding._check_shapes(net, p, B, x)                       # the right sizes pass
        with pytest.raises(ValueError):
            binding._check_shapes(net, p[:-1], B, x)              # one parameter short
        with pytest.raises(ValueError):
            binding._check_shapes(net, torch.cat([p, p[:1]]), B, x)
        with pytest.raises(ValueError):
            binding._check_shapes(net, p, B, x[:, :1].contiguous())  # wrong input dimension
        with pytest.raises(ValueError):
            binding._check_shapes(net, p, B, x.reshape(-1))
        if B is not None:
            with pytest.raises(ValueError):
                binding._check_shapes(net, p, B[:, :-1].contiguous(), x)
            with pytest.raises(ValueError):
                binding._check_shapes(net, p, None, x)
        else:
            with pytest.raises(ValueError):
                binding._check_shapes(net, p, torch.zeros(4), x)
    c = synth.make_case("burgers", n_points=10)
    p, x = torch.from_numpy(c["params"]), torch.from_numpy(c["points"])
    a = [dict(points=torch.from_numpy(c["anchors"][0]["points"]),
              targets=torch.from_numpy(c["anchors"][0]["targets"]))]
    binding._check_shapes(c["net"], p, None, x, a)
    with pytest.raises(ValueError):
        binding._check_shapes(c["net"], p, None, x, [dict(a[0], targets=a[0]["targets"][:-1])])


def test_batched_tune_table_validation(lib):
    """chunk_points: a multiple of 128, 0 (the default) or -1 (the instance on launches of
    its own, whose single-network workspace is added to the call's)."""
    cfg = synth.CONFIGS["burgers"]
    nets = [dict(cfg["net"], widths=[64] * 3), dict(cfg["net"], widths=[256] * 3)]
    n = [5000, 7000]
    base = binding.batched_workspace_bytes(nets, cfg["pde"], n, "bf16x3")
    sep = binding.batched_workspace_bytes(nets, cfg["pde"], n, "bf16x3",
                                          [dict(chunk_points=0), dict(chunk_points=-1)])
    single = ws(nets[1], cfg["pde"], 7000, prec="bf16x3")
    assert sep >= single
    assert binding.batched_workspace_bytes(nets, cfg["pde"], n, "bf16x3",
                                           [dict(chunk_points=-1), dict(chunk_points=-1)]) >= single
    assert base > 0
    for bad in (-2, 100):
        assert code_of(lambda: binding.batched_workspace_bytes(nets, cfg["pde"], n, "bf16x3",
                                                               [dict(chunk_points=bad), {}])) == -1
