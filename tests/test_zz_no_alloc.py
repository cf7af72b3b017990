"""The allocation-free entry point (pinn_residual_bwd_noalloc) against the workspace entry
point (pinn_residual_bwd) on the same inputs: two calls in a row on the library's static
scratch, the second with a smaller problem (the scratch then holds the first call's
leftovers), each checked to the precision gate; and the size limit, refused on the host."""
import numpy as np
import pytest

from conftest import gpu_available
from paper_2604_15645_amd import binding, synth

TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "fp16x3": 1e-4}


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def test_noalloc_refuses_problems_beyond_its_scratch():
    """A problem whose workspace exceeds PINN_NOALLOC_MAX_BYTES fails with PINN_E_WORKSPACE
    before any HIP call (this container has no GPU: a HIP call would fail otherwise)."""
    import ctypes
    case = synth.CONFIGS["maxwell"]
    need = binding.workspace_bytes(case["net"], case["pde"], 1 << 20, (), "bf16x3", True)
    assert need > binding.NOALLOC_MAX_BYTES
    n, p = binding.net_struct(case["net"]), binding.pde_struct(case["pde"])
    arr = binding._anchor_array(())
    rc = binding.lib().pinn_residual_bwd_noalloc(ctypes.byref(n), ctypes.byref(p), 16, None, 16, 1 << 20,
                                                 arr, 0, binding.PRECS["bf16x3"], 0, None, 16, 16, 16, None)
    assert rc == -3


@pytest.mark.gpu
def test_noalloc_matches_workspace_entry_twice():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    calls = [("burgers", None, "bf16x3"), ("burgers", 1000, "fp16x3")]   # the second is smaller
    sizes = []
    for name, n, prec in calls:
        case = synth.make_case(name, n_points=n, seed=321, perturb=True)
        params, B, pts = t(case["params"]), t(case["B"]), t(case["points"])
        anchors = [dict(a, points=t(a["points"]), targets=t(a["targets"])) for a in case["anchors"]]
        need = binding.workspace_bytes(case["net"], case["pde"], len(case["points"]), anchors, prec, True)
        assert need <= binding.NOALLOC_MAX_BYTES
        sizes.append(need)
        print("noalloc call: %s, %d points, %s, workspace %d bytes" % (name, len(case["points"]), prec, need),
              flush=True)
        got = binding.residual_step_noalloc(case["net"], case["pde"], params, B, pts, anchors, prec=prec)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in got.items()}
        ref = binding.residual_step(case["net"], case["pde"], params, B, pts, anchors, prec=prec)
        torch.cuda.synchronize()
        ref = {k: v.cpu().numpy() for k, v in ref.items()}
        errs = {k: relerr(got[k], ref[k]) for k in ("loss", "grad", "residual")}
        same = all(np.array_equal(got[k], ref[k]) for k in ("loss", "grad", "residual"))
        print(name, prec, {k: "%.2e" % v for k, v in errs.items()}, "bitwise identical:", same)
        assert all(v <= TOL[prec] for v in errs.values()), (name, prec, errs)
    assert sizes[1] < sizes[0]
