"""A step captured in a HIP graph and replayed (binding.StepGraph): every replay equals the
eager call on the same inputs, with eager work and in-place parameter updates between the
replays."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    return torch.device("cuda:0")


def inputs(name, n, dev, seed):
    import torch
    from paper_2604_15645_amd import synth
    case = synth.make_case(name, n_points=n, seed=seed, perturb=True)
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    anchors = [dict(a, points=t(a["points"]), targets=t(a["targets"])) for a in case["anchors"]]
    return case, t(case["params"]), t(case["B"]), t(case["points"]), anchors


# Burgers with its two anchor sets (identity embedding, narrow layers), Maxwell (Fourier
# embedding, width 256: kernels with more than 64 KiB of LDS)
@pytest.mark.parametrize("name,n,prec", [("burgers", 1000, "bf16x3"), ("burgers", 1000, "fp32"),
                                         ("maxwell", 700, "bf16x3"), ("maxwell", 700, "fp16x3")])
def test_graph_replays_equal_eager_calls(dev, name, n, prec):
    import torch
    from paper_2604_15645_amd import binding
    case, params, B, pts, anchors = inputs(name, n, dev, 150)
    other, p2, B2, x2, a2 = inputs("ns", 900, dev, 151)
    g = binding.StepGraph(case["net"], case["pde"], params, B, pts, anchors, prec=prec)
    ws = binding.Workspace(dev)
    for rep in range(4):
        out = g.replay()
        got = {k: v.clone() for k, v in out.items()}
        torch.cuda.synchronize()
        ref = binding.residual_step(case["net"], case["pde"], params, B, pts, anchors, prec=prec, workspace=ws)
        # unrelated eager work on the same stream between the replays
        binding.residual_step(other["net"], other["pde"], p2, B2, x2, a2, prec=prec, workspace=ws)
        torch.cuda.synchronize()
        for k in ("loss", "grad", "residual"):
            assert torch.equal(got[k], ref[k]), (rep, k)
        # the replay reads the parameters in place
        params.mul_(1.0 + 2.0 ** -8)
