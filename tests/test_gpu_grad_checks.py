"""The HIP path's gradient against central differences of its own loss, and the
torch.autograd.Function wrapper."""
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


def setup(name, n, dev, seed=21):
    import torch
    from paper_2604_15645_amd import synth
    case = synth.make_case(name, n_points=n, seed=seed, perturb=True)
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    anchors = [dict(a, points=t(a["points"]), targets=t(a["targets"])) for a in case["anchors"]]
    return case, t(case["params"]), t(case["B"]), t(case["points"]), anchors


@pytest.mark.parametrize("name", ["burgers", "euler", "ns", "maxwell"])
def test_directional_derivative_matches_central_difference(dev, name):
    """dL/dtheta . v against central difference quotients of the loss (Richardson-
    extrapolated), GPU FP32 path only, several random directions; the FP32 loss limits the
    quotient to ~1e-4 relative."""
    import torch
    from paper_2604_15645_amd import binding
    case, params, B, pts, anchors = setup(name, 600 if name != "maxwell" else 200, dev)
    net, pde = case["net"], case["pde"]
    g = binding.residual_step(net, pde, params, B, pts, anchors, prec="fp32")["grad"].clone()
    rng = np.random.Generator(np.random.PCG64(3))
    for k in range(3):
        v = torch.from_numpy(rng.normal(size=params.numel()).astype(np.float32)).to(dev)
        v /= v.norm()
        def quotient(h):
            lp = binding.residual_step(net, pde, params + h * v, B, pts, anchors, prec="fp32",
                                       grad=False, residual=False)["loss"][0].item()
            lm = binding.residual_step(net, pde, params - h * v, B, pts, anchors, prec="fp32",
                                       grad=False, residual=False)["loss"][0].item()
            return (lp - lm) / (2 * h)
        # A large step keeps the FP32 rounding noise of the loss (~3e-7 L / h) small; one
        # Richardson level leaves O(h^4) truncation, below 1e-5 relative on these networks
        # at h = 0.2 (checked with the FP64 oracle's loss).
        h = 0.2
        fd = (4 * quotient(h / 2) - quotient(h)) / 3
        an = float((g * v.double()).sum())
        scale = max(abs(an), 1e-3 * float(g.norm()))
        print(name, k, "analytic %.6e fd %.6e" % (an, fd))
        assert abs(fd - an) <= 2e-3 * scale + 1e-9, (name, k, an, fd)


def test_autograd_function(dev):
    import torch
    from paper_2604_15645_amd import binding
    from paper_2604_15645_amd.autograd import pinn_loss
    case, params, B, pts, anchors = setup("euler", 500, dev)
    p = params.clone().requires_grad_(True)
    loss = pinn_loss(p, pts, B, case["net"], case["pde"], anchors, prec="fp32")
    (3.0 * loss).backward()
    ref = binding.residual_step(case["net"], case["pde"], params, B, pts, anchors, prec="fp32")
    torch.cuda.synchronize()
    assert abs(loss.item() - ref["loss"][0].item()) <= 1e-6 * abs(ref["loss"][0].item())
    want = (3.0 * ref["grad"]).float()
    assert torch.allclose(p.grad, want, rtol=1e-5, atol=1e-7 * float(want.abs().max()))


def test_nonfinite_parameter_check(dev):
    import torch
    from paper_2604_15645_amd import binding
    case, params, B, pts, anchors = setup("burgers", 300, dev)
    bad = params.clone()
    bad[5] = float("nan")
    with pytest.raises(binding.PinnError) as e:
        binding.residual_step(case["net"], case["pde"], bad, B, pts, anchors, prec="fp32",
                              flags=binding.FLAG_CHECK_FINITE)
    assert e.value.code == -4
    out = binding.residual_step(case["net"], case["pde"], params, B, pts, anchors, prec="fp32",
                                flags=binding.FLAG_CHECK_FINITE)
    torch.cuda.synchronize()
    assert torch.isfinite(out["grad"]).all()
