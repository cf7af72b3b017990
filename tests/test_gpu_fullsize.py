"""Full benchmark sizes, in the launch configuration bench.py times.

The oracle cannot evaluate a million-point gradient in a test, so at full size the HIP path
is checked on (a) residuals at sampled points, computed one by one by the oracle, and (b)
properties that hold at any size: each loss term equals lambda/N times the FP64 sum of the
returned squared residuals, and the gradient of the whole set equals the sum of the
gradients of two shards evaluated with the global N."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "fp16x3": 1e-4}


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


@pytest.fixture(scope="module")
def dev():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    return torch.device("cuda:0")


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "fp16x3"])
@pytest.mark.parametrize("name", ["burgers", "euler", "ns", "maxwell", "euler2d"])
def test_full_size(oracle, dev, name, prec):
    import torch
    from paper_2604_15645_amd import binding, synth
    case = synth.make_case(name)               # the benchmark workload, full size
    net, pde = case["net"], case["pde"]
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    params, B, pts = t(case["params"]), t(case["B"]), t(case["points"])
    anchors = [dict(a, points=t(a["points"]), targets=t(a["targets"])) for a in case["anchors"]]
    n = len(case["points"])
    out = binding.residual_step(net, pde, params, B, pts, anchors, prec=prec)
    torch.cuda.synchronize()
    res = out["residual"].cpu().numpy().astype(np.float64)
    loss = out["loss"].cpu().numpy()
    grad = out["grad"].cpu().numpy()
    assert np.isfinite(res).all() and np.isfinite(grad).all()

    # (a) residuals at sampled points
    idx = np.random.Generator(np.random.PCG64(7)).choice(n, size=256, replace=False)
    ref = oracle.loss_grad(net, pde, case["params"], case["B"], case["points"][idx], want_grad=False)
    for c in range(res.shape[1]):
        assert relerr(res[idx, c], ref["residual"][:, c]) <= TOL[prec], (name, c)

    # (b1) every residual loss term from the returned residuals
    lam = pde.get("lambda_res", [1, 1, 1])
    for c in range(res.shape[1]):
        want = lam[c] / n * np.sum(res[:, c] ** 2)
        assert abs(loss[1 + c] - want) <= 1e-6 * want, (name, c, loss[1 + c], want)

    # (b2) shard additivity of the gradient (global N, supervision sets on the first shard)
    half = n // 2
    pde_g = dict(pde, norm_N=float(n))
    g1 = binding.residual_step(net, pde_g, params, B, pts[:half].contiguous(), anchors, prec=prec)
    gsum = g1["grad"].clone()
    lsum = g1["loss"][0].item()
    g2 = binding.residual_step(net, pde_g, params, B, pts[half:].contiguous(), (), prec=prec)
    torch.cuda.synchronize()
    gsum += g2["grad"]
    lsum += g2["loss"][0].item()
    assert relerr(gsum.cpu().numpy(), grad) <= 1e-5
    assert abs(lsum - loss[0]) <= 1e-6 * abs(loss[0])


def test_full_sweep_batched_matches_single_calls(dev):
    """The 64-network sweep in one batched launch against separate calls (sampled)."""
    import torch
    from paper_2604_15645_amd import binding, synth
    insts = synth.make_sweep()
    params = [torch.from_numpy(c["params"]).to(dev) for c in insts]
    pts = [torch.from_numpy(c["points"]).to(dev) for c in insts]
    out = binding.batched_step([c["net"] for c in insts], insts[0]["pde"], params, pts, prec="bf16x3")
    torch.cuda.synchronize()
    losses = out["losses"].cpu().numpy()
    grads = [g.cpu().numpy() for g in out["grads"]]
    for i in (0, 7, 30, 63):
        c = insts[i]
        one = binding.residual_step(c["net"], c["pde"], params[i], None, pts[i], (), prec="bf16x3")
        torch.cuda.synchronize()
        assert relerr(losses[i], one["loss"].cpu().numpy()) < 1e-5
        assert relerr(grads[i], one["grad"].cpu().numpy()) < 1e-4
