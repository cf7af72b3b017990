"""Per-term gradients and the loss-balancing update (Sec. 2.6.4) on the GPU, against the
FP64 oracle: every term's gradient to the precision gate, their sum against the fused
step, and the device-side weight update against the oracle's."""
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


def to_dev(case, dev):
    import torch
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    anchors = [dict(a, points=t(a["points"]), targets=t(a["targets"])) for a in case["anchors"]]
    return t(case["params"]), t(case["B"]), t(case["points"]), anchors


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("name", ["burgers", "allen_cahn", "euler2d"])
def test_term_gradients_match_oracle(oracle, dev, name, prec):
    import torch
    from paper_2604_15645_amd import binding, synth
    case = synth.make_case(name, n_points=1500, seed=71, perturb=True)
    params, B, pts, anchors = to_dev(case, dev)
    out = binding.term_grads(case["net"], case["pde"], params, B, pts, anchors, prec=prec)
    torch.cuda.synchronize()
    loss, grads = out["loss"].cpu().numpy(), out["grads"].cpu().numpy()
    rloss, rgrads = oracle.term_grads(case["net"], case["pde"], case["params"], case["B"], case["points"],
                                      case["anchors"])
    assert grads.shape[0] == len(rgrads) == 1 + len(case["anchors"])
    errs = {"loss%d" % k: abs(loss[k] - rloss[k]) / abs(rloss[k]) for k in range(len(rloss))}
    for t, g in enumerate(rgrads):
        errs["grad_term%d" % t] = relerr(grads[t], g)
    print(name, prec, {k: "%.2e" % v for k, v in errs.items()})
    assert all(v <= TOL[prec] for v in errs.values()), errs
    # the terms add up to the fused step's gradient (same kernels, other point groupings)
    full = binding.residual_step(case["net"], case["pde"], params, B, pts, anchors, prec=prec)
    torch.cuda.synchronize()
    assert relerr(grads.sum(0), full["grad"].cpu().numpy()) <= TOL[prec]
    assert relerr(loss, full["loss"].cpu().numpy()) <= TOL[prec]


def test_balance_update_matches_oracle(oracle, dev):
    import torch
    from paper_2604_15645_amd import binding
    rng = np.random.Generator(np.random.PCG64(72))
    g = np.stack([rng.normal(size=5000) * s for s in (1e-3, 0.7, 42.0)])
    lam0 = np.array([1.0, 2.5, 0.2])
    for alpha, eps in ((0.9, 1e-9), (0.0, 0.0), (1.0, 1e-9)):
        gt = torch.from_numpy(g).to(dev)
        lt = torch.from_numpy(lam0.copy()).to(dev)
        hat = binding.balance_update(gt, lt, alpha=alpha, eps=eps)
        torch.cuda.synchronize()
        rl, rh = oracle.balance_update(list(g), lam0, alpha=alpha, eps=eps)
        assert relerr(hat.cpu().numpy(), rh) < 1e-13
        assert relerr(lt.cpu().numpy(), rl) < 1e-13


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("name", ["burgers", "maxwell", "euler2d"])
def test_causal_loss_matches_oracle(oracle, dev, name, prec):
    """Temporal causality (Sec. 2.6.8): points sorted by time into segments of uneven size;
    segment losses, weights, the weighted loss terms and the gradient against the oracle."""
    import torch
    from paper_2604_15645_amd import binding, synth
    n = 1800 if name == "burgers" else 700
    case = synth.make_case(name, n_points=n, seed=73, perturb=True)
    tcol = case["net"]["d_in"] - 1
    pts = case["points"][np.argsort(case["points"][:, tcol], kind="stable")]
    case["points"] = np.ascontiguousarray(pts)
    bin_n = [n // 5, n // 3, n - n // 5 - n // 3 - n // 7, n // 7]
    # a tenth of the weight or more gone by the end (the random 2D Euler network's segment
    # losses are of order 1e7)
    eps = {"burgers": 50.0, "maxwell": 1.5, "euler2d": 3e-8}[name]
    params, B, dpts, anchors = to_dev(case, dev)
    out = binding.causal_step(case["net"], case["pde"], params, B, dpts, bin_n, eps, anchors, prec=prec)
    torch.cuda.synchronize()
    ref = oracle.causal_loss_grad(case["net"], case["pde"], case["params"], case["B"], case["points"], bin_n,
                                  eps, case["anchors"])
    got = {k: v.cpu().numpy() for k, v in out.items()}
    errs = {"grad": relerr(got["grad"], ref["grad"]), "bin_loss": relerr(got["bin_loss"], ref["bin_loss"]),
            "w": relerr(got["w"], ref["w"])}
    for k in range(len(ref["loss"])):
        errs["loss%d" % k] = abs(got["loss"][k] - ref["loss"][k]) / abs(ref["loss"][k])
    print(name, prec, {k: "%.2e" % v for k, v in errs.items()}, "w", ref["w"])
    assert all(v <= TOL[prec] for v in errs.values()), errs
    assert ref["w"][-1] < 0.9   # the weights are not all one
