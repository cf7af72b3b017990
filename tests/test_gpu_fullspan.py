"""The gradient against the FP64 oracle at the accumulation spans of the full-size launches.

At the benchmark sizes every work-group of the forward, the hidden-layer backward and the
embedding-layer backward sums its own range of points before the fixed-order FP64
reduction across work-groups.  A smaller point set with a reduced work-group count gives
each work-group exactly the range it has at full size, so the oracle can check the whole
gradient, every layer's block and every loss term at the span the benchmark runs:

  Maxwell (RFF 128, 6 x 256 sine), 1,048,576 points, 256 work-groups: forward 4,096 points
      per work-group, hidden-layer weight gradient 8,192, embedding-layer gradient 4,096;
      65,536 points with 16 work-groups reproduce all three.
  Navier-Stokes (5 x 128 tanh, RWF), 262,144 points, 256 work-groups: forward 1,024 points,
      hidden-layer weight gradient 2,048; 32,768 points with 32 work-groups reproduce both.

Tolerances are the gates of the path: FP32 1e-5, BF16X3 and FP16X3 1e-4 (normwise, relative)."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "fp16x3": 1e-4}
CASES = {"maxwell": (65536, 16), "ns": (32768, 32)}


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


_ref = {}


def reference(oracle, name):
    from paper_2604_15645_amd import synth
    if name not in _ref:
        n, _ = CASES[name]
        case = synth.make_case(name, n_points=n)       # the benchmark's own input recipe
        _ref[name] = (case, oracle.loss_grad(case["net"], case["pde"], case["params"], case["B"],
                                             case["points"], case["anchors"]))
    return _ref[name]


def layer_blocks(net):
    """(first, last) parameter index of every linear layer: W (or V), s, b together."""
    from paper_2604_15645_amd import synth
    out, off = [], 0
    for no, ni in synth.layer_dims(net):
        k = no * ni + (no if net.get("rwf") else 0) + (no if net.get("has_bias", True) else 0)
        out.append((off, off + k))
        off += k
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("name", ["maxwell", "ns"])
def test_gradient_at_full_size_spans(oracle, dev, name, prec):
    import torch
    from paper_2604_15645_amd import binding
    case, ref = reference(oracle, name)
    n, grid = CASES[name]
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    out = binding.residual_step(case["net"], case["pde"], t(case["params"]), t(case["B"]),
                                t(case["points"]), (), prec=prec, tune={"grid": grid})
    torch.cuda.synchronize()
    res = out["residual"].cpu().numpy()
    loss = out["loss"].cpu().numpy()
    grad = out["grad"].cpu().numpy()
    errs = {"res%d" % c: relerr(res[:, c], ref["residual"][:, c]) for c in range(res.shape[1])}
    for k in range(len(loss)):
        errs["loss%d" % k] = abs(loss[k] - ref["loss"][k]) / abs(ref["loss"][k])
    errs["grad"] = relerr(grad, ref["grad"])
    for li, (a, b) in enumerate(layer_blocks(case["net"])):
        errs["grad_layer%d" % li] = relerr(grad[a:b], ref["grad"][a:b])
    print(name, prec, {k: "%.2e" % v for k, v in errs.items()})
    bad = {k: v for k, v in errs.items() if not v <= TOL[prec]}
    assert not bad, (name, prec, bad)
