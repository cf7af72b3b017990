"""The launch-shape autotuner on the device: it returns a shape the library accepts, the
tuned call agrees with the default one (only the grouping of partial sums differs), and a
second call is served from the cache."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def dev():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    return torch.device("cuda:0")


def test_tune_single(dev, tmp_path):
    import torch
    from paper_2604_15645_amd import autotune, binding, synth
    c = synth.make_case("euler", n_points=20000, perturb=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    params, B, pts = t(c["params"]), t(c["B"]), t(c["points"])
    cache = autotune.TuneCache(str(tmp_path / "tune.json"))
    tune, ms, table = autotune.tune_single(c["net"], c["pde"], params, B, pts, (), prec="bf16x3", cache=cache)
    assert len(table) >= 2 and ms == min(r["ms"] for r in table)
    a = binding.residual_step(c["net"], c["pde"], params, B, pts, (), prec="bf16x3", tune=tune)
    ga, la = a["grad"].clone(), a["loss"].clone()
    b = binding.residual_step(c["net"], c["pde"], params, B, pts, (), prec="bf16x3")
    torch.cuda.synchronize()
    assert relerr(la.cpu(), b["loss"].cpu()) < 1e-6
    assert relerr(ga.cpu(), b["grad"].cpu()) < 1e-5
    tune2, ms2, _ = autotune.tune_single(c["net"], c["pde"], params, B, pts, (), prec="bf16x3",
                                         cache=autotune.TuneCache(str(tmp_path / "tune.json")))
    assert tune2 == tune and ms2 == ms


def test_tune_batched(dev, tmp_path):
    import torch
    from paper_2604_15645_amd import autotune, binding, synth
    insts = synth.make_sweep(scale=0.02)[:12]
    params = [torch.from_numpy(c["params"]).to(dev) for c in insts]
    pts = [torch.from_numpy(c["points"]).to(dev) for c in insts]
    nets = [c["net"] for c in insts]
    cache = autotune.TuneCache(str(tmp_path / "tune.json"))
    table, ms, log = autotune.tune_batched(nets, insts[0]["pde"], params, pts, prec="fp32", cache=cache,
                                           chunks=(512, 2048), grids=(0, 64))
    assert len(table) == len(insts) and ms == min(r["ms"] for r in log)
    a = binding.batched_step(nets, insts[0]["pde"], params, pts, prec="fp32", tune_table=table)
    la, ga = a["losses"].clone(), [g.clone() for g in a["grads"]]
    b = binding.batched_step(nets, insts[0]["pde"], params, pts, prec="fp32")
    torch.cuda.synchronize()
    for i in range(len(insts)):
        assert relerr(la[i].cpu(), b["losses"][i].cpu()) < 1e-6
        assert relerr(ga[i].cpu(), b["grads"][i].cpu()) < 1e-5
