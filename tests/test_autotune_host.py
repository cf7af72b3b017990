"""Host-side logic of the launch-shape autotuner (no device needed)."""
import json

from paper_2604_15645_amd import autotune, synth


def test_width_class():
    assert autotune.width_class({"widths": [32, 32]}) == 32
    assert autotune.width_class({"widths": [96, 64]}) == 128
    assert autotune.width_class({"widths": [256] * 6, "n_freq": 128}) == 256


def test_signatures_are_stable_and_discriminating():
    c = synth.make_case("ns", n_points=1000)
    s1 = autotune.signature(c["net"], c["pde"], 1000, "bf16x3")
    s2 = autotune.signature(c["net"], c["pde"], 1024, "bf16x3")
    s3 = autotune.signature(c["net"], c["pde"], 1025, "bf16x3")
    s4 = autotune.signature(c["net"], c["pde"], 1000, "fp32")
    assert s1 == s2 and s1 != s3 and s1 != s4
    sweep = synth.make_sweep(scale=0.01)
    nets = [c["net"] for c in sweep]
    n = [len(c["points"]) for c in sweep]
    b1 = autotune.batch_signature(nets, n, "bf16x3")
    assert b1 == autotune.batch_signature(nets[::-1], n[::-1], "bf16x3")   # order-free
    assert b1 != autotune.batch_signature(nets[:-1], n[:-1], "bf16x3")


def test_expand_table():
    sweep = synth.make_sweep(scale=0.01)[:8]
    nets = [c["net"] for c in sweep]
    t = autotune.expand_table(nets, {32: 512, 64: 1024, 128: 2048, 256: 4096}, 128)
    for s, e in zip(nets, t):
        assert e == {"chunk_points": {32: 512, 64: 1024, 128: 2048, 256: 4096}[max(s["widths"])], "grid": 128}


def test_cache_roundtrip(tmp_path):
    p = tmp_path / "sub" / "tune.json"
    c = autotune.TuneCache(str(p))
    assert c.get("dev", "sig") is None
    c.put("dev", "sig", {"tune": {"tile_points": 16}, "ms": 1.5})
    c2 = autotune.TuneCache(str(p))
    assert c2.get("dev", "sig")["tune"] == {"tile_points": 16}
    assert json.loads(p.read_text())["dev"]["sig"]["ms"] == 1.5
    assert not (tmp_path / "sub" / "tune.json.tmp").exists()


def test_default_chunks_match_library_defaults():
    # the C ABI's defaults, as stated in include/pinn.h's pinn_tune documentation
    assert autotune.DEFAULT_CHUNK == {32: 4096, 64: 4096, 128: 2048, 256: 1024}
    # work-item sizes are multiples of 128; -1 is the own-launches option of the batched call
    for c in autotune.CHUNKS:
        assert c == -1 or (c > 0 and c % 128 == 0)


def test_candidate_shapes_are_the_library_shapes():
    """Every forward-tile and split-backward candidate the tuner times is a shape the
    library plans for that width (checked by the host-side workspace query), and shapes
    outside the lists are refused."""
    from paper_2604_15645_amd import binding
    for name, h in (("burgers", 32), ("euler", 64), ("ns", 128), ("maxwell", 256)):
        net, pde = synth.CONFIGS[name]["net"], synth.CONFIGS[name]["pde"]
        for tp in autotune.fwd_tiles(h):
            for bp in autotune.bwd_tiles(h):
                tune = {"tile_points": tp, "bwd_points": bp}
                assert binding.workspace_bytes(net, pde, 5000, (), "bf16x3", True, tune) > 0, (name, tune)
        for bad in ({"tile_points": 48}, {"tile_points": 8}, {"bwd_points": 4}):
            try:
                binding.workspace_bytes(net, pde, 5000, (), "bf16x3", True, bad)
                raise AssertionError((name, bad))
            except binding.PinnError as e:
                assert e.code == -2
    # the split-role sub-tile is a split-precision, uniform-width choice
    net, pde = synth.CONFIGS["ns"]["net"], synth.CONFIGS["ns"]["pde"]
    for prec in ("fp32",):
        try:
            binding.workspace_bytes(net, pde, 5000, (), prec, True, {"bwd_points": 16})
            raise AssertionError(prec)
        except binding.PinnError as e:
            assert e.code == -2
    assert autotune.fwd_tiles(256) == (0, 16) and autotune.fwd_tiles(32) == (0, 64, 16)
    assert autotune.bwd_tiles(64) == (0,) and autotune.bwd_tiles(256) == (0, 8)
