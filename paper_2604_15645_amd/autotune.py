"""Launch-shape autotuner for the fused residual + gradient step.

The tunable launch parameters are those of `pinn_tune` in include/pinn.h:

* single network (`pinn_residual_bwd`): the forward tile size (`tile_points`: the default
  for the hidden width, half of it, or 16 points), the sub-tile of the split-role
  hidden-layer backward (`bwd_points`: the default or half of it) and the work-group count
  (`grid`); every combination the library builds for the network is timed;
* many networks in one persistent launch (`pinn_batched_bwd`): the points per work item
  (`chunk_points`) for each hidden-width class, or -1 for a class whose networks run
  faster as fused steps of their own after the persistent launch, and the work-group
  count.

Each candidate is timed on the device with HIP events around real calls of the library
(median of `reps` calls after one warm-up call), and the fastest is kept.  The batched
table is tuned by coordinate descent over the width classes present.  Results are cached
in a JSON file keyed by the device name and a signature of the problem, so a tuned table
is reused by later runs; the cache path is `$PINN_TUNE_CACHE`, else
`~/.cache/paper_2604_15645_amd/tune.json`.

Changing a launch parameter changes how partial sums are grouped, so results of
different tunings agree to rounding, not bitwise; a given tuning is bitwise repeatable.
"""
import json
import os
import statistics

from . import binding

GRIDS = (0, 128)                        # 0 = the library's default (one per compute unit)
# batched work-item sizes (multiples of 128); -1: the class's instances run as fused steps
# of their own after the persistent launch
CHUNKS = (512, 1024, 2048, 4096, 8192, -1)
DEFAULT_CHUNK = {32: 4096, 64: 4096, 128: 2048, 256: 1024}   # the library's defaults


def default_cache_path():
    p = os.environ.get("PINN_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2604_15645_amd", "tune.json")


class TuneCache:
    """JSON file of {device: {signature: entry}}; writes are atomic (rename)."""

    def __init__(self, path=None):
        self.path = path or default_cache_path()
        self.data = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.data = json.load(f)

    def get(self, device, sig):
        return self.data.get(device, {}).get(sig)

    def put(self, device, sig, entry):
        self.data.setdefault(device, {})[sig] = entry
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def width_class(net_spec):
    """The hidden-width template class (32, 64, 128 or 256) the library compiles for."""
    w = max(net_spec["widths"])
    for h in (32, 64, 128, 256):
        if w <= h:
            return h
    raise ValueError("hidden width above 256")


FWD_DEFAULT = {32: 128, 64: 64, 128: 64, 256: 32}   # the library's forward tile per width
SPLIT_DEFAULT = {128: 32, 256: 16}                   # split-role backward sub-tile per width


def fwd_tiles(h):
    """Forward tile candidates of a width class: the default (0), half of it, 16 points."""
    half = FWD_DEFAULT[h] // 2
    return (0,) + ((half,) if half >= 32 else ()) + (16,)


def bwd_tiles(h):
    """Split-backward sub-tile candidates: the default (0) and half of it."""
    return (0,) + ((SPLIT_DEFAULT[h] // 2,) if h in SPLIT_DEFAULT else ())


def signature(net_spec, pde_spec, n_points, prec):
    """Problem signature of a single-network call; point counts rounded to powers of two."""
    n = 1 << max(0, int(n_points) - 1).bit_length()
    return "single|%s|%s|d%d|%s|%s|m%d|rwf%d|lap%d|n%d|%s" % (
        pde_spec["pde"], net_spec["act"], net_spec["d_in"],
        "x".join(str(w) for w in net_spec["widths"]), net_spec["d_out"], net_spec.get("n_freq", 0),
        int(bool(net_spec.get("rwf"))), int(pde_spec.get("lap_mask", 0)), n, prec)


def batch_signature(net_specs, n_points, prec):
    """Signature of a batched call: per (width class, depth), the number of networks and
    their total points rounded to a power of two."""
    per = {}
    for s, n in zip(net_specs, n_points):
        k = (width_class(s), len(s["widths"]))
        c, v = per.get(k, (0, 0))
        per[k] = (c + 1, v + int(n))
    parts = ["h%dd%d:%dx%d" % (h, d, c, 1 << max(0, v - 1).bit_length()) for (h, d), (c, v) in sorted(per.items())]
    return "batched|%s|%s|%s" % (net_specs[0]["act"], prec, ",".join(parts))


def expand_table(net_specs, chunk_by_class, grid):
    """Per-instance pinn_tune dicts from a chunk size per width class."""
    return [{"chunk_points": int(chunk_by_class[width_class(s)]), "grid": int(grid)} for s in net_specs]


def _device_key(device):
    import torch
    p = torch.cuda.get_device_properties(device)
    return "%s|%s" % (p.name, getattr(p, "gcnArchName", ""))


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        t.append(e0.elapsed_time(e1))
    return statistics.median(t)


def tune_single(net_spec, pde_spec, params, B, points, anchors=(), prec="bf16x3", reps=3,
                cache=None, force=False):
    """Best pinn_tune dict for one network; returns (tune, ms, table of all candidates)."""
    dev = points.device
    cache = cache if cache is not None else TuneCache()
    sig = signature(net_spec, pde_spec, points.shape[0], prec)
    key = _device_key(dev)
    hit = cache.get(key, sig)
    if hit and not force:
        return hit["tune"], hit["ms"], hit.get("table", [])
    ws = binding.Workspace(dev)
    # one untimed call first, so that no candidate pays for first-use costs (workspace
    # growth, code-object loading)
    binding.residual_step(net_spec, pde_spec, params, B, points, anchors, prec=prec, residual=False,
                          workspace=ws)
    table = []
    h = width_class(net_spec)
    for tp in fwd_tiles(h):
        for bp in bwd_tiles(h):
            for grid in GRIDS:
                tune = {"tile_points": tp, "bwd_points": bp, "grid": grid}
                try:
                    ms = _time(lambda: binding.residual_step(net_spec, pde_spec, params, B, points, anchors,
                                                             prec=prec, residual=False, tune=tune,
                                                             workspace=ws), reps)
                except binding.PinnError:
                    continue          # shape the library does not build for this network
                table.append({"tune": tune, "ms": ms})
    best = min(table, key=lambda r: r["ms"])
    cache.put(key, sig, {"tune": best["tune"], "ms": best["ms"], "table": table})
    return best["tune"], best["ms"], table


def tune_batched(net_specs, pde_spec, params, points, prec="bf16x3", reps=2, cache=None, force=False,
                 chunks=CHUNKS, grids=GRIDS):
    """Per-instance tune table for one batched launch, by coordinate descent over the
    width classes present (two rounds), then over the work-group count.  Returns (table, ms,
    log)."""
    dev = points[0].device
    cache = cache if cache is not None else TuneCache()
    sig = batch_signature(net_specs, [p.shape[0] for p in points], prec)
    key = _device_key(dev)
    hit = cache.get(key, sig)
    if hit and not force:
        return expand_table(net_specs, {int(k): v for k, v in hit["chunks"].items()}, hit["grid"]), hit["ms"], \
            hit.get("log", [])
    classes = sorted({width_class(s) for s in net_specs})
    best_chunks = {h: DEFAULT_CHUNK[h] for h in classes}
    best_grid = 0
    ws = binding.Workspace(dev)
    log = []

    def run(ch, grid):
        tt = expand_table(net_specs, ch, grid)
        return _time(lambda: binding.batched_step(net_specs, pde_spec, params, points, prec=prec,
                                                  tune_table=tt, workspace=ws), reps)

    run(best_chunks, best_grid)          # untimed: first-use costs
    best_ms = run(best_chunks, best_grid)
    log.append({"chunks": dict(best_chunks), "grid": best_grid, "ms": best_ms})
    # two rounds over the classes: a class's best choice depends on what the others run
    # (which networks share the persistent launch)
    for _ in range(2):
        for h in classes:
            for c in chunks:
                if c == best_chunks[h]:
                    continue
                trial = dict(best_chunks)
                trial[h] = c
                ms = run(trial, best_grid)
                log.append({"chunks": dict(trial), "grid": best_grid, "ms": ms})
                if ms < best_ms:
                    best_ms, best_chunks = ms, trial
    for grid in grids:
        if grid == best_grid:
            continue
        ms = run(best_chunks, grid)
        log.append({"chunks": dict(best_chunks), "grid": grid, "ms": ms})
        if ms < best_ms:
            best_ms, best_grid = ms, grid
    cache.put(key, sig, {"chunks": {str(k): v for k, v in best_chunks.items()}, "grid": best_grid,
                         "ms": best_ms, "log": log})
    return expand_table(net_specs, best_chunks, best_grid), best_ms, log
