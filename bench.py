"""Benchmark of the fused PINN residual + parameter-gradient step on one MI355X.

A step is one pinn_residual_bwd call over the whole synthetic collocation set: embedding
jets, every hidden layer, output layer, PDE residual, loss, and dL/dtheta for every
parameter.  Inputs are resident in device memory before the timed region starts.

Headline workload: 2D Maxwell (E_z, H_x, H_y) network with 128 Fourier frequencies
(sigma = 2) and 6 x 256 sine layers, 1,048,576 uniform points on [0,1]^3 -- the largest
single-GPU configuration of the benchmark set.  The BF16X3 path is the reported value;
the same three-product split with IEEE half parts (FP16X3, same matrix-core rate, 22
instead of 16 significant bits per operand) and the plain FP32 matrix-core path are timed
beside it.  The other configurations (Burgers,
1D Euler, Navier-Stokes, 2D Euler, and the 64-network Burgers sweep in one persistent
launch) are timed in the same run and reported as extra keys of the same JSON line.

Launch shapes: unless --no-autotune or an explicit shape is given, every configuration and
precision is timed with the shape the autotuner picks on this device before the timed
region (forward tile, split-backward sub-tile and work-group count for one network; work
item sizes and work-group count for the batched sweep); the chosen shape, the time of the
library's default shape and the number of candidates are reported beside each result, and
parity is measured at the chosen shape.

Roofline: the contractions are dense matrix products, so the bound is the matrix-core
rate.  For bf16x3 every logical product is three BF16 products, so the achieved rate is
3 x algorithmic FLOPs / time against the 2.5 PFLOP/s dense BF16 peak; FP32 is algorithmic
FLOPs / time against 157.3 TFLOP/s.  Algorithmic FLOPs per point: 2 C n_in n_out per
linear layer in the forward (2 d_in n_out for an identity-embedding first layer), the same
again for each weight gradient and for each input adjoint (none for the first layer).

Prints one JSON line.  --gpus above 1 is refused: the benchmark runs on one GPU (how the
points would shard over several is a design note, not a run).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "collocation points/sec for fused residual+grad step, BF16x3 vs FP32 at 1e-4 rel err"
PEAK = {"bf16": 2.5e15, "fp32": 157.3e12}   # dense matrix-core peaks, FLOP/s
HBM_PEAK = 8.0e12
TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "fp16x3": 1e-4}
N_PROD = {"bf16x3": 3, "fp16x3": 3, "fp32": 1}
PEAK_OF = {"bf16x3": "bf16", "fp16x3": "bf16", "fp32": "fp32"}   # FP16 dense peak = BF16


def channels(net, pde):
    """Jet channels that carry data (value, first derivatives, Laplacian)."""
    return 1 + net["d_in"] + (1 if pde.get("lap_mask", 0) else 0)


def kernel_flops(net, pde, n_points):
    """Algorithmic FLOPs per launch of each kernel kind, and of the whole step.

    A linear layer n_in -> n_out applied to C jet channels costs 2 C n_in n_out per point;
    the identity-embedding first layer costs 2 d_in n_out (its derivative channels are
    the weight columns).  Backward: the weight gradient costs the same as the layer, the
    input adjoint too, except for the first layer (inputs are not differentiated)."""
    from paper_2604_15645_amd import synth
    C = channels(net, pde)
    dims = synth.layer_dims(net)
    rff = net.get("n_freq", 0) > 0
    per_layer = []
    for li, (no, ni) in enumerate(dims):
        if li == 0 and not rff:
            per_layer.append(2 * net["d_in"] * no)
        else:
            per_layer.append(2 * C * ni * no)
    fwd = sum(per_layer)
    out = {"k_forward": fwd * n_points}
    hidden = [2 * per_layer[j] * n_points for j in range(1, len(dims) - 1)]
    out["k_backward"] = hidden[0] if hidden else 0
    out["k_backward_embed"] = per_layer[0] * n_points if rff else 0
    step = fwd + per_layer[-1] + per_layer[-1]  # forward, output-layer W grad and input adjoint
    step += sum(2 * per_layer[j] for j in range(1, len(dims) - 1))
    step += per_layer[0]  # first-layer weight gradient
    return out, step * n_points


def kernel_bytes(net, pde, n_points):
    """HBM bytes per launch of each kernel kind that this design moves between kernels
    (the pre-activation stash and the adjoints, C FP32 channels per neuron and point, plus
    the points): the traffic of the layer-by-layer backward, not a property of the method."""
    from paper_2604_15645_amd import synth
    C = channels(net, pde)
    dims = synth.layer_dims(net)
    jet = 4 * C
    widths = [no for no, _ in dims[:-1]]
    out = {"k_forward": (16 + jet * (sum(widths[:-1]) + widths[-1])) * n_points}
    if len(dims) > 2:
        no, ni = dims[1]
        out["k_backward"] = jet * (no + 2 * ni) * n_points
    out["k_backward_embed"] = (jet * dims[0][0] + 16) * n_points
    return out


def source_sha256():
    """Hash of the kernel and host sources (the counter summaries record the one they were
    taken on)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2604_15645_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(config, kernel):
    """HBM bytes per launch of `kernel` on this workload from the committed counter summary
    (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by the copy calibration), or None when no
    summary exists or the sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "%s_bf16x3_traffic.json" % config)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    k = rec.get("kernels", {}).get(kernel)
    if rec.get("source_sha256") != source_sha256() or k is None:
        return None
    return k["hbm_bytes_per_launch"]


def make_inputs(name, n_points, dev):
    import numpy as np
    import torch
    from paper_2604_15645_amd import synth
    case = synth.make_case(name, n_points=n_points)
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    anchors = [dict(a, points=t(a["points"]), targets=t(a["targets"])) for a in case["anchors"]]
    return case, t(case["params"]), t(case["B"]), t(case["points"]), anchors


def time_steps(case, params, B, pts, anchors, prec, steps, warmup, tune=None, per_kernel=True):
    """Mean ms per step over `steps` calls after `warmup` calls (HIP events on the stream
    the library launches on), the per-kernel record of the timed calls, and the outputs."""
    import torch
    from paper_2604_15645_amd import binding
    net, pde = case["net"], case["pde"]
    ws = binding.Workspace(pts.device)
    r = binding.residual_step(net, pde, params, B, pts, anchors, prec=prec, residual=True,
                              workspace=ws, tune=tune)
    out = dict(r)
    for _ in range(max(0, warmup - 1)):
        binding.residual_step(net, pde, params, B, pts, anchors, prec=prec, workspace=ws,
                              out=out, tune=tune)
    torch.cuda.synchronize()
    binding.timing_collect()          # drop anything recorded before the timed region
    binding.timing_enable(per_kernel)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        binding.residual_step(net, pde, params, B, pts, anchors, prec=prec, workspace=ws,
                              out=out, tune=tune)
    e1.record()
    torch.cuda.synchronize()
    binding.timing_enable(False)
    kernels = binding.timing_collect()
    ms = e0.elapsed_time(e1) / steps
    del ws
    return ms, kernels, out


def time_graph(case, params, B, pts, anchors, prec, steps, warmup, tune=None):
    """Mean ms per step of the same step captured once in a HIP graph and replayed
    (binding.StepGraph: every kernel of the step, one graph launch)."""
    import torch
    from paper_2604_15645_amd import binding
    g = binding.StepGraph(case["net"], case["pde"], params, B, pts, anchors, prec=prec, tune=tune)
    for _ in range(max(1, warmup)):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del g
    return ms


def tune_shape(case, params, B, pts, anchors, prec, cache):
    """The autotuner's launch shape for one network and precision, timed on this device
    (every candidate shape, median of three calls); returns (tune, record)."""
    from paper_2604_15645_amd import autotune
    tune, ms, table = autotune.tune_single(case["net"], case["pde"], params, B, pts, anchors, prec=prec,
                                           cache=cache, force=True)
    default = [r["ms"] for r in table if not any(r["tune"].values())]
    return tune, {"tune": tune, "ms": ms, "default_shape_ms": default[0] if default else None,
                  "candidates": len(table)}


def is_default(tune):
    return tune is None or not any(tune.values())


def relerr(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def parity(out, ref):
    import numpy as np
    lo = out["loss"].cpu().numpy()
    return {"residual": relerr(out["residual"].cpu().numpy(), ref["residual"]),
            "loss": float(np.max(np.abs(lo - ref["loss"]) / np.abs(ref["loss"]))),
            "grad": relerr(out["grad"].cpu().numpy(), ref["grad"])}


def bench_config(name, dev, steps, warmup, sample, fp32=True, cache=None):
    """One single-network configuration at full size: every precision with its autotuned
    launch shape (when a tune cache is given), matrix-core fractions of the whole step, and
    parity on a prefix of the points (oracle) at that shape."""
    import torch
    from oracle import oracle
    from paper_2604_15645_amd import binding, synth
    case, params, B, pts, anchors = make_inputs(name, None, dev)
    net, pde = case["net"], case["pde"]
    n = len(case["points"])
    n_total = n + sum(len(a["points"]) for a in case["anchors"])
    _, step_flops = kernel_flops(net, pde, n_total)
    rec = {"workload": describe(net, pde, n), "points": n}
    precs = ("bf16x3", "fp16x3", "fp32") if fp32 else ("bf16x3", "fp16x3")
    m = min(sample, n)
    ref = oracle.loss_grad(net, pde, case["params"], case["B"], case["points"][:m], case["anchors"])
    for prec in precs:
        tune, trec = tune_shape(case, params, B, pts, anchors, prec, cache) if cache else (None, None)
        ms, _, _ = time_steps(case, params, B, pts, anchors, prec, steps, warmup, tune=tune, per_kernel=False)
        gms = time_graph(case, params, B, pts, anchors, prec, steps, warmup, tune=tune)
        o = binding.residual_step(net, pde, params, B, pts[:m].contiguous(), anchors, prec=prec, tune=tune)
        torch.cuda.synchronize()
        rec[prec] = {"ms_per_step": ms, "points_per_s": n / (ms / 1e3),
                     "graph_ms_per_step": gms, "graph_points_per_s": n / (gms / 1e3),
                     "mfma_frac": N_PROD[prec] * step_flops / (ms / 1e3) / PEAK[PEAK_OF[prec]],
                     "parity": dict(parity(o, ref), tol=TOL[prec], sample_points=m)}
        if trec:
            rec[prec]["autotune"] = trec
    if fp32:
        rec["speedup_bf16x3_vs_fp32"] = rec["fp32"]["ms_per_step"] / rec["bf16x3"]["ms_per_step"]
    return rec


def bench_sweep(dev, steps, warmup, cache=None):
    """The 64 Burgers networks of uneven width, depth and point count in one persistent
    launch (pinn_batched_bwd, work-item sizes and grid from the autotuner when a tune cache
    is given), against the same networks as 64 separate calls."""
    import numpy as np
    import torch
    from oracle import oracle
    from paper_2604_15645_amd import binding, synth
    insts = synth.make_sweep()
    nets = [c["net"] for c in insts]
    pde = insts[0]["pde"]
    params = [torch.from_numpy(c["params"]).to(dev) for c in insts]
    pts = [torch.from_numpy(c["points"]).to(dev) for c in insts]
    n_tot = sum(len(c["points"]) for c in insts)
    flops = sum(kernel_flops(c["net"], c["pde"], len(c["points"]))[1] for c in insts)
    rec = {"workload": "64 Burgers networks, widths 32-256, depths 3-6, %d points in all" % n_tot,
           "points": n_tot, "alg_tflop": flops / 1e12}
    # parity: the smallest instance of each width class, whole gradient against the oracle
    pick = {}
    for i, c in enumerate(insts):
        w = c["net"]["widths"][0]
        if w not in pick or len(c["points"]) < len(insts[pick[w]]["points"]):
            pick[w] = i
    refs = {i: oracle.loss_grad(insts[i]["net"], pde, insts[i]["params"], None, insts[i]["points"],
                                want_residual=False) for i in sorted(pick.values())}
    for prec in ("bf16x3", "fp16x3", "fp32"):
        table, trec = None, None
        if cache:
            from paper_2604_15645_amd import autotune
            table, tms, log = autotune.tune_batched(nets, pde, params, pts, prec=prec, cache=cache, force=True)
            best = min(log, key=lambda r: r["ms"])
            trec = {"chunk_points": {str(k): v for k, v in best["chunks"].items()}, "grid": best["grid"],
                    "ms": tms, "default_shape_ms": log[0]["ms"], "candidates": len(log)}
        ws = binding.Workspace(dev)
        run = lambda: binding.batched_step(nets, pde, params, pts, prec=prec, workspace=ws, tune_table=table)
        out = run()
        for _ in range(max(0, warmup - 1)):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            out = run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        # the same networks as separate calls, one after the other
        ws1 = binding.Workspace(dev)
        single = lambda: [binding.residual_step(c["net"], pde, params[i], None, pts[i], (), prec=prec,
                                                residual=False, workspace=ws1)
                          for i, c in enumerate(insts)]
        single()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(max(1, steps // 4)):
            single()
        e1.record()
        torch.cuda.synchronize()
        ms1 = e0.elapsed_time(e1) / max(1, steps // 4)
        losses = out["losses"].cpu().numpy()
        worst = {"loss": 0.0, "grad": 0.0}
        for i, ref in refs.items():
            worst["loss"] = max(worst["loss"], float(np.max(np.abs(losses[i] - ref["loss"]) /
                                                            np.abs(ref["loss"]))))
            worst["grad"] = max(worst["grad"], relerr(out["grads"][i].cpu().numpy(), ref["grad"]))
        rec[prec] = {"ms_per_step": ms, "points_per_s": n_tot / (ms / 1e3),
                     "mfma_frac": N_PROD[prec] * flops / (ms / 1e3) / PEAK[PEAK_OF[prec]],
                     "separate_calls_ms": ms1, "speedup_vs_separate_calls": ms1 / ms,
                     "parity": dict(worst, tol=TOL[prec],
                                    instances=[int(i) for i in sorted(refs)])}
        if trec:
            rec[prec]["autotune"] = trec
        del ws, ws1
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="maxwell", help="burgers | euler | ns | maxwell")
    ap.add_argument("--points", type=int, default=0, help="override the point count")
    ap.add_argument("--sample", type=int, default=65536, help="CPU-baseline / parity prefix")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the other configurations and the batched sweep")
    ap.add_argument("--tile-points", type=int, default=0, help="forward tile points (0 = the library's)")
    ap.add_argument("--grid", type=int, default=0, help="work-group cap (0 = the library's)")
    ap.add_argument("--bwd-points", type=int, default=0,
                    help="split-backward sub-tile points (0 = the library's)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the library's default launch shapes instead of the autotuner's")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only (--gpus 1): the fused step is measured on one GPU's "
              "share of the points; runs on several GPUs are not provided", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2604_15645_amd import binding, synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "launches": 3}))
        return
    name = args.config
    n_points = args.points or synth.CONFIGS[name]["n_points"]
    case, params, B, pts, anchors = make_inputs(name, n_points, dev)
    net, pde = case["net"], case["pde"]
    n_total = n_points + sum(len(a["points"]) for a in case["anchors"])
    print("bench: %s, %d points" % (name, n_points), file=sys.stderr, flush=True)

    fixed = {"tile_points": args.tile_points, "grid": args.grid, "bwd_points": args.bwd_points}
    explicit = any(fixed.values())
    cache = None
    if not explicit and not args.no_autotune:
        import tempfile
        from paper_2604_15645_amd import autotune
        # a fresh cache per run: every shape is timed on this device, with this library
        cache = autotune.TuneCache(os.path.join(tempfile.mkdtemp(prefix="pinn_tune_"), "tune.json"))
    tunes, trecs = {}, {}
    for prec in ("bf16x3", "fp16x3") + (() if args.no_fp32 else ("fp32",)):
        if cache:
            tunes[prec], trecs[prec] = tune_shape(case, params, B, pts, anchors, prec, cache)
        elif explicit:
            # the split-role sub-tile exists in the split precisions only
            tunes[prec] = dict(fixed, bwd_points=0) if prec == "fp32" else fixed
        else:
            tunes[prec] = None
    tune = tunes["bf16x3"]
    print("bench: shapes %s" % json.dumps(tunes), file=sys.stderr, flush=True)
    ms16, k16, out16 = time_steps(case, params, B, pts, anchors, "bf16x3", args.steps, args.warmup, tune)
    ms_h, k_h, _ = time_steps(case, params, B, pts, anchors, "fp16x3", args.steps, args.warmup, tunes["fp16x3"])
    fp16x3 = {"value": n_points / (ms_h / 1e3), "ms_per_step": ms_h,
              "kernels_ms": {k: v[1] / v[0] for k, v in k_h.items()},
              **({"autotune": trecs["fp16x3"]} if "fp16x3" in trecs else {})}
    fp32 = None
    if not args.no_fp32:
        ms32, k32, _ = time_steps(case, params, B, pts, anchors, "fp32",
                                  max(2, args.steps // 4), min(args.warmup, 2), tunes["fp32"])
        fp32 = {"value": n_points / (ms32 / 1e3), "ms_per_step": ms32,
                "kernels_ms": {k: v[1] / v[0] for k, v in k32.items()},
                **({"autotune": trecs["fp32"]} if "fp32" in trecs else {})}
    print("bench: timed", file=sys.stderr, flush=True)

    # matrix-core roofline of the dominant kernel (largest summed time per step), from the
    # library's own per-launch events on the stream its kernels run on
    flops, step_flops = kernel_flops(net, pde, n_total)
    nbytes = kernel_bytes(net, pde, n_total)
    dom = max(k16, key=lambda k: k16[k][1])
    launches, tot = k16[dom]
    avg_ms = tot / launches
    alg = flops.get(dom, 0)
    n_prod = N_PROD["bf16x3"]
    roof = None
    if alg:
        mfma = n_prod * alg / (avg_ms / 1e3)
        # the committed counters were taken at the library's default shape
        is_full = n_points == synth.CONFIGS[name]["n_points"] and is_default(tune)
        roof = {"kernel": dom, "bound": "mfma", "achieved": mfma / 1e12, "peak": PEAK["bf16"] / 1e12,
                "unit": "TFLOP/s", "frac": mfma / PEAK["bf16"],
                "traffic": measured_traffic(name, dom) if is_full else None,
                "alg_flops_per_launch": alg, "n_prod": n_prod, "avg_launch_ms": avg_ms,
                "launches_per_step": launches / args.steps,
                "step_frac": n_prod * step_flops / (ms16 / 1e3) / PEAK["bf16"]}
        if nbytes.get(dom):
            roof["stash_bytes_per_launch"] = nbytes[dom]
            roof["stash_gbs"] = nbytes[dom] / (avg_ms / 1e3) / 1e9
            roof["stash_hbm_frac"] = nbytes[dom] / (avg_ms / 1e3) / HBM_PEAK

    result = {
        "metric": METRIC,
        "value": n_points / (ms16 / 1e3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms16,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3",
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (name, describe(net, pde, n_points)),
                   "points": n_points, "params": synth.param_count(net), "parallelism": "none",
                   "tune": tune or {}},
        "step_alg_tflop": step_flops / 1e12,
        "step_mfma_frac": n_prod * step_flops / (ms16 / 1e3) / PEAK["bf16"],
        "kernels_ms": {k: v[1] / v[0] for k, v in k16.items()},
        "kernel_launches_per_step": {k: v[0] / args.steps for k, v in k16.items()},
        "roofline": roof,
    }
    if "bf16x3" in trecs:
        result["autotune"] = trecs["bf16x3"]
    fp16x3["step_mfma_frac"] = n_prod * step_flops / (fp16x3["ms_per_step"] / 1e3) / PEAK["bf16"]
    result["fp16x3"] = fp16x3
    if fp32:
        result["fp32"] = fp32
        result["fp32"]["step_mfma_frac_fp32"] = step_flops / (fp32["ms_per_step"] / 1e3) / PEAK["fp32"]
        result["speedup_bf16x3_vs_fp32"] = fp32["ms_per_step"] / ms16

    if not args.no_cpu_baseline:
        from oracle import oracle
        m = min(args.sample, n_points)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        t0 = time.time()
        ref = oracle.loss_grad(net, pde, case["params"], case["B"], case["points"][:m],
                               case["anchors"], n_threads=threads)
        dt = time.time() - t0
        m1 = min(m, 1024)
        t0 = time.time()
        oracle.loss_grad(net, pde, case["params"], case["B"], case["points"][:m1], case["anchors"],
                         n_threads=1)
        dt1 = time.time() - t0
        result["cpu_baseline"] = {"value": m / dt, "unit": "points/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": "first %d of the %d points (+%d supervision points), "
                                            "FP64 loss and gradient, %.1f s" %
                                            (m, n_points, n_total - n_points, dt),
                                  "single_thread": {"value": m1 / dt1, "unit": "points/s",
                                                    "sample": "first %d points, %.1f s" % (m1, dt1)}}
        # parity at the benchmark's own shape: the prefix through the GPU path
        par = {}
        ptsm = pts[:m].contiguous()
        for prec in ("bf16x3", "fp16x3", "fp32"):
            o = binding.residual_step(net, pde, params, B, ptsm, anchors, prec=prec, tune=tunes.get(prec))
            torch.cuda.synchronize()
            par[prec] = dict(parity(o, ref), tol=TOL[prec])
        full = out16["residual"].cpu().numpy()[:m]
        par["bf16x3_full_run_residual"] = relerr(full, ref["residual"])
        result["parity_vs_oracle"] = par
        print("bench: cpu baseline and parity done", file=sys.stderr, flush=True)

    if not args.no_others and not args.points and not explicit:
        others = {}
        for other in ("burgers", "euler", "ns", "maxwell", "euler2d"):
            if other == name:
                continue
            others[other] = bench_config(other, dev, args.steps, args.warmup, 8192,
                                         fp32=not args.no_fp32, cache=cache)
            print("bench: %s done" % other, file=sys.stderr, flush=True)
        result["configs"] = others
        result["sweep"] = bench_sweep(dev, max(3, args.steps // 2), args.warmup, cache=cache)
        print("bench: sweep done", file=sys.stderr, flush=True)
    print(json.dumps(result))


def describe(net, pde, n):
    emb = "RFF m=%d" % net["n_freq"] if net.get("n_freq") else "identity"
    if net.get("periodic_mask"):
        emb = "periodic " + ",".join("xyt"[k] if net["d_in"] == 3 else "xt"[k]
                                     for k in range(net["d_in"]) if (net["periodic_mask"] >> k) & 1)
    return "%s, %s, %dx%d %s -> %d%s, %d points" % (
        pde["pde"], emb, len(net["widths"]), max(net["widths"]), net["act"], net["d_out"],
        ", RWF" if net.get("rwf") else "", n)


if __name__ == "__main__":
    main()
