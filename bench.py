"""Benchmark of the fused PINN residual + parameter-gradient step on one MI355X.

A step is one pinn_residual_bwd call over the whole synthetic collocation set: embedding
jets, every hidden layer, output layer, PDE residual, loss, and dL/dtheta for every
parameter.  Inputs are resident in device memory before the timed region starts.

Default workload: 2D Maxwell (E_z, H_x, H_y) network with 128 Fourier frequencies
(sigma = 2) and 6 x 256 sine layers, 1,048,576 uniform points on [0,1]^3 -- the largest
single-GPU configuration of the benchmark set.  The BF16X3 path is the reported value;
the plain FP32 matrix-core path is timed beside it.

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
TOL = {"fp32": 1e-5, "bf16x3": 1e-4}


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
    """Algorithmic HBM bytes per launch of each kernel kind: the jets that must cross HBM
    between the kernels (C FP32 channels per neuron and point), plus the points.

    Forward: points in, pre-activation jets of the hidden layers the backward reads (all but
    the last) out, adjoint jets of the last hidden layer out.  Hidden-layer backward: the
    layer's output adjoint and its input pre-activations in, the input adjoint out.
    Embedding-layer backward: its output adjoint and the points in."""
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


def measured_traffic(config, kernel):
    """HBM bytes per launch of `kernel` on this workload from the committed counter summary
    (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by the copy calibration), or None when no
    summary exists or the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_bf16x3_traffic.json" % config)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_2604_15645_amd", "csrc", "pinn_kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    k = rec.get("kernels", {}).get(kernel)
    if rec.get("source_sha256") != sha or k is None:
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


def time_steps(case, params, B, pts, anchors, prec, steps, warmup, tune=None):
    import torch
    from paper_2604_15645_amd import binding
    net, pde = case["net"], case["pde"]
    ws = binding.Workspace(pts.device)
    out = {}
    r = binding.residual_step(net, pde, params, B, pts, anchors, prec=prec, residual=True,
                              workspace=ws, tune=tune)
    out = dict(r)
    for _ in range(max(0, warmup - 1)):
        binding.residual_step(net, pde, params, B, pts, anchors, prec=prec, workspace=ws,
                              out=out, tune=tune)
    torch.cuda.synchronize()
    binding.timing_collect()          # drop anything recorded before the timed region
    binding.timing_enable(True)
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
    res = {k: v for k, v in out.items()}
    del ws
    return ms, kernels, res


def relerr(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


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
    ap.add_argument("--tile-points", type=int, default=0, help="forward tile points (0 = the library's)")
    ap.add_argument("--grid", type=int, default=0, help="work-group cap (0 = the library's)")
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

    tune = {"tile_points": args.tile_points, "grid": args.grid} if args.tile_points or args.grid else None
    ms16, k16, out16 = time_steps(case, params, B, pts, anchors, "bf16x3", args.steps, args.warmup, tune)
    fp32 = None
    if not args.no_fp32:
        ms32, k32, out32 = time_steps(case, params, B, pts, anchors, "fp32",
                                      max(2, args.steps // 4), min(args.warmup, 2))
        fp32 = {"value": n_points / (ms32 / 1e3), "ms_per_step": ms32,
                "kernels_ms": {k: v[1] / v[0] for k, v in k32.items()}}

    # roofline of the dominant kernel (largest summed time per step): the bound is the
    # resource whose peak gives the longer lower limit on the launch (HBM bytes at 8 TB/s or
    # bf16 matrix-core FLOPs at 2.5 PFLOP/s); the other resource's figures are reported too
    flops, step_flops = kernel_flops(net, pde, n_total)
    nbytes = kernel_bytes(net, pde, n_total)
    dom = max(k16, key=lambda k: k16[k][1])
    launches, tot = k16[dom]
    avg_ms = tot / launches
    alg = flops.get(dom, 0)
    alg_b = nbytes.get(dom, 0)
    n_prod = 3  # BF16X3: three bf16 matrix-core products per logical FP32 product
    roof = None
    if alg and alg_b:
        mfma = n_prod * alg / (avg_ms / 1e3)
        hbm = alg_b / (avg_ms / 1e3)
        hbm_bound = alg_b / HBM_PEAK >= n_prod * alg / PEAK["bf16"]
        traffic = measured_traffic(name, dom) if n_points == synth.CONFIGS[name]["n_points"] else None
        if hbm_bound:
            roof = {"kernel": dom, "bound": "hbm", "achieved": hbm / 1e9, "peak": HBM_PEAK / 1e9,
                    "unit": "GB/s", "frac": hbm / HBM_PEAK, "traffic": traffic,
                    "mfma_achieved_tflops": mfma / 1e12, "mfma_frac": mfma / PEAK["bf16"]}
        else:
            roof = {"kernel": dom, "bound": "mfma", "achieved": mfma / 1e12, "peak": PEAK["bf16"] / 1e12,
                    "unit": "TFLOP/s", "frac": mfma / PEAK["bf16"], "traffic": traffic,
                    "hbm_achieved_gbs": hbm / 1e9, "hbm_frac": hbm / HBM_PEAK}
        roof.update({"alg_bytes_per_launch": alg_b, "alg_flops_per_launch": alg, "n_prod": n_prod,
                     "avg_launch_ms": avg_ms})

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
                   **({"tune": tune} if tune else {})},
        "step_alg_tflop": step_flops / 1e12,
        "step_mfma_frac": n_prod * step_flops / (ms16 / 1e3) / PEAK["bf16"],
        "kernels_ms": {k: v[1] / v[0] for k, v in k16.items()},
        "kernel_launches_per_step": {k: v[0] / args.steps for k, v in k16.items()},
        "roofline": roof,
    }
    if fp32:
        result["fp32"] = fp32
        result["fp32"]["step_mfma_frac_fp32"] = step_flops / (fp32["ms_per_step"] / 1e3) / PEAK["fp32"]
        result["speedup_bf16x3_vs_fp32"] = fp32["ms_per_step"] / ms16

    if not args.no_cpu_baseline:
        from oracle import oracle
        m = min(args.sample, n_points)
        sample = dict(case, points=case["points"][:m])
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        t0 = time.time()
        ref = oracle.loss_grad(net, pde, case["params"], case["B"], sample["points"],
                               case["anchors"], n_threads=threads)
        dt = time.time() - t0
        result["cpu_baseline"] = {"value": m / dt, "unit": "points/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": "first %d of the %d points (+%d supervision points), "
                                            "FP64 loss and gradient, %.1f s" %
                                            (m, n_points, n_total - n_points, dt)}
        # parity at the benchmark's own shape: the prefix through the GPU path
        par = {}
        ptsm = pts[:m].contiguous()
        for prec in ("bf16x3", "fp32"):
            o = binding.residual_step(net, pde, params, B, ptsm, anchors, prec=prec)
            torch.cuda.synchronize()
            g = o["grad"].cpu().numpy()
            lo = o["loss"].cpu().numpy()
            rs = o["residual"].cpu().numpy()
            par[prec] = {"residual": relerr(rs, ref["residual"]),
                         "loss": float(np.max(np.abs(lo - ref["loss"]) / np.abs(ref["loss"]))),
                         "grad": relerr(g, ref["grad"]), "tol": TOL[prec]}
        full = out16["residual"].cpu().numpy()[:m]
        par["bf16x3_full_run_residual"] = relerr(full, ref["residual"])
        result["parity_vs_oracle"] = par
    print(json.dumps(result))


def describe(net, pde, n):
    emb = "RFF m=%d" % net["n_freq"] if net.get("n_freq") else "identity"
    return "%s, %s, %dx%d %s -> %d%s, %d points" % (
        pde["pde"], emb, len(net["widths"]), max(net["widths"]), net["act"], net["d_out"],
        ", RWF" if net.get("rwf") else "", n)


if __name__ == "__main__":
    main()
