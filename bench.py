#!/usr/bin/env python3
"""Benchmark: Gpixel-iterations/s of the coarse-to-fine TV-L1 flow solve on one MI355X.

Workload (default): one synthetic 640x480 FP32 pair (rich texture, piecewise-constant motion),
5-level pyramid (factor 1/2), 5 warps per level, 50 pADMM iterations per warp.  A step is one
whole solve (pyramid, warps, iterations, energy / gap) with the frames already resident in HBM;
the solve is replayed from a hipGraph.  value = pixel-iterations of a step / step time.

Also reported on the same JSON line:
  roofline      the ADMM iteration kernels (the dominant kernels; the autotuner picks one-pass or
                K-iteration tiles per level): 76 algorithmic bytes per pixel per launch (12 FP32
                planes read, 7 written) x pixels x launches / their time, timed with HIP events
                around each warp's iteration block during instrumented solves, against the 8 TB/s
                HBM peak; one_pass_equivalent_GBs counts 76 B per pixel-iteration instead
  cpu_baseline  the FP64 NumPy oracle on a bounded sample of the same workload, one core
  per_level     Gpixel-iter/s of each level's iteration blocks
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
# FP32 planes read + written per pixel by one launch of an iteration kernel (increment form):
# reads du, dv, s, q1x, q1y, q2x, q2y, I_x, I_y, I_t, u0, v0 (+ w, px, py); writes the 7 (10) state planes
BYTES_PER_PX_LAUNCH = {False: 4 * (12 + 7), True: 4 * (15 + 10)}
BYTES_PER_PX_ITER_ONEPASS = BYTES_PER_PX_LAUNCH   # one launch = one iteration for the one-pass kernel


def kernel_sha():
    h = hashlib.sha256()
    for f in ("admm.hip", "admm_tb.hip", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2011_10979_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the iteration kernel from committed rocprofv3 counter runs, if they
    were taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = d.get(workload)
    if not e or e.get("kernel_sha") != kernel_sha():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(pair, args):
    """Time the oracle on a bounded sample of the workload: the full pyramid and warps with
    `cpu_iters` iterations per warp instead of 50."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np
    from oracle import Params, solve_pair
    from oracle.pyramid import level_shapes
    I0 = pair.I0.astype(np.float32).astype(np.float64)
    I1 = pair.I1.astype(np.float32).astype(np.float64)
    p = Params(scheme=args.scheme, levels=args.levels, warps=args.warps, iters=args.cpu_iters)
    t0 = time.perf_counter()
    solve_pair(I0, I1, p)
    dt = time.perf_counter() - t0
    px = sum(h * w for h, w in level_shapes(I0.shape[0], I0.shape[1], args.levels))
    pxi = px * args.warps * args.cpu_iters
    return {"value": pxi / dt / 1e9, "unit": "Gpixel-iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{I0.shape[1]}x{I0.shape[0]}, {args.levels} levels x {args.warps} warps x "
                      f"{args.cpu_iters} iterations ({pxi / 1e6:.1f} M px-iter, {dt:.1f} s, FP64 NumPy, 1 thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scheme", default="padmm")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--levels", type=int, default=5)
    ap.add_argument("--warps", type=int, default=5)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--H", type=int, default=480)
    ap.add_argument("--W", type=int, default=640)
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; pairs would be sharded across GPUs with no "
              "communication, and no multi-GPU figure is produced.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2011_10979_amd as fm

    dev = torch.device("cuda:0")
    pair = synth.vga_pair(seed=1, H=args.H, W=args.W)
    I0 = torch.from_numpy(pair.I0.astype(np.float32)).to(dev)
    I1 = torch.from_numpy(pair.I1.astype(np.float32)).to(dev)
    ctx = fm.Context(0)
    params = fm.Params(scheme=args.scheme, storage=args.storage, levels=args.levels, warps=args.warps,
                       iters=args.iters, use_graph=1)
    u = torch.empty_like(I0)
    v = torch.empty_like(I0)
    tuning = None
    if not args.no_autotune:
        # one-time choice of the iteration kernel per level shape (outside the timed region)
        tuning = {k: v_["choice"] for k, v_ in ctx.autotune(args.H, args.W, params).items()}
        print(f"[bench] autotuned: {tuning}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        ctx.solve(I0, I1, params, u=u, v=v)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        _, _, res = ctx.solve(I0, I1, params, u=u, v=v)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_event = start.elapsed_time(end)
    ms_step = max(ms_event, wall * 1e3) / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step", file=sys.stderr, flush=True)

    shapes = []
    h, w = args.H, args.W
    for _ in range(args.levels):
        shapes.append((h, w))
        h, w = (h + 1) // 2, (w + 1) // 2
    px_iter = sum(a * b for a, b in shapes) * args.warps * args.iters
    value = px_iter / (ms_step * 1e-3) / 1e9

    # Per-level iteration timing: the same solve with direct launches and HIP events around each
    # warp's block of iteration kernels on the solve stream.
    ctx.set_stats(True)
    p_inst = fm.Params(**{**params.__dict__, "use_graph": 0})
    lvl_ms = [0.0] * args.levels
    lvl_launch = [0] * args.levels
    reps = 3
    for _ in range(reps):
        ctx.solve(I0, I1, p_inst, u=u, v=v)
        s = ctx.stats()
        for l in range(args.levels):
            lvl_ms[l] += s["iter_ms"][l]
            lvl_launch[l] += s["iter_launches"][l]
    ctx.set_stats(False)
    per_level = []
    for l, (a, b) in enumerate(shapes):
        gpx = a * b * lvl_launch[l] / (lvl_ms[l] * 1e-3) / 1e9 if lvl_ms[l] > 0 else None
        per_level.append({"level": l, "H": a, "W": b, "Gpx_iter_s": gpx,
                          "us_per_iter": 1e3 * lvl_ms[l] / max(1, lvl_launch[l])})

    has_w = params.beta > 0
    roof = None
    if args.scheme in ("padmm", "rpadmm2"):
        # Dominant kernel = the iteration kernel (one-pass or K-iteration tiles, per the tuning).
        # Algorithmic bytes of one launch: the 12 (15 with the w / p block) FP32 planes it reads
        # and the 7 (10) it writes, once per pixel of the level, whatever K the launch advances.
        per_px = BYTES_PER_PX_LAUNCH[has_w]
        tot_bytes = 0.0
        tot_ms = 0.0
        tot_launches = 0
        tot_pxiter = 0.0
        for l, (a, b) in enumerate(shapes):
            key = f"{a}x{b}{'w' if has_w else ''}i{args.iters}"
            ch = (tuning or {}).get(key, {"mode": 1, "K": 1})
            if ch["mode"] == 1:
                per_warp = args.iters
            elif ch["K"] == 0:
                per_warp = 1                                   # resident: a warp in one launch
            else:
                per_warp = -(-args.iters // ch["K"])
            n = per_warp * args.warps * reps
            tot_launches += n
            tot_bytes += per_px * a * b * n
            tot_ms += lvl_ms[l]
            tot_pxiter += a * b * lvl_launch[l]
        launch_s = tot_ms * 1e-3 / max(1, tot_launches)
        achieved = tot_bytes / (tot_ms * 1e-3) / 1e9
        traffic = measured_traffic(f"{args.W}x{args.H}")
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "admm iteration kernels (tuned per level)",
                "per_unit": f"{per_px} B per pixel per launch",
                "avg_launch_us": round(launch_s * 1e6, 3), "launches_per_step": tot_launches // reps,
                "one_pass_equivalent_GBs": round(BYTES_PER_PX_ITER_ONEPASS[has_w] * tot_pxiter
                                                 / (tot_ms * 1e-3) / 1e9, 1)}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(pair, args)

    line = {
        "metric": "Gpixel-iter/s (coarse-to-fine TV-L1 flow solve, pixel-iterations over all levels)",
        "value": round(value, 3), "unit": "Gpixel-iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.storage == "f32" else "f32 (f16-stored pyramids)",
        "data": "synthetic",
        "config": {"workload": f"{args.W}x{args.H} pair, {args.levels}-level pyramid x {args.warps} warps x "
                               f"{args.iters} iterations, {args.scheme}",
                   "H": args.H, "W": args.W, "levels": args.levels, "warps": args.warps, "iters": args.iters,
                   "scheme": args.scheme, "storage": args.storage, "px_iter_per_step": px_iter,
                   "graph": True, "autotuned": tuning},
        "energy": res["energy"], "gap": res["gap"],
        "per_level": per_level,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
