#!/usr/bin/env python3
"""Benchmark: Gpixel-iterations/s of the coarse-to-fine TV-L1 flow solve on one MI355X.

Workload (default): one synthetic 640x480 FP32 pair (rich texture, piecewise-constant motion),
5-level pyramid (factor 1/2), 5 warps per level, 50 pADMM iterations per warp.  A step is one
whole solve (pyramid, warps, iterations, energy / gap) with the frames already resident in HBM;
the solve is replayed from a hipGraph.  value = pixel-iterations of a step / step time.

Also reported on the same JSON line:
  roofline      the dominant kernel: the ADMM iteration kernel of the finest level (about three
                quarters of all pixel-iterations; the autotuner picks one-pass or K-iteration tiles
                per level).  Algorithmic bytes of one launch = 76 B per pixel (12 FP32 planes read,
                7 written, once per launch whatever K it advances) x the level's pixels; launch
                duration from HIP events on the solve stream around each warp's block of iteration
                launches, averaged over instrumented solves; peak = 8 TB/s HBM.  traffic = HBM bytes
                per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs (calibrated against a
                plain copy), when they were taken on the current kernel source, else null.
  cpu_baseline  the FP64 NumPy oracle on the same workload (solved twice, about 10-15 s), one core
  per_level     Gpixel-iter/s of each level's iteration blocks

Other modes:
  --save-tuning F / --load-tuning F   write the autotuned per-level kernel choices to F, or apply
                                      them from F instead of tuning (for profiler runs)
  --calibrate-copy MB                 time a plain device-to-device copy of MB MiB (the reference
                                      kernel for the HBM counter calibration) and exit
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


def kernel_sha():
    h = hashlib.sha256()
    for f in ("admm.hip", "admm_tb.hip", "admm_args.hpp"):
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
    `cpu_iters` iterations per warp (default: all of them), solved `cpu_reps` times."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np
    from oracle import Params, solve_pair
    from oracle.pyramid import level_shapes
    I0 = pair.I0.astype(np.float32).astype(np.float64)
    I1 = pair.I1.astype(np.float32).astype(np.float64)
    iters = args.cpu_iters or args.iters
    p = Params(scheme=args.scheme, levels=args.levels, warps=args.warps, iters=iters)
    t0 = time.perf_counter()
    for _ in range(args.cpu_reps):
        solve_pair(I0, I1, p)
    dt = time.perf_counter() - t0
    px = sum(h * w for h, w in level_shapes(I0.shape[0], I0.shape[1], args.levels))
    pxi = px * args.warps * iters * args.cpu_reps
    return {"value": pxi / dt / 1e9, "unit": "Gpixel-iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{args.cpu_reps} x the {I0.shape[1]}x{I0.shape[0]} solve, {args.levels} levels x {args.warps} "
                      f"warps x {iters} iterations ({pxi / 1e6:.1f} M px-iter, {dt:.1f} s, FP64 NumPy, 1 thread)"}


def calibrate_copy(mb, steps):
    """Plain device-to-device copies of `mb` MiB: the kernel of known traffic (mb MiB read and mb
    MiB written per launch) that scales the HBM counters."""
    import torch
    n = mb * (1 << 20) // 4
    x = torch.ones(n, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, steps)):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(1, steps)
    print(json.dumps({"copy_MiB": mb, "ms": round(dt * 1e3, 4), "GBs": round(2 * mb * (1 << 20) / dt / 1e9, 1)}),
          flush=True)


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
    ap.add_argument("--cpu-iters", type=int, default=0, help="iterations per warp of the oracle sample (0: all)")
    ap.add_argument("--cpu-reps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--save-tuning", default=None)
    ap.add_argument("--load-tuning", default=None)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; pairs would be sharded across GPUs with no "
              "communication, and no multi-GPU figure is produced.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2011_10979_amd as fm

    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy, args.steps)
        return

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
    if args.load_tuning:
        with open(args.load_tuning) as fh:
            tuning = json.load(fh)
        for key, ch in tuning.items():
            ctx.set_choice(key, ch["mode"], ch["K"], ch["rows"])
        print(f"[bench] loaded tuning: {tuning}", file=sys.stderr, flush=True)
    elif not args.no_autotune:
        # one-time choice of the iteration kernel per level shape (outside the timed region)
        tuning = {k: v_["choice"] for k, v_ in ctx.autotune(args.H, args.W, params).items()}
        print(f"[bench] autotuned: {tuning}", file=sys.stderr, flush=True)
    if args.save_tuning and tuning is not None:
        with open(args.save_tuning, "w") as fh:
            json.dump(tuning, fh)
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
    lvl_iters = [0] * args.levels
    reps = 3
    for _ in range(reps):
        ctx.solve(I0, I1, p_inst, u=u, v=v)
        s = ctx.stats()
        for l in range(args.levels):
            lvl_ms[l] += s["iter_ms"][l]
            lvl_iters[l] += s["iterations"][l]
    ctx.set_stats(False)
    per_level = []
    for l, (a, b) in enumerate(shapes):
        gpx = a * b * lvl_iters[l] / (lvl_ms[l] * 1e-3) / 1e9 if lvl_ms[l] > 0 else None
        per_level.append({"level": l, "H": a, "W": b, "Gpx_iter_s": gpx,
                          "us_per_iter": 1e3 * lvl_ms[l] / max(1, lvl_iters[l])})

    has_w = params.beta > 0
    roof = None
    if args.scheme in ("padmm", "rpadmm2"):
        # Dominant kernel: the iteration kernel of level 0.  Kernel launches per warp follow the
        # level's choice: `iters` for the one-pass kernel, ceil(iters / K) for K-iteration tiles,
        # one for a resident tile.
        def launches_per_warp(l):
            a, b = shapes[l]
            key = f"{a}x{b}{'w' if has_w else ''}i{args.iters}"
            ch = (tuning or {}).get(key, {"mode": 1, "K": 1})
            if ch["mode"] == 1:
                return args.iters, ch
            if ch["K"] == 0:
                return 1, ch
            return -(-args.iters // ch["K"]), ch
        per_px = BYTES_PER_PX_LAUNCH[has_w]
        n0, ch0 = launches_per_warp(0)
        n0 *= args.warps * reps
        launch_s = lvl_ms[0] * 1e-3 / n0
        bytes_launch = per_px * shapes[0][0] * shapes[0][1]
        achieved = bytes_launch / launch_s / 1e9
        traffic = measured_traffic(f"{args.W}x{args.H}")
        all_launches = sum(launches_per_warp(l)[0] for l in range(args.levels)) * args.warps
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"ADMM iteration kernel, level 0 ({shapes[0][1]}x{shapes[0][0]}), choice {ch0}",
                "per_unit": f"{per_px} B per pixel per launch", "bytes_per_launch": bytes_launch,
                "avg_launch_us": round(launch_s * 1e6, 3), "launches_per_step_level0": n0 // reps,
                "iteration_launches_per_step": all_launches,
                # the same pixel-iterations priced at one HBM pass per iteration (76 B per pixel-iteration)
                "one_pass_equivalent_GBs": round(per_px * shapes[0][0] * shapes[0][1] * lvl_iters[0]
                                                 / (lvl_ms[0] * 1e-3) / 1e9, 1)}

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
