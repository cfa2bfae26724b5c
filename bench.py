#!/usr/bin/env python3
"""Benchmark of the coarse-to-fine TV-L1 flow solvers on one MI355X.

Default workload (--mode batch): 64 synthetic pairs of uneven sizes (W ~ U[128, 1280], H ~ U[96, 720],
seeds 1000 + k; even k piecewise-constant motion, odd k rotation + zoom with occlusions), pyramid
depth by size, 5 warps x 50 pADMM iterations per level, FP32, solved together by the batched path
(autotuned stage choices, graph replay).  A step is one batched solve of all 64 pairs with the frames
already resident in HBM; value = pixel-iterations of all pairs and levels / step time.

Also reported on the same JSON line:
  pairs_per_s, per_level     pairs per second; Gpixel-iter/s and launch time of each level's stage
  plain_sequential           the same 64 pairs as 64 plain solves in turn (built-in plan; tiles at
                             every level, with a bitwise comparison against the batched flows)
  roofline                   the dominant kernel, the batched K-iteration tile kernel (every stage):
                             algorithmic bytes of the pixel-iterations one launch advances (68 B per
                             pixel-iteration, one pass per iteration) / average launch duration from
                             HIP events on the solve stream, against 8 TB/s; beside it the one-pass
                             figure (76 B per pixel per launch, a launch makes one pass for all K
                             iterations) and, when a rocprofv3 counter record of the same kernel
                             source and stage choices exists, the DRAM traffic per launch
  serving                    a Poisson trace (200 pairs/s, 1000 requests after 100) through the
                             continuous-batching engine with frames uploaded per request: pairs/s, p50 /
                             p99 latency, and the capacity with 300 requests arriving at once
  oracle_check               every batched flow against the FP64 oracle (max |du|, |dv|, pixels above
                             1e-4 px, mean and p99.9 endpoint error)
  cpu_baseline               the oracle on one core (the 8 smallest pairs in turn);
  cpu_baseline_all_cores     the oracle on all 64 pairs, one process per pair on the host's cores

Other modes:
  --mode single     one pair solved repeatedly: 640x480 (5 levels), or --pair hd for the 1920x1080
                    precision-form workload (6 levels; --storage f16 for FP16-stored pyramids); per-level
                    rates, roofline of the level-0 iteration kernel, oracle CPU baseline
  --mode serve      Poisson arrivals (mean 200 pairs/s, seed 7) of pairs drawn from a pool of 10
                    pre-generated pairs per size (320x240, 640x480, 1024x436, 1280x720, 1920x1080 with
                    probabilities 0.3, 0.3, 0.2, 0.1, 0.1), 2000 requests after 200 warm-up ones, served
                    by the continuous-batching engine (8 GiB budget), frames uploaded per request (unless
                    --no-ingest); value = completed pairs/s, with p50 / p99 latency; the same trace
                    through a one-at-a-time plain-solve server beside it
  --mode batch --batch-only [--no-autotune]   the batched solve alone (for profiler runs)
  --mode compare    every scheme of Sec. 4 (pADMM, rpADMMI, rpADMMII, Zach-pADMM, pDR, ALG1) on the
                    same synthetic pair (--pair vga or hd): time per solve, endpoint / angular error
                    against the ground-truth motion, energy and gap at equal iteration counts
  --save-tuning F / --load-tuning F   single mode: write the autotuned per-level kernel choices to F,
                                      or apply them from F instead of tuning (for profiler runs)
  --save-batch-tuning F / --load-batch-tuning F   the same for the batched stage choices
  --choice KEY=MODE,K,ROWS            single mode: then pin one level shape's choice
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
# Algorithmic HBM bytes of one ADMM-family iteration per pixel in its plain form (one pass per
# iteration, FP32): read 7 state planes (u, v, s, q1x, q1y, q2x, q2y) and I_x, I_y, I_t, write the 7
# state planes; with the illumination field 3 more state planes (w, p_x, p_y) each way.
BYTES_PER_PX_ITER = {False: 4 * (10 + 7), True: 4 * (13 + 10)}


# pDR / ALG1 tile kernels, per launch: reads X, X bar, y, I_x, I_y, I_t, u0, v0; writes X, X bar, y, Theta
# (for ALG1 this is also one iteration done in one pass)
PDR_TB_BYTES_PER_PX_LAUNCH = {False: 4 * ((2 + 2 + 4 + 5) + (2 + 2 + 4 + 1)), True: 4 * ((3 + 3 + 6 + 5) + (3 + 3 + 6 + 1))}
# pDR / ALG1 per pixel-iteration in one fused pass (plain form): read X, X bar, y and I_x, I_y, I_t,
# write X, X bar, y
PDR_TB_BYTES_PER_PX_ITER = {False: 4 * ((2 + 2 + 4 + 3) + (2 + 2 + 4)), True: 4 * ((3 + 3 + 6 + 3) + (3 + 3 + 6))}


def pdr_bytes_per_px_iter(has_w, sweeps):
    """FP32 planes one pDR iteration reads and writes per pixel over its 2n + 1 passes (n sweeps):
    rhs + first red half sweep, n - 1 (black, red) pairs plus the last black half sweep, and the
    final pass (last red half sweep, resolvent, dual update)."""
    if has_w:
        rhs, colour, final = 12 + 4.5, 6 + 1.5, 20 + 11.5
    else:
        rhs, colour, final = 8 + 3, 4 + 1, 15 + 8
    return 4 * (rhs + (2 * sweeps - 1) * colour + final)


def kernel_sha():
    """Hash of the iteration kernels' sources and of the tile planner (which sets the tiles a launch
    loads, and so its traffic)."""
    h = hashlib.sha256()
    for f in ("admm.hip", "admm_tb.hip", "admm_rows.hip", "admm_args.hpp", "tb_plan.cpp", "geometry.cpp"):
        with open(os.path.join(ROOT, "paper_2011_10979_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, choice):
    """HBM bytes per launch of the level-0 iteration kernel from committed rocprofv3 counter runs,
    if they were taken on the current kernel and planner source with the same level-0 choice
    (mode, K, tile width) as this run (else None).  The record holds one entry per measured choice:
    the autotuner's pick among candidates within a percent of each other varies between runs."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = d.get(workload)
    if not e or e.get("kernel_sha") != kernel_sha() or not choice:
        return None
    keys = ("mode", "K", "rows")
    for m in e.get("entries", []):
        c = m.get("choice") or {}
        if all(c.get(k) == choice.get(k) for k in keys):
            return m.get("bytes_per_launch")
    return None


def host_cpu():
    """The host's CPU model and logical CPU count, as the kernel reports them."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model} ({os.cpu_count()} logical CPUs)"


def cpu_baseline(pair, args):
    """Time the oracle on a bounded sample of the workload: the full pyramid and warps with
    `cpu_iters` iterations per warp (default: all of them), solved `cpu_reps` times, with every
    BLAS / OpenMP pool held to one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import Params, solve_pair
    from oracle.pyramid import level_shapes
    I0 = pair.I0.astype(np.float32).astype(np.float64)
    I1 = pair.I1.astype(np.float32).astype(np.float64)
    iters = args.cpu_iters or args.iters
    p = Params(scheme=args.scheme, levels=args.levels, warps=args.warps, iters=iters)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(args.cpu_reps):
            solve_pair(I0, I1, p)
        dt = time.perf_counter() - t0
    px = sum(h * w for h, w in level_shapes(I0.shape[0], I0.shape[1], args.levels))
    pxi = px * args.warps * iters * args.cpu_reps
    return {"value": pxi / dt / 1e9, "unit": "Gpixel-iter/s", "cores": 1, "kind": "oracle", "host": host_cpu(),
            "sample": f"{args.cpu_reps} x the {I0.shape[1]}x{I0.shape[0]} solve, {args.levels} levels x {args.warps} "
                      f"warps x {iters} iterations ({pxi / 1e6:.1f} M px-iter, {dt:.1f} s, FP64 NumPy, 1 thread)"}


def roofline(ms, launches, iters, px, has_w, kernel, traffic, reps, per_iter=None, per_launch=None):
    """HBM roofline of an iteration kernel from event-timed blocks of its launches.  achieved =
    algorithmic bytes of the pixel-iterations one launch advances (`per_iter` B per pixel-iteration,
    one pass per iteration) / average launch duration, against 8 TB/s; a launch of K iterations makes
    one pass for all K, so this can exceed the peak.  Beside it the one-pass figure (`per_launch` B
    per pixel per launch) and, with `traffic` (measured DRAM bytes per launch), the DRAM rate."""
    per_iter = per_iter or BYTES_PER_PX_ITER[has_w]
    per_launch = per_launch or BYTES_PER_PX_LAUNCH[has_w]
    launch_s = ms * 1e-3 / max(1, launches)
    pxi_launch = px * iters / max(1, launches)
    achieved = per_iter * pxi_launch / launch_s / 1e9
    one_pass = per_launch * px / launch_s / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
         "traffic_source": ("looked up: profiles/traffic.json (rocprofv3 FETCH_SIZE / WRITE_SIZE runs on this kernel "
                            "source and choice, copy-calibrated)") if traffic else None,
         "kernel": kernel, "per_unit": f"{per_iter} B per pixel-iteration", "px_iter_per_launch": round(pxi_launch),
         "bytes_per_launch": round(per_iter * pxi_launch), "avg_launch_us": round(launch_s * 1e6, 3),
         "launches_per_step_level0": launches // reps,
         "one_pass_per_launch": {"per_unit": f"{per_launch} B per pixel per launch", "GBs": round(one_pass, 1),
                                 "frac": round(one_pass / HBM_PEAK_GBS, 4)}}
    if traffic:
        r["dram_GBs"] = round(traffic / launch_s / 1e9, 1)
        r["dram_frac"] = round(r["dram_GBs"] / HBM_PEAK_GBS, 4)
    return r


def _gen_batch_pair(k):
    import synth
    p = synth.batch_pair(k)
    return p.I0.astype("float32"), p.I1.astype("float32")


def _oracle_pair(job):
    from oracle import Params, solve_pair
    I0, I1, kw = job
    t0 = time.perf_counter()
    r = solve_pair(I0.astype("float64"), I1.astype("float64"), Params(**kw))
    return r["u"], r["v"], time.perf_counter() - t0


def _oracle_check(job):
    """Worker: the FP64 oracle on one pair, compared with the GPU flow (u, v) of the same pair.
    Returns the parity figures and the oracle's solve time."""
    import numpy as np
    from oracle import Params, solve_pair
    I0, I1, u, v, kw = job
    t0 = time.perf_counter()
    r = solve_pair(I0.astype("float64"), I1.astype("float64"), Params(**kw))
    dt = time.perf_counter() - t0
    du = np.abs(u.astype("float64") - r["u"])
    dv = np.abs(v.astype("float64") - r["v"])
    d = np.maximum(du, dv)
    epe = np.hypot(du, dv)
    return {"max_abs_px": float(d.max()), "over_1e-4": int((d > 1e-4).sum()), "mean_epe_px": float(epe.mean()),
            "p999_epe_px": float(np.quantile(epe, 0.999)), "max_epe_px": float(epe.max()), "oracle_s": dt}


def batch_sha():
    """Hash of the batched path's tile kernel and of the sources that plan its tiles."""
    h = hashlib.sha256()
    for f in ("admm_tb.hip", "admm_rows.hip", "admm_args.hpp", "tb_plan.cpp", "multi.cpp", "geometry.cpp"):
        with open(os.path.join(ROOT, "paper_2011_10979_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def batch_traffic(signature, iters):
    """DRAM bytes per launch of a batched tile kernel, averaged over its launches in one batched
    solve, from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE record of each of its stages (level,
    order, tile code, K, width), when every such stage was measured on the current kernel and
    planner source (else None).  A stage makes ceil(iters / K) launches per warp."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        e = json.load(open(path)).get("batch64")
    except (OSError, ValueError):
        return None
    if not e or e.get("kernel_sha") != batch_sha() or not isinstance(signature, list):
        return None
    rec = {(m["level"], m["order"], m.get("nt", 1025), m["K"], m["ew"]): m["bytes_per_launch"]
           for m in e.get("stages", [])}
    tot = n = 0
    for level, order, nt, K, ew in signature:
        b = rec.get((level, order, nt, K, ew))
        if b is None:
            return None
        launches = -(-iters // K)
        tot += b * launches
        n += launches
    return round(tot / n) if n else None


def pair_px(H, W, levels):
    tot = 0
    for _ in range(levels):
        tot += H * W
        H, W = (H + 1) // 2, (W + 1) // 2
    return tot


def _gen_map(fn, items, workers):
    """Synthetic inputs in a fork pool of `workers` processes, or in this process when it is 1.
    Under a profiler that sets up the GPU before the program starts, forked workers inherit that
    state, and the profiler's handlers in them can stall when the pool ends them; profiled runs
    therefore pass 1."""
    import multiprocessing as mp
    items = list(items)
    if workers <= 1:
        return [fn(x) for x in items]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(fn, items)


def run_batch(args):
    """The headline configuration: 64 uneven pairs solved together by the batched path, beside 64
    sequential plain solves, a short served trace and the FP64 oracle on every pair."""
    import multiprocessing as mp
    import numpy as np
    import torch
    import synth
    import paper_2011_10979_amd as fm
    n = args.pairs
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    host = _gen_map(_gen_batch_pair, range(n), args.gen_workers)
    print(f"[bench] generated {n} pairs in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    frames = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev),
               synth.levels_by_size(*a.shape)) for a, b in host]
    shapes = [a.shape for a, _ in host]
    params = fm.Params(scheme=args.scheme, storage=args.storage, warps=args.warps, iters=args.iters, use_graph=1)
    pxi_pair = [pair_px(H, W, lv) * args.warps * args.iters for (H, W), (_, _, lv) in zip(shapes, frames)]
    px_iter = sum(pxi_pair)
    ctx = fm.Context(0)
    tuning = None
    if args.load_batch_tuning:
        # stage choices measured by an earlier run (profiler runs: no tuning launches in the trace)
        with open(args.load_batch_tuning) as fh:
            tuning = json.load(fh)
        for st in tuning:
            if args.scheme in ("pdr", "alg1"):                                 # pDR / ALG1: the tile code
                ctx.set_batched_stage(frames, st["level"], st["nt"], st["K"], 64, params)
                continue
            order = st["nt"] if st.get("nt", 1025) != 1025 else st["order"]     # wave-row tiles: their code
            ctx.set_batched_stage(frames, st["level"], order, st["K"], st["ew"], params)
        print(f"[bench] loaded batched stage choices: {tuning}", file=sys.stderr, flush=True)
    elif not args.no_autotune:
        t0 = time.perf_counter()
        tuning = ctx.autotune_batched(frames, params).get("stages")
        print(f"[bench] batched autotune {time.perf_counter() - t0:.1f} s: {tuning}", file=sys.stderr, flush=True)
    if args.save_batch_tuning and tuning:
        with open(args.save_batch_tuning, "w") as fh:
            json.dump(tuning, fh)
    for _ in range(args.warmup):
        out = ctx.solve_batched(frames, params)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        out = ctx.solve_batched(frames, params)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = max(start.elapsed_time(end), wall * 1e3) / args.steps
    value = px_iter / (ms_step * 1e-3) / 1e9
    print(f"[bench] batched: {ms_step:.2f} ms per batch, {value:.2f} Gpx-iter/s", file=sys.stderr, flush=True)
    if args.batch_only:                      # the batched solve alone (for profiler runs)
        print(json.dumps({"metric": "Gpixel-iter/s (batched solves only)", "value": round(value, 3),
                          "unit": "Gpixel-iter/s", "ms_per_step": round(ms_step, 3), "steps": args.steps,
                          "autotuned": not args.no_autotune, "px_iter_per_step": px_iter}), flush=True)
        ctx.close()
        return

    # per-stage timing: direct launches, HIP events on the solve stream around each stage's tile
    # launches
    ctx.set_stats(True)
    p_inst = fm.Params(**{**params.__dict__, "use_graph": 0})
    reps = 2
    nl = max(lv for _, _, lv in frames)
    ms = [0.0] * nl
    launches = [0] * nl
    iters = [0] * nl
    for _ in range(reps):
        ctx.solve_batched(frames, p_inst)
        s = ctx.stats()
        for l in range(nl):
            ms[l] += s["iter_ms"][l]
            launches[l] += s["launches"][l]
            iters[l] += s["iterations"][l]
    level_px = s["level_px"]
    ctx.set_stats(False)
    per_level = [{"level": l, "pixels": level_px[l], "Gpx_iter_s": round(level_px[l] * iters[l] / (ms[l] * 1e-3) / 1e9, 2),
                  "us_per_launch": round(1e3 * ms[l] / max(1, launches[l]), 2), "launches_per_step": launches[l] // reps}
                 for l in range(nl)]
    has_w = params.beta > 0
    pd = args.scheme in ("pdr", "alg1")
    # the dominant kernel: the stages' tile kernel (ADMM: general tiles from the table or from work
    # queues, or wave-row tiles; pDR: general, two-cell or one-cell wave-row tiles) that takes the
    # most time, over the levels that run it
    wt = "true" if has_w else "false"
    by_level = {st["level"]: st for st in tuning} if tuning else {}

    def kname(st):
        nt = st.get("nt", 1025)
        if args.scheme == "pdr":
            if nt in (2050, 3074):
                return f"pdr_rows1_table_kernel<{wt}, 16, {3 if nt == 3074 else 2}>"
            if nt in (4098, 6145):
                return f"pdr_rows_table_kernel<{wt}, 16, {3 if nt == 6145 else 2}>"
            return f"pdr_tb_table_kernel (general tiles, code {nt})"
        if args.scheme == "alg1":
            if nt in (2050, 3074):
                return f"alg1_rows_table_kernel<{wt}, 16, {3 if nt == 3074 else 2}>"
            return f"alg1_tb_table_kernel (general tiles, code {nt})"
        if nt in (2049, 3073, 4097):
            return f"admm_rows_table_kernel<{wt}, 16, {(nt - 1) // 1024}>"
        return f"admm_tb_{'queue' if st['order'] == 1 else 'table'}_kernel<{wt}, 1024, 2>"
    if by_level and all(l in by_level for l in range(nl)):
        groups = {}
        for l in range(nl):
            groups.setdefault(kname(by_level[l]), []).append(l)
        kernel, sel = max(groups.items(), key=lambda kv: sum(ms[l] for l in kv[1]))
    else:
        sel = list(range(nl))
        kernel = {"pdr": "pDR tile kernels", "alg1": "ALG1 tile kernels"}.get(
            args.scheme, "batched ADMM tile kernels") + " (built-in stage choices)"
    tile_ms = sum(ms[l] for l in sel)
    tile_launches = sum(launches[l] for l in sel)
    tile_pxi = sum(level_px[l] * iters[l] for l in sel)                  # over `reps` solves
    tile_px_launch = sum(level_px[l] * launches[l] for l in sel)
    launch_s = tile_ms * 1e-3 / tile_launches
    per_iter = (PDR_TB_BYTES_PER_PX_ITER if pd else BYTES_PER_PX_ITER)[has_w]
    per_launch = (PDR_TB_BYTES_PER_PX_LAUNCH if pd else BYTES_PER_PX_LAUNCH)[has_w]
    alg_launch = per_iter * tile_pxi / tile_launches                     # algorithmic bytes per launch
    achieved = alg_launch / launch_s / 1e9
    if pd:                                                  # the DRAM record covers the ADMM batch only
        signature, traffic = "pDR / ALG1 stages", None
    else:
        signature = ([[l, by_level[l]["order"], by_level[l].get("nt", 1025), by_level[l]["K"], by_level[l]["ew"]]
                      for l in sel] if by_level else "built-in")
        traffic = batch_traffic(signature, args.iters)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_source": ("looked up: profiles/traffic.json (rocprofv3 FETCH_SIZE / WRITE_SIZE runs on this "
                               "kernel source and stage choice, copy-calibrated)") if traffic else None,
            "kernel": f"{kernel} (batched K-iteration tile kernel, levels {sel})",
            "per_unit": f"{per_iter} B per pixel-iteration",
            "px_iter_per_launch": round(tile_pxi / tile_launches), "bytes_per_launch": round(alg_launch),
            "avg_launch_us": round(launch_s * 1e6, 3), "launches_per_step": tile_launches // reps,
            "note": "K iterations per launch share one pass over HBM, so the algorithmic rate can exceed the "
                    "HBM peak; dram_* figures are the measured traffic",
            "one_pass_per_launch": {"per_unit": f"{per_launch} B per pixel per launch",
                                    "GBs": round(per_launch * tile_px_launch / tile_launches / launch_s / 1e9, 1)}}
    roof["one_pass_per_launch"]["frac"] = round(roof["one_pass_per_launch"]["GBs"] / HBM_PEAK_GBS, 4)
    if traffic:
        roof["dram_GBs"] = round(traffic / launch_s / 1e9, 1)
        roof["dram_frac"] = round(roof["dram_GBs"] / HBM_PEAK_GBS, 4)
    print(f"[bench] roofline {roof}", file=sys.stderr, flush=True)

    # 64 sequential plain solves of the same pairs: built-in kernel plan, then tiles at every level
    plain = {}
    big = max(range(n), key=lambda k: pxi_pair[k])
    for label, mode in (("builtin", 0), ("tiles", 4)):
        fm.set_tuning("tb_mode", mode)
        # the largest pair first: the context's arena reaches its final size (growing it drops the
        # captured graphs), then a pass that captures each shape's graph, then the timed pass
        I0, I1, lv = frames[big]
        ctx.solve(I0, I1, fm.Params(**{**params.__dict__, "levels": lv}))
        outs = []
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            outs = [ctx.solve(I0, I1, fm.Params(**{**params.__dict__, "levels": lv}))
                    for I0, I1, lv in frames]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        plain[label] = {"ms": round(dt * 1e3, 3), "pairs_per_s": round(n / dt, 2),
                        "Gpx_iter_s": round(px_iter / dt / 1e9, 3)}
        if mode == 4:
            same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) for a, b in zip(out, outs))
            plain[label]["batched_bitwise_equal"] = bool(same)
    fm.set_tuning("tb_mode", 0)
    print(f"[bench] plain: {plain}", file=sys.stderr, flush=True)

    serving = None
    if not args.no_serve:
        serving = serve_leg(args, ctx, ingest=True, with_plain=False, n_meas=args.batch_serve_requests,
                            n_warm=100, capacity=300)
        serving.pop("_pool")
        print(f"[bench] serving: {serving}", file=sys.stderr, flush=True)
    ctx.close()

    # the FP64 oracle on every pair of the batch (one process per pair on all host cores): parity
    # of every batched flow, and the oracle's own rate on all cores; then on one core
    check = cpu_all = cpu = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits
        os.environ.setdefault("OMP_NUM_THREADS", "1")
        order = sorted(range(n), key=lambda k: -pxi_pair[k])           # largest first: shorter tail
        jobs = [(host[k][0], host[k][1], out[k][0].cpu().numpy(), out[k][1].cpu().numpy(),
                 dict(scheme=args.scheme, levels=frames[k][2], warps=args.warps, iters=args.iters)) for k in order]
        print(f"[bench] oracle on all {n} pairs, {workers} processes ...", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(workers) as pool:
            res = pool.map(_oracle_check, jobs, chunksize=1)
        dt_all = time.perf_counter() - t0
        worst = max(range(n), key=lambda i: res[i]["max_abs_px"])
        check = {"gate": "endpoint error <= 0.01 px against the FP64 oracle at every pixel of every pair",
                 "pairs": n, "max_epe_px": max(r["max_epe_px"] for r in res),
                 "max_mean_epe_px": max(r["mean_epe_px"] for r in res),
                 "max_p999_epe_px": max(r["p999_epe_px"] for r in res),
                 "max_abs_px": max(r["max_abs_px"] for r in res),
                 "worst_pair": [int(order[worst])] + list(shapes[order[worst]]),
                 "pixels_over_1e-4": sum(r["over_1e-4"] for r in res)}
        check["met"] = check["max_epe_px"] <= 1e-2
        cpu_all = {"value": round(px_iter / dt_all / 1e9, 4), "unit": "Gpixel-iter/s", "cores": workers,
                   "kind": "oracle", "pairs_per_s": round(n / dt_all, 3), "host": host_cpu(),
                   "sample": f"all {n} pairs of the batch, one process per pair ({px_iter / 1e9:.2f} G px-iter, "
                             f"{dt_all:.1f} s wall, FP64 NumPy, one BLAS thread each)"}
        small = sorted(range(n), key=lambda k: pxi_pair[k])[:args.cpu_pairs]
        pxi = sum(pxi_pair[k] for k in small)
        print(f"[bench] oracle on {len(small)} pairs, one core ...", file=sys.stderr, flush=True)
        with threadpool_limits(limits=1):
            from oracle import Params, solve_pair
            t0 = time.perf_counter()
            for k in small:
                solve_pair(host[k][0].astype("float64"), host[k][1].astype("float64"),
                           Params(scheme=args.scheme, levels=frames[k][2], warps=args.warps, iters=args.iters))
            dt = time.perf_counter() - t0
        cpu = {"value": round(pxi / dt / 1e9, 4), "unit": "Gpixel-iter/s", "cores": 1, "kind": "oracle",
               "pairs_per_s": round(len(small) / dt, 3), "host": host_cpu(),
               "sample": f"the {len(small)} smallest pairs of the batch in turn ({pxi / 1e6:.0f} M px-iter, "
                         f"{dt:.1f} s, FP64 NumPy, 1 thread)"}
    line = {
        "metric": "Gpixel-iter/s per level; pairs/s + p50/p99 latency at EPE<=0.01px vs oracle",
        "value": round(value, 3), "unit": "Gpixel-iter/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n} synthetic pairs of uneven sizes (128x96 .. 1280x720, seeds 1000+k), pyramid "
                               f"depth by size x {args.warps} warps x {args.iters} iterations, {args.scheme}, "
                               f"solved together by the batched path",
                   "pairs": n, "px_iter_per_step": px_iter, "graph": True, "stage_choices": tuning or "built-in"},
        "pairs_per_s": round(n / (ms_step * 1e-3), 2),
        "plain_sequential": plain,
        "speedup_vs_best_plain": round(min(p_["ms"] for p_ in plain.values()) / ms_step, 3),
        "per_level": per_level, "roofline": roof, "serving": serving, "oracle_check": check,
        "cpu_baseline": cpu, "cpu_baseline_all_cores": cpu_all,
    }
    print(json.dumps(line), flush=True)


def _gen_serving_pair(job):
    import synth
    si, j = job
    H, W = synth.SERVING_SIZES[si]
    p = synth.vga_pair(5000 + 100 * si + j, H, W) if j % 2 == 0 else synth.hd_pair(5000 + 100 * si + j, H, W)
    return p.I0.astype("float32"), p.I1.astype("float32")


def _percentiles(lat):
    import numpy as np
    a = np.asarray(lat) * 1e3
    return {"n": int(a.size), "p50_ms": round(float(np.percentile(a, 50)), 3), "p99_ms": round(float(np.percentile(a, 99)), 3),
            "mean_ms": round(float(a.mean()), 3), "max_ms": round(float(a.max()), 3)}


def serve_leg(args, ctx, ingest=True, with_plain=True, n_meas=None, n_warm=None, capacity=None):
    """A Poisson request trace through the continuous-batching engine (and, with `with_plain`,
    through a one-at-a-time plain-solve server).  With `ingest` each request's frames start in
    pinned host memory and are uploaded on the serving stream when the request arrives, inside its
    latency window; otherwise they are already on the device."""
    import multiprocessing as mp
    import numpy as np
    import torch
    import synth
    import paper_2011_10979_amd as fm
    workers = max(1, min(16, os.cpu_count() or 1))
    per = args.pool
    t0 = time.perf_counter()
    host = _gen_map(_gen_serving_pair, [(si, j) for si in range(len(synth.SERVING_SIZES)) for j in range(per)],
                    args.gen_workers)
    print(f"[bench] generated {len(host)} pool pairs in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    pool_host = [[None] * per for _ in synth.SERVING_SIZES]
    pool_dev = [[None] * per for _ in synth.SERVING_SIZES]
    for si in range(len(synth.SERVING_SIZES)):
        for j in range(per):
            a, b = host[si * per + j]
            pool_host[si][j] = (torch.from_numpy(a).pin_memory(), torch.from_numpy(b).pin_memory())
            if not ingest or with_plain:
                pool_dev[si][j] = (torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
    levels = [synth.levels_by_size(H, W) for H, W in synth.SERVING_SIZES]
    n_warm = args.serve_warmup if n_warm is None else n_warm
    n_meas = args.requests if n_meas is None else n_meas
    t_arr, size_idx = synth.serving_trace(n_warm + n_meas, args.rate, seed=7)
    pick = np.random.default_rng(8).integers(0, per, size=n_warm + n_meas)
    params = fm.Params(scheme=args.scheme, storage=args.storage, warps=args.warps, iters=args.iters)
    px_iter = [pair_px(*synth.SERVING_SIZES[si], levels[si]) * args.warps * args.iters for si in size_idx]
    torch.cuda.synchronize()

    def frames_of(i):
        si, j = size_idx[i], pick[i]
        if not ingest:
            return pool_dev[si][j]
        h0, h1 = pool_host[si][j]
        d0 = torch.empty(h0.shape, dtype=torch.float32, device=dev)
        d1 = torch.empty(h1.shape, dtype=torch.float32, device=dev)
        d0.copy_(h0, non_blocking=True)        # stream-ordered before the engine's import of the pair
        d1.copy_(h1, non_blocking=True)
        return d0, d1

    def replay(label, submit, advance, poll, t_arr=t_arr, n_warm=n_warm, n_meas=n_meas):
        lat = [None] * len(t_arr)
        done_t = [None] * len(t_arr)
        pending = {}
        i = 0
        start = time.perf_counter()
        last_print = start
        while i < len(t_arr) or pending:
            now = time.perf_counter() - start
            while i < len(t_arr) and t_arr[i] <= now:
                pending[submit(i)] = i
                i += 1
            if pending:
                advance()
                now = time.perf_counter() - start
                for t in list(pending):
                    if poll(t):
                        k = pending.pop(t)
                        lat[k] = now - t_arr[k]
                        done_t[k] = now
            elif i < len(t_arr):
                time.sleep(max(0.0, t_arr[i] - now))
            if time.perf_counter() - last_print > 5:
                last_print = time.perf_counter()
                print(f"[bench] {label}: {i} submitted, {len(pending)} pending", file=sys.stderr, flush=True)
        meas = lat[n_warm:]
        t_first = t_arr[n_warm] if n_warm else 0.0
        t_last = max(done_t[n_warm:])
        pxi = sum(px_iter[k % len(px_iter)] for k in range(n_warm, n_warm + n_meas))
        out = {"pairs_per_s": round(float(n_meas / (t_last - t_first)), 2),
               "Gpx_iter_s": round(float(pxi / (t_last - t_first) / 1e9), 3)}
        out.update(_percentiles(meas))
        per_size = {}
        for si, (H, W) in enumerate(synth.SERVING_SIZES):
            sel = [meas[k] for k in range(n_meas) if size_idx[(n_warm + k) % len(size_idx)] == si]
            if sel:
                per_size[f"{W}x{H}"] = _percentiles(sel)
        out["per_size"] = per_size
        return out

    # continuous batching
    srv = fm.Server(ctx, params, budget_bytes=args.budget_gib << 30, max_active=args.max_active)

    def s_submit(i):
        I0, I1 = frames_of(i)
        return srv.submit(I0, I1, levels[size_idx[i]])

    def s_poll(t):
        return srv.poll(t) is not None

    served = replay("engine", s_submit, srv.step, s_poll)
    sst = srv.stats()
    served["engine"] = {k: sst[k] for k in ("epochs", "peak_active", "peak_bytes_in_use", "arena_bytes")}
    # capacity: the first `capacity` requests of the trace all arriving at once
    n_cap = min(args.capacity if capacity is None else capacity, len(t_arr))
    cap_arr = np.zeros(n_cap)
    cap_served = replay("engine capacity", s_submit, srv.step, s_poll, cap_arr, 0, n_cap) if n_cap else None
    srv.close()
    result = {"workload": f"Poisson arrivals {args.rate}/s, {n_meas} requests after {n_warm}, sizes "
                          f"320x240/640x480/1024x436/1280x720/1920x1080 (p .3/.3/.2/.1/.1), pool of {per} pairs per "
                          f"size, pyramid depth by size x {args.warps} warps x {args.iters} iterations, {args.scheme}",
              "frames": "uploaded from pinned host memory inside each request's latency" if ingest
                        else "resident on the device before the trace",
              "budget_GiB": args.budget_gib, "max_active": args.max_active,
              "engine": served, "engine_capacity": {"requests": n_cap, "arriving": "all at once",
                                                    **(cap_served or {})}}
    if with_plain:
        # one at a time: a FIFO of plain solves (graph replay per size, tiles at every level)
        fm.set_tuning("tb_mode", 4)
        gp = fm.Params(**{**params.__dict__, "use_graph": 1})
        for si in range(len(synth.SERVING_SIZES)):                     # capture each size's graph
            ctx.solve(*pool_dev[si][0], fm.Params(**{**gp.__dict__, "levels": levels[si]}))
        queue = []
        finished = set()
        tick = [0]

        def p_submit(i):
            tick[0] += 1
            queue.append((tick[0], frames_of(i), i))
            return tick[0]

        def p_advance():
            if queue:
                t, (I0, I1), i = queue.pop(0)
                ctx.solve(I0, I1, fm.Params(**{**gp.__dict__, "levels": levels[size_idx[i]]}))
                finished.add(t)

        result["plain_one_at_a_time"] = replay("plain", p_submit, p_advance, lambda t: t in finished)
        result["plain_capacity"] = replay("plain capacity", p_submit, p_advance, lambda t: t in finished, cap_arr,
                                          0, n_cap) if n_cap else None
        fm.set_tuning("tb_mode", 0)
    result["_pool"] = (host, pool_dev, levels)
    return result


def run_serve(args):
    """The serving configuration: a Poisson request trace through the continuous-batching engine and
    through a one-at-a-time plain-solve server, with a check of served flows against the oracle."""
    import multiprocessing as mp
    import numpy as np
    import torch
    import paper_2011_10979_amd as fm
    ctx = fm.Context(0)
    res = serve_leg(args, ctx, ingest=not args.no_ingest, with_plain=True)
    host, pool_dev, levels = res.pop("_pool")
    per = args.pool
    check = None
    if not args.no_cpu_baseline:
        # served flows of the smallest size's pool pairs against the FP64 oracle
        seen = list(range(min(per, args.oracle_pairs)))
        dev = torch.device("cuda:0")
        params = fm.Params(scheme=args.scheme, storage=args.storage, warps=args.warps, iters=args.iters)
        srv = fm.Server(ctx, params, budget_bytes=1 << 30, max_active=8)
        tk = {j: srv.submit(torch.from_numpy(host[j][0]).to(dev), torch.from_numpy(host[j][1]).to(dev), levels[0])
              for j in seen}
        srv.drain()
        got = {j: srv.poll(t) for j, t in tk.items()}
        srv.close()
        jobs = [(host[j][0], host[j][1], got[j][0].cpu().numpy(), got[j][1].cpu().numpy(),
                 dict(scheme=args.scheme, levels=levels[0], warps=args.warps, iters=args.iters)) for j in seen]
        os.environ.setdefault("OMP_NUM_THREADS", "1")
        with mp.get_context("fork").Pool(min(16, max(1, len(jobs)))) as pool:
            rs = pool.map(_oracle_check, jobs)
        check = {"size": "320x240", "pairs": len(jobs), "max_abs_px": max(r["max_abs_px"] for r in rs),
                 "pixels_over_1e-4": sum(r["over_1e-4"] for r in rs),
                 "max_mean_epe_px": max(r["mean_epe_px"] for r in rs)}
    line = {
        "metric": "pairs/s with p50 / p99 latency (served coarse-to-fine TV-L1 flow solves, Poisson arrivals)",
        "value": res["engine"]["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": res.pop("workload"), "budget_GiB": args.budget_gib, "max_active": args.max_active,
                   "frames": res.pop("frames")},
        **res, "oracle_check": check,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


COMPARE = [  # (label, scheme, relax, beta): the schemes and parameters of Sec. 4 / Table 1
    ("pADMM", "padmm", 1.0, 0.05), ("rpADMMI r=1.618", "padmm", 1.618, 0.05), ("rpADMMII rho=1.9", "rpadmm2", 1.9, 0.05),
    ("Zach-pADMM (beta=0)", "padmm", 1.0, 0.0), ("pDR", "pdr", 1.0, 0.05), ("ALG1", "alg1", 1.0, 0.05)]


def run_compare(args):
    """Every scheme of Sec. 4 on the same synthetic pair at the same iteration counts: time per solve
    on the GPU (autotuned, graph replay) and the accuracy against the ground-truth motion (mean
    endpoint and angular error), with the final warp's energy and gap."""
    import numpy as np
    import torch
    import synth
    import paper_2011_10979_amd as fm
    if args.pair == "hd":
        pair = synth.hd_pair(seed=2)
        levels = 6
    else:
        pair = synth.vga_pair(seed=1, H=args.H, W=args.W)
        levels = args.levels
    H, W = pair.I0.shape
    dev = torch.device("cuda:0")
    I0 = torch.from_numpy(pair.I0.astype(np.float32)).to(dev)
    I1 = torch.from_numpy(pair.I1.astype(np.float32)).to(dev)
    px = 0
    h, w = H, W
    for _ in range(levels):
        px += h * w
        h, w = (h + 1) // 2, (w + 1) // 2
    rows = []
    for label, scheme, relax, beta in COMPARE:
        ctx = fm.Context(0)
        p = fm.Params(scheme=scheme, relax=relax, beta=beta, levels=levels, warps=args.warps, iters=args.iters,
                      use_graph=1)
        ctx.autotune(H, W, p)
        for _ in range(2):
            u, v, res = ctx.solve(I0, I1, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            u, v, res = ctx.solve(I0, I1, p)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        un, vn = u.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)
        epe = float(np.hypot(un - pair.u, vn - pair.v).mean())
        cosang = (un * pair.u + vn * pair.v + 1.0) / (np.sqrt(un ** 2 + vn ** 2 + 1.0) * np.sqrt(pair.u ** 2 + pair.v ** 2 + 1.0))
        aae = float(np.degrees(np.arccos(np.clip(cosang, -1.0, 1.0))).mean())
        rows.append({"scheme": label, "beta": beta, "ms_per_solve": round(ms, 3),
                     "Gpx_iter_s": round(px * args.warps * args.iters / (ms * 1e-3) / 1e9, 2),
                     "epe_px": round(epe, 4), "aae_deg": round(aae, 3), "energy": res["energy"], "gap": res["gap"]})
        print(f"[bench] {rows[-1]}", file=sys.stderr, flush=True)
        ctx.close()
    ref = next(r for r in rows if r["scheme"] == "pADMM")
    for r in rows:
        r["time_vs_pADMM"] = round(r["ms_per_solve"] / ref["ms_per_solve"], 3)
    line = {"metric": "scheme comparison (time per solve, accuracy against the synthetic ground truth)",
            "config": {"workload": f"{W}x{H} pair ({args.pair}), {levels} levels x {args.warps} warps x {args.iters} "
                                   f"iterations, every scheme of Sec. 4", "data": "synthetic"},
            "rows": rows}
    print(json.dumps(line), flush=True)


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
    ap.add_argument("--no-graph", action="store_true", help="single mode: launch every kernel directly instead "
                    "of replaying the solve's captured graph")
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="set a library tuning knob (flow_tune_set) before the run, e.g. serve_graph=0")
    ap.add_argument("--batch-only", action="store_true",
                    help="batch mode: time the batched solve only (no plain solves, per-stage timing or oracle check)")
    ap.add_argument("--save-tuning", default=None)
    ap.add_argument("--save-batch-tuning", default=None, help="batch mode: write the autotuned stage choices")
    ap.add_argument("--load-batch-tuning", default=None,
                    help="batch mode: apply stage choices from a file instead of tuning (for profiler runs)")
    ap.add_argument("--load-tuning", default=None)
    ap.add_argument("--choice", action="append", default=[], metavar="KEY=MODE,K,ROWS",
                    help="after tuning, pin one level shape's kernel choice, e.g. 480x640i50=4,9,48")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB")
    ap.add_argument("--mode", default="batch", choices=["single", "batch", "serve", "compare"])
    ap.add_argument("--pair", default="vga", choices=["vga", "hd"])
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--pool", type=int, default=10)
    ap.add_argument("--budget-gib", type=int, default=8)
    ap.add_argument("--max-active", type=int, default=64)
    ap.add_argument("--capacity", type=int, default=600, help="requests of the saturation run (0: none)")
    ap.add_argument("--pairs", type=int, default=64)
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="processes that build the synthetic pairs (1: in this process, for profiler runs)")
    ap.add_argument("--oracle-pairs", type=int, default=4)
    ap.add_argument("--cpu-pairs", type=int, default=8, help="batch mode: pairs of the one-core oracle sample")
    ap.add_argument("--no-serve", action="store_true", help="batch mode: skip the served-trace leg")
    ap.add_argument("--batch-serve-requests", type=int, default=1000,
                    help="batch mode: requests of the served-trace leg (after 100 warm-up ones)")
    ap.add_argument("--no-ingest", action="store_true",
                    help="serve mode: frames resident on the device before the trace (no upload per request)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU; pairs would be sharded across GPUs with no "
              "communication, and no multi-GPU figure is produced.", file=sys.stderr)
        sys.exit(2)

    import paper_2011_10979_amd as fm

    for kv in args.tune:
        key, _, val = kv.partition("=")
        fm.set_tuning(key, int(val))
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy, args.steps)
        return
    if args.mode == "batch":
        run_batch(args)
        return
    if args.mode == "serve":
        run_serve(args)
        return
    if args.mode == "compare":
        run_compare(args)
        return
    run_single(args)


def run_single(args):
    """One pair (640x480, or the 1920x1080 pair with --pair hd) solved repeatedly."""
    import numpy as np
    import torch
    import synth
    import paper_2011_10979_amd as fm
    dev = torch.device("cuda:0")
    if args.pair == "hd":
        # the 1920x1080 plain-vs-precision-form workload: rotation plus zoom with occlusions, 6 levels
        pair = synth.hd_pair(seed=2)
        args.H, args.W = pair.I0.shape
        args.levels = 6
    else:
        pair = synth.vga_pair(seed=1, H=args.H, W=args.W)
    I0 = torch.from_numpy(pair.I0.astype(np.float32)).to(dev)
    I1 = torch.from_numpy(pair.I1.astype(np.float32)).to(dev)
    ctx = fm.Context(0)
    params = fm.Params(scheme=args.scheme, storage=args.storage, levels=args.levels, warps=args.warps,
                       iters=args.iters, use_graph=0 if args.no_graph else 1)
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
    for kv in args.choice:
        key, _, val = kv.partition("=")
        mode, K, rows = (int(x) for x in val.split(","))
        ctx.set_choice(key, mode, K, rows)
        tuning = dict(tuning or {}, **{key: {"mode": mode, "K": K, "rows": rows}})
        print(f"[bench] pinned {key}: mode {mode}, K {K}, rows {rows}", file=sys.stderr, flush=True)
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
    lvl_launch = [0] * args.levels
    reps = 3
    for _ in range(reps):
        ctx.solve(I0, I1, p_inst, u=u, v=v)
        s = ctx.stats()
        for l in range(args.levels):
            lvl_ms[l] += s["iter_ms"][l]
            lvl_iters[l] += s["iterations"][l]
            lvl_launch[l] += s["launches"][l]
    ctx.set_stats(False)
    per_level = []
    for l, (a, b) in enumerate(shapes):
        gpx = a * b * lvl_iters[l] / (lvl_ms[l] * 1e-3) / 1e9 if lvl_ms[l] > 0 else None
        per_level.append({"level": l, "H": a, "W": b, "Gpx_iter_s": gpx,
                          "us_per_iter": 1e3 * lvl_ms[l] / max(1, lvl_iters[l])})

    has_w = params.beta > 0
    roof = None
    if args.scheme in ("padmm", "rpadmm2"):
        roof = roofline(lvl_ms[0], lvl_launch[0], lvl_iters[0], shapes[0][0] * shapes[0][1], has_w,
                        f"ADMM iteration kernel, level 0 ({shapes[0][1]}x{shapes[0][0]}), choice "
                        f"{(tuning or {}).get(f'{shapes[0][0]}x{shapes[0][1]}i{args.iters}')}",
                        measured_traffic(f"{args.W}x{args.H}",
                                         (tuning or {}).get(f"{shapes[0][0]}x{shapes[0][1]}i{args.iters}")), reps)
        roof["iteration_launches_per_step"] = sum(lvl_launch) // reps
    elif args.scheme in ("pdr", "alg1"):
        suffix = "a" if args.scheme == "alg1" else f"p{params.gs_sweeps}"
        key0 = f"{shapes[0][0]}x{shapes[0][1]}{'w' if has_w else ''}i{args.iters}{suffix}"
        ch0 = (tuning or {}).get(key0, {"mode": 5})
        if ch0["mode"] != 1:
            # K-iteration pDR / ALG1 tiles (every mode but the three-pass iteration's): per launch
            # the kernel reads X, X bar, y and the linearisation once and writes X, X bar, y and
            # Theta once
            name = "ALG1" if args.scheme == "alg1" else "pDR"
            roof = roofline(lvl_ms[0], lvl_launch[0], lvl_iters[0], shapes[0][0] * shapes[0][1], has_w,
                            f"{name} tile kernel, level 0 ({shapes[0][1]}x{shapes[0][0]}), choice {ch0}",
                            None, reps, per_iter=PDR_TB_BYTES_PER_PX_ITER[has_w],
                            per_launch=PDR_TB_BYTES_PER_PX_LAUNCH[has_w])
        else:
            # three-pass pDR: the unit is one iteration (2n + 1 passes over the level)
            roof = roofline(lvl_ms[0], lvl_iters[0], lvl_iters[0], shapes[0][0] * shapes[0][1], has_w,
                            f"pDR iteration, level 0 ({shapes[0][1]}x{shapes[0][0]}): {2 * params.gs_sweeps + 1} passes",
                            None, reps, per_iter=PDR_TB_BYTES_PER_PX_ITER[has_w],
                            per_launch=pdr_bytes_per_px_iter(has_w, params.gs_sweeps))
        roof["iteration_launches_per_step"] = sum(lvl_launch) // reps

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
        "config": {"workload": f"{args.W}x{args.H} pair{' (rotation + zoom, occluding rectangles)' if args.pair == 'hd' else ''}, "
                               f"{args.levels}-level pyramid x {args.warps} warps x {args.iters} iterations, {args.scheme}",
                   "H": args.H, "W": args.W, "levels": args.levels, "warps": args.warps, "iters": args.iters,
                   "scheme": args.scheme, "storage": args.storage, "px_iter_per_step": px_iter,
                   "graph": not args.no_graph, "autotuned": tuning},
        "energy": res["energy"], "gap": res["gap"],
        "per_level": per_level,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
