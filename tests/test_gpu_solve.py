"""End-to-end parity of flow_solve against the FP64 oracle, plus graph replay, precision forms
and error paths.

Bar: max |du|, |dv| <= 1e-4 px for FP32 storage at a fixed iteration count (same inputs rounded to
FP32 on both sides); FP16-stored pyramids: mean endpoint-error difference <= 1e-2 px.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2011_10979_amd as fm  # noqa: E402
import synth  # noqa: E402
from oracle import Params as OParams, solve_pair  # noqa: E402
from helpers import to_dev, to_np, f32, oracle_refs, assert_parity, TOL_F32  # noqa: E402



@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fm.Context(0)
    yield c
    c.close()


def run_both(ctx, pair, pad=0, **kw):
    I0, I1 = f32(pair.I0), f32(pair.I1)
    oscheme = kw.get("scheme", "padmm")
    op = OParams(**{k: v for k, v in kw.items() if k in OParams.__dataclass_fields__})
    ref = solve_pair(I0, I1, op)
    u, v, res = ctx.solve(to_dev(I0, pad), to_dev(I1, pad), fm.Params(**kw))
    del oscheme
    return to_np(u), to_np(v), res, ref


def parity_check(ctx, pair, name, pad=0, full_size=False, **kw):
    """GPU solve against the FP64 oracle (run alongside in a second process) under the FP32 bar of
    helpers.assert_parity (every pixel within 1e-4 px -- or, for a pixel above it, within F_PROBE x
    the oracle's own departure under FP32 rounding of its state --, energy and gap); full-size
    workloads also bound the mean difference by 1e-5 px."""
    import multiprocessing as mp
    I0, I1 = f32(pair.I0), f32(pair.I1)
    okw = {k: v for k, v in kw.items() if k in OParams.__dataclass_fields__}
    with mp.get_context("fork").Pool(1) as pool:
        get = oracle_refs([(I0, I1, okw)], pool)
        u, v, res = ctx.solve(to_dev(I0, pad), to_dev(I1, pad), fm.Params(**kw))
        u, v = to_np(u), to_np(v)
        ref = get(900)[0]
    assert_parity(name, u, v, res, ref, mean_tol=1e-5 if full_size else None, job=(I0, I1, okw))
    return u, v, ref["u"], ref["v"]


def report(name, du, dv):
    d = np.maximum(np.abs(du), np.abs(dv))
    print(f"[parity] {name}: max {d.max():.3e} p99.9 {np.quantile(d, 0.999):.3e} mean {d.mean():.3e}", flush=True)
    return d


@pytest.mark.parametrize("scheme,relax,beta", [("padmm", 1.0, 0.0), ("padmm", 1.618, 0.0), ("rpadmm2", 1.9, 0.0),
                                               ("padmm", 1.0, 0.05), ("pdr", 1.0, 0.0), ("pdr", 1.0, 0.05),
                                               ("alg1", 1.0, 0.0), ("alg1", 1.0, 0.05)])
def test_translation_single_scale(ctx, scheme, relax, beta):
    """64x64 translation pair, one level, one warp, 200 iterations (the single-scale workload)."""
    print(f"[case] translation {scheme} {relax} {beta}", flush=True)
    pair = synth.translation_pair(0)
    u, v, res, ref = run_both(ctx, pair, pad=3, scheme=scheme, relax=relax, beta=beta, levels=1, warps=1, iters=200)
    d = report(f"translation {scheme}", u - ref["u"], v - ref["v"])
    assert d.max() <= TOL_F32
    assert abs(res["energy"] - ref["energy"]) <= 1e-5 * ref["energy"]
    assert abs(res["gap"] - ref["gap"]) <= 1e-5 * ref["energy"] + 1e-3
    # sanity on the motion itself (pDR moves more slowly per iteration than the ADMM family)
    slack = 0.06 if scheme in ("pdr", "alg1") else 0.03
    assert abs(u.mean() - 0.3) < slack and abs(v.mean() + 0.2) < slack


@pytest.mark.parametrize("scheme,relax,beta", [("padmm", 1.0, 0.0), ("rpadmm2", 1.9, 0.05), ("pdr", 1.0, 0.0),
                                               ("pdr", 1.0, 0.05), ("alg1", 1.0, 0.0), ("alg1", 1.0, 0.05)])
def test_multilevel_small(ctx, scheme, relax, beta):
    print(f"[case] multilevel 96x128 {scheme} {beta}", flush=True)
    pair = synth.vga_pair(seed=5, H=96, W=128)
    parity_check(ctx, pair, f"multilevel 96x128 {scheme} {beta}", scheme=scheme, relax=relax, beta=beta,
                      levels=3, warps=3, iters=40)


def test_odd_sizes_and_degenerate_levels(ctx):
    """Odd sides whose pyramid ends at a 2-pixel side; pitch padding on the inputs."""
    print("[case] odd 35x9", flush=True)
    pair = synth.vga_pair(seed=9, H=35, W=9)
    parity_check(ctx, pair, "odd 35x9", pad=5, levels=3, warps=2, iters=30)


@pytest.mark.parametrize("H,W,levels,iters,scheme", [(2, 2, 1, 10, "padmm"), (2, 37, 1, 10, "pdr"),
                                                      (29, 2, 1, 10, "alg1"), (5, 3, 2, 7, "rpadmm2"),
                                                      (20, 24, 2, 0, "padmm"), (2, 2, 1, 6, "pdr")])
def test_smallest_images_and_zero_iterations(ctx, H, W, levels, iters, scheme):
    """The degenerate cases of the method: 2-pixel sides (every pixel on the image border, where
    the forward differences vanish), a 3 x 2 coarse level, and zero iterations (the flow stays at
    its zero start; energy and gap are those of the zero flow)."""
    print(f"[case] smallest {H}x{W} levels {levels} iters {iters} {scheme}", flush=True)
    rng = np.random.default_rng(H * 1000 + W * 10 + iters)
    I0 = rng.uniform(0.0, 1.0, (H, W))
    pair = type("Pair", (), {})()
    pair.I0, pair.I1 = I0, np.clip(I0 + rng.normal(0.0, 0.05, (H, W)), 0.0, 1.0)
    relax = 1.9 if scheme == "rpadmm2" else 1.0
    u, v, _, _ = parity_check(ctx, pair, f"smallest {H}x{W}", scheme=scheme, relax=relax, levels=levels,
                                   warps=2, iters=iters, use_graph=0)
    if iters == 0:
        assert not u.any() and not v.any()


def test_single_row_or_column_is_rejected(ctx):
    for shape in ((1, 16), (16, 1)):
        I = torch.zeros(shape, dtype=torch.float32, device="cuda")
        with pytest.raises(fm.FlowError) as e:
            ctx.solve(I, I.clone(), fm.Params(levels=1, warps=1, iters=1))
        assert e.value.status == fm.FLOW_E_INVAL


@pytest.mark.parametrize("plan", ["builtin", "autotuned"])
def test_vga_bench_workload_full_size(ctx, plan):
    """The 640x480 workload (5 levels x 5 warps x 50, pADMM, graph replay) against the full FP64
    oracle solve, with the built-in kernel plan and with the plan the benchmark times (the
    autotuner's per-level choice, K-iteration tiles); also mean <= 1e-5 px."""
    print(f"[case] vga 640x480 5x5x50 plan {plan}", flush=True)
    pair = synth.vga_pair(seed=1)
    kw = dict(levels=5, warps=5, iters=50)
    c = ctx
    if plan == "autotuned":
        c = fm.Context(0)
        rep = c.autotune(480, 640, fm.Params(**kw))
        print(f"[parity] vga autotuned plan: { {k: e['choice'] for k, e in rep.items()} }", flush=True)
    try:
        u, v, ru, rv = parity_check(c, pair, f"vga 640x480 {plan}", full_size=True, **kw)
    finally:
        if c is not ctx:
            c.close()
    epe_gpu = np.hypot(u - pair.u, v - pair.v).mean()
    epe_ora = np.hypot(ru - pair.u, rv - pair.v).mean()
    print(f"[parity] vga {plan} EPE vs truth gpu {epe_gpu:.4f} oracle {epe_ora:.4f}", flush=True)


@pytest.mark.parametrize("scheme", ["pdr", "alg1"])
def test_vga_pd_schemes_autotuned_full_size(scheme):
    """pDR (one symmetric sweep) and ALG1 on the 640x480 workload (5 levels x 5 warps x 50, beta = 0)
    with the plan their benchmark times (the autotuner's per-level choice: wave-row tiles on the
    large levels) against the full FP64 oracle solve; also mean <= 1e-5 px."""
    print(f"[case] vga 640x480 5x5x50 {scheme} autotuned", flush=True)
    pair = synth.vga_pair(seed=1)
    kw = dict(scheme=scheme, levels=5, warps=5, iters=50)
    c = fm.Context(0)
    try:
        rep = c.autotune(480, 640, fm.Params(**kw))
        print(f"[parity] vga {scheme} autotuned plan: { {k: e['choice'] for k, e in rep.items()} }", flush=True)
        parity_check(c, pair, f"vga 640x480 {scheme} autotuned", full_size=True, **kw)
    finally:
        c.close()


def test_graph_replay_equals_direct_launches(ctx):
    pair = synth.vga_pair(seed=3, H=120, W=160)
    I0, I1 = to_dev(pair.I0), to_dev(pair.I1)
    outs = []
    for g in (0, 1, 1):
        u, v, r = ctx.solve(I0, I1, fm.Params(levels=3, warps=2, iters=20, use_graph=g))
        outs.append((to_np(u), to_np(v), r["energy"]))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1]) and o[2] == outs[0][2]


def test_fp16_storage_within_bound(ctx):
    """FP16-stored image and derivative pyramids, FP32 arithmetic: against the oracle's FP16 storage
    form (the same binary16 pyramid planes, FP64 solve) the FP32 bar; against the FP32 form a mean
    endpoint-error difference <= 1e-2 px (the contract), p99.9 and max reported."""
    import multiprocessing as mp
    print("[case] fp16 storage 240x320", flush=True)
    pair = synth.vga_pair(seed=4, H=240, W=320)
    I0, I1 = f32(pair.I0), f32(pair.I1)
    kw = dict(levels=4, warps=3, iters=40)
    with mp.get_context("fork").Pool(2) as pool:
        get = oracle_refs([(I0, I1, kw), (I0, I1, dict(kw, storage="f16"))], pool)
        u, v, res = ctx.solve(to_dev(I0), to_dev(I1), fm.Params(**kw, storage="f16"))
        u, v = to_np(u), to_np(v)
        r32, r16 = get(900)
    assert_parity("fp16 240x320 vs the oracle's fp16 form", u, v, res, r16, job=(I0, I1, dict(kw, storage="f16")))
    epe = np.hypot(u - r32["u"], v - r32["v"])
    print(f"[parity] fp16 EPE vs the FP32 form mean {epe.mean():.3e} p99.9 {np.quantile(epe, 0.999):.3e} "
          f"max {epe.max():.3e}", flush=True)
    assert epe.mean() <= 1e-2


def test_stopping_tolerance_stops_early(ctx):
    pair = synth.translation_pair(0)
    I0, I1 = to_dev(pair.I0), to_dev(pair.I1)
    ctx.set_stats(True)
    _, _, r_fixed = ctx.solve(I0, I1, fm.Params(levels=1, warps=1, iters=2000, use_graph=0))
    n_fixed = ctx.stats()["iterations"][0]
    _, _, r_tol = ctx.solve(I0, I1, fm.Params(levels=1, warps=1, iters=2000, tol=2e-3, check_every=50))
    n_tol = ctx.stats()["iterations"][0]
    ctx.set_stats(False)
    assert n_fixed == 2000 and n_tol < 2000
    assert abs(r_tol["gap"]) <= 2e-3 * r_tol["energy"]


def test_error_paths(ctx):
    pair = synth.translation_pair(0)
    I0, I1 = to_dev(pair.I0), to_dev(pair.I1)
    with pytest.raises(fm.FlowError) as e:
        ctx.solve(I0, I1, fm.Params(levels=7))      # 64 -> 1 px at the 7th level
    assert e.value.status == fm.FLOW_E_INVAL
    with pytest.raises(fm.FlowError) as e:
        ctx.solve(I0, I1, fm.Params(scheme="rpadmm2", relax=2.5))
    assert e.value.status == fm.FLOW_E_INVAL
    small = fm.Context(0, hbm_budget_bytes=1 << 16)
    with pytest.raises(fm.FlowError) as e:
        small.solve(I0, I1, fm.Params(levels=1, warps=1, iters=1))
    assert e.value.status == fm.FLOW_E_NOMEM
    small.close()
    bad = I0.clone()
    bad[3, 4] = float("nan")
    with pytest.raises(fm.FlowError) as e:
        ctx.solve(bad, I1, fm.Params(levels=1, warps=1, iters=5, use_graph=0))
    assert e.value.status == fm.FLOW_E_NONFINITE


def test_autotuned_solve_keeps_parity():
    """The autotuner only changes which kernel runs each level (speed); the tuned solve still meets
    the oracle bar, and the report names one choice per level shape."""
    print("[case] autotuned multilevel", flush=True)
    c = fm.Context(0)
    try:
        rep = c.autotune(96, 128, fm.Params(levels=3, warps=3, iters=40))
        assert len(rep) == 3
        for key, entry in rep.items():
            assert entry["choice"]["mode"] in (1, 2, 3, 4, 6, 7, 8, 9) and entry["choice"]["us_per_iter"] > 0
            assert len(entry["candidates"]) >= 4
        pair = synth.vga_pair(seed=5, H=96, W=128)
        parity_check(c, pair, "autotuned 96x128", levels=3, warps=3, iters=40)
    finally:
        c.close()


@pytest.mark.parametrize("mode,k,ew", [(4, 4, 32), (4, 8, 48), (7, 4, 96), (6, 2, 16), (2, 4, 64), (8, 8, 24),
                                       (9, 4, 40)])
def test_tuned_tile_widths_keep_parity(mode, k, ew):
    """A tuned choice may also set the width of the tiles' extended region (tuning field `rows` of
    the tile modes); any width gives the same iteration, so the solve still meets the oracle bar."""
    print(f"[case] tile width mode {mode} K {k} ew {ew}", flush=True)
    c = fm.Context(0)
    try:
        for key in ("96x128i40", "48x64i40", "24x32i40"):
            c.set_choice(key, mode, k, ew)
        pair = synth.vga_pair(seed=5, H=96, W=128)
        parity_check(c, pair, f"tile width {mode}/{k}/{ew}", levels=3, warps=3, iters=40)
    finally:
        c.close()


def test_tuning_choice_rows_are_checked(ctx):
    with pytest.raises(fm.FlowError):
        ctx.set_choice("96x128i40", 1, 0, 16)      # one-pass strip height: 0, 2, 4 or 8
    with pytest.raises(fm.FlowError):
        ctx.set_choice("96x128i40", 4, 4, 8)       # tile width: 0 or 16..512


@pytest.mark.parametrize("mode,k", [(1, 0), (2, 2), (3, 4), (4, 8), (7, 4), (6, 2), (8, 4), (9, 2), (12, 6), (13, 5),
                                    (14, 10)])
def test_every_kernel_mode_keeps_parity(ctx, mode, k):
    """Each forced kernel choice (one-pass; tiles of 256 / 1024 / small 1024 threads; wave-row tiles)
    meets the bar."""
    print(f"[case] forced mode {mode} K {k}", flush=True)
    fm.set_tuning("tb_mode", mode)
    fm.set_tuning("tb_k", k)
    try:
        pair = synth.vga_pair(seed=6, H=120, W=150)
        parity_check(ctx, pair, f"mode {mode} K {k}", levels=3, warps=2, iters=30)
    finally:
        fm.set_tuning("tb_mode", 0)
        fm.set_tuning("tb_k", 0)


@pytest.mark.parametrize("mode,k,beta", [(1, 0, 0.0), (5, 1, 0.0), (5, 2, 0.0), (5, 3, 0.05), (5, 2, 0.05),
                                         (6, 1, 0.0), (6, 2, 0.05), (10, 1, 0.0), (10, 2, 0.0), (10, 3, 0.0),
                                         (10, 2, 0.05), (11, 2, 0.0), (11, 4, 0.0), (11, 2, 0.05), (12, 2, 0.0),
                                         (12, 1, 0.05), (13, 2, 0.0), (13, 3, 0.0), (13, 2, 0.05), (14, 2, 0.0),
                                         (14, 3, 0.0), (14, 2, 0.05), (15, 1, 0.0), (15, 2, 0.05)])
def test_every_pdr_kernel_mode_keeps_parity(ctx, mode, k, beta):
    """pDR with the three-pass iteration and with K-iteration tiles of 1024 and 512 threads, one or
    two cells of each colour per thread (K = 1 .. 4; the coarsest levels resident; two cells per
    colour with beta > 0 fall back to one) meets the bar."""
    print(f"[case] forced pDR mode {mode} K {k} beta {beta}", flush=True)
    fm.set_tuning("pdr_mode", mode)
    fm.set_tuning("pdr_k", k)
    try:
        pair = synth.vga_pair(seed=6, H=120, W=150)
        parity_check(ctx, pair, f"pdr mode {mode} K {k}", scheme="pdr", beta=beta, levels=3, warps=2, iters=30)
    finally:
        fm.set_tuning("pdr_mode", 0)
        fm.set_tuning("pdr_k", 0)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_pdr_tile_shapes_give_bitwise_the_same_solve(ctx, k):
    """Every pDR tile shape (1024 or 512 threads, one or two cells of each colour per thread, wave-row
    tiles of 128 x 32, 128 x 48, 64 x 48 and 64 x 32 cells) forms
    each cell's update with the same expressions on the same operands, and tiling never changes
    them: with the same K per launch the solves agree bit for bit."""
    print(f"[case] pDR tile shapes K {k}", flush=True)
    pair = synth.vga_pair(seed=7, H=150, W=190)
    I0, I1 = to_dev(f32(pair.I0)), to_dev(f32(pair.I1))
    out = {}
    try:
        for mode in (5, 6, 10, 11, 12, 13, 14, 15):
            fm.set_tuning("pdr_mode", mode)
            fm.set_tuning("pdr_k", k)
            out[mode] = ctx.solve(I0, I1, fm.Params(scheme="pdr", levels=3, warps=2, iters=20))
    finally:
        fm.set_tuning("pdr_mode", 0)
        fm.set_tuning("pdr_k", 0)
    for mode in (6, 10, 11, 12, 13, 14, 15):
        assert torch.equal(out[mode][0], out[5][0]) and torch.equal(out[mode][1], out[5][1]), mode
        assert out[mode][2]["energy"] == out[5][2]["energy"], mode


@pytest.mark.parametrize("k,beta", [(2, 0.0), (5, 0.0), (3, 0.05)])
def test_alg1_tile_shapes_give_bitwise_the_same_solve(k, beta):
    """Every ALG1 tile shape (1024 or 512 threads, wave-row tiles of 64 x 48 and 64 x 32 cells) forms
    each cell's update with the same expressions on the same operands: with the same K per launch
    the solves agree bit for bit."""
    print(f"[case] ALG1 tile shapes K {k} beta {beta}", flush=True)
    pair = synth.vga_pair(seed=8, H=150, W=190)
    I0, I1 = to_dev(f32(pair.I0)), to_dev(f32(pair.I1))
    modes = (5, 6, 14, 15) if beta == 0 else (5, 6, 15)
    out = {}
    for mode in modes:
        c = fm.Context(0)
        try:
            for H, W in [(150, 190), (75, 95), (38, 48)]:
                c.set_choice(f"{H}x{W}{'w' if beta > 0 else ''}i20a", mode, k)
            out[mode] = c.solve(I0, I1, fm.Params(scheme="alg1", beta=beta, levels=3, warps=2, iters=20))
        finally:
            c.close()
    for mode in modes[1:]:
        assert torch.equal(out[mode][0], out[5][0]) and torch.equal(out[mode][1], out[5][1]), mode
        assert out[mode][2]["energy"] == out[5][2]["energy"], mode


@pytest.mark.parametrize("mode,k,beta", [(5, 1, 0.0), (5, 4, 0.0), (6, 2, 0.05), (6, 8, 0.0), (14, 3, 0.0),
                                         (14, 10, 0.0), (15, 4, 0.05), (15, 10, 0.0)])
def test_every_alg1_kernel_mode_keeps_parity(ctx, mode, k, beta):
    """ALG1 with tiles of 1024 and 512 threads and wave-row tiles of 64 x 48 / 64 x 32 cells, several K
    (coarse levels resident), meets the bar."""
    print(f"[case] forced ALG1 mode {mode} K {k} beta {beta}", flush=True)
    c = fm.Context(0)
    try:
        pair = synth.vga_pair(seed=6, H=120, W=150)
        p = fm.Params(scheme="alg1", beta=beta, levels=3, warps=2, iters=30)
        shapes = [(120, 150), (60, 75), (30, 38)]
        for H, W in shapes:
            c.set_choice(f"{H}x{W}{'w' if beta > 0 else ''}i30a", mode, k)
        parity_check(c, pair, f"alg1 mode {mode} K {k}", scheme="alg1", beta=beta, levels=3, warps=2, iters=30)
    finally:
        c.close()
