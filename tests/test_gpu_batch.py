"""Batched solves: many pairs of uneven sizes advanced together, one launch per pipeline step over
all pairs (tile table in XCD order or per-XCD work queues).

Checks: parity of every batched pair with the FP64 oracle (same per-pixel bar as plain solves);
a pair's results are bitwise the same alone, in a mix, under every stage choice (order, K, tile
width, autotuned), and equal to a plain solve that uses the same tile kernel at every level;
graph replays pick up new frames; invalid pairs are rejected before anything runs.
"""
import multiprocessing as mp

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2011_10979_amd as fm  # noqa: E402
import synth  # noqa: E402
from helpers import to_dev, to_np, f32, oracle_refs, assert_parity  # noqa: E402

KW = dict(levels=3, warps=2, iters=30)
# (H, W, seed, levels): uneven sides, ragged tiles, a pair with fewer levels, a tiny one
MIX = [(70, 90, 31, 0), (45, 130, 32, 0), (33, 35, 33, 2), (96, 128, 34, 0), (20, 300, 35, 2)]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fm.Context(0)
    yield c
    c.close()


@pytest.fixture(autouse=True)
def reset_knobs():
    yield
    for k, v in (("tb_mode", 0), ("tb_k", 0), ("batch_order", -1), ("batch_k", 0), ("batch_ew", 0), ("batch_nt", 0)):
        fm.set_tuning(k, v)


def frames(spec, pad=0):
    out = []
    for H, W, seed, lv in spec:
        p = synth.vga_pair(seed=seed, H=H, W=W)
        out.append((f32(p.I0), f32(p.I1), lv, to_dev(f32(p.I0), pad), to_dev(f32(p.I1), pad)))
    return out


def batched(ctx, fr, **kw):
    return ctx.solve_batched([(d0, d1, lv) for _, _, lv, d0, d1 in fr], fm.Params(**kw))


def same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a[:2], b[:2])) and a[2]["energy"] == b[2]["energy"] \
        and a[2]["gap"] == b[2]["gap"]


@pytest.mark.parametrize("scheme,relax,beta", [("padmm", 1.0, 0.0), ("rpadmm2", 1.9, 0.05)])
def test_batched_pairs_match_the_oracle(ctx, scheme, relax, beta):
    print(f"[case] batched parity {scheme} {beta}", flush=True)
    fr = frames(MIX[:4], pad=3)
    kw = dict(KW, scheme=scheme, relax=relax, beta=beta)
    okw = dict(KW, scheme=scheme, relax=relax, beta=beta)
    jobs = []
    for I0, I1, lv, _, _ in fr:
        jobs.append((I0, I1, dict(okw, levels=lv or KW["levels"])))
    with mp.get_context("fork").Pool(4) as pool:
        fut = oracle_refs(jobs, pool)
        out = batched(ctx, fr, **kw)
        refs = fut(900)
    for k, (u, v, res) in enumerate(out):
        assert_parity(f"batched pair {k} {MIX[k][:2]}", to_np(u), to_np(v), res, refs[k])


def test_batched_equals_plain_tile_solves_bitwise(ctx):
    print("[case] batched vs plain mode-4 solves", flush=True)
    fr = frames(MIX, pad=2)
    out = batched(ctx, fr, **KW)
    fm.set_tuning("tb_mode", 4)        # plain solves on small 1024-thread tiles at every level
    for k, (I0, I1, lv, d0, d1) in enumerate(fr):
        u, v, res = ctx.solve(d0, d1, fm.Params(**dict(KW, levels=lv or KW["levels"])))
        assert same(out[k], (u, v, res)), f"pair {k}"


@pytest.mark.parametrize("order,K,ew,nt", [(0, 0, 0, 0), (1, 0, 0, 0), (0, 2, 0, 0), (1, 8, 128, 0), (0, 5, 96, 0),
                                           (1, 3, 64, 0), (0, 8, 64, 3073), (0, 4, 0, 2049), (0, 10, 48, 4097)])
def test_pair_alone_equals_pair_in_mix_under_every_choice(ctx, order, K, ew, nt):
    print(f"[case] alone vs mix order={order} K={K} ew={ew} nt={nt}", flush=True)
    fr = frames(MIX)
    alone = batched(ctx, [fr[3]], **KW)[0]
    fm.set_tuning("batch_order", order)
    fm.set_tuning("batch_k", K)
    fm.set_tuning("batch_ew", ew)
    fm.set_tuning("batch_nt", nt)
    mix = batched(ctx, [fr[1], fr[3], fr[0], fr[4]], **KW)
    assert same(alone, mix[1])
    mix2 = batched(ctx, fr, **KW)
    assert same(mix[0], mix2[1]) and same(mix[2], mix2[0]) and same(mix[3], mix2[4])


def test_autotuned_batch_keeps_results(ctx):
    print("[case] batched autotune", flush=True)
    fr = frames(MIX)
    before = batched(ctx, fr, **KW)
    ctx.autotune_batched([(d0, d1, lv) for _, _, lv, d0, d1 in fr], fm.Params(**KW))
    after = batched(ctx, fr, **KW)
    for a, b in zip(before, after):
        assert same(a, b)


def test_pinned_stage_choices_keep_results(ctx):
    """Stage choices set by hand (the entries an autotune report lists) change speed only: the
    batch's results stay bitwise the same, with the general tiles from the table or from work
    queues and with the wave-row tiles; a level no pair has, an order that is neither 0 / 1 nor a
    wave-row code, or a wave-row width above 64 is refused."""
    print("[case] batched pinned stage choices", flush=True)
    fr = frames(MIX)
    pairs = [(d0, d1, lv) for _, _, lv, d0, d1 in fr]
    before = batched(ctx, fr, **KW)
    for pins in (((0, 1, 3, 48), (1, 0, 7, 96), (2, 0, 30, 64)),
                 ((0, 3073, 8, 64), (1, 2049, 5, 64), (2, 4097, 10, 48))):
        for level, order, K, ew in pins:
            ctx.set_batched_stage(pairs, level, order, K, ew, fm.Params(**KW))
        after = batched(ctx, fr, **KW)
        for a, b in zip(before, after):
            assert same(a, b)
    with pytest.raises(fm.FlowError):
        ctx.set_batched_stage(pairs, 7, 0, 4, 64, fm.Params(**KW))
    with pytest.raises(fm.FlowError):
        ctx.set_batched_stage(pairs, 0, 2, 4, 64, fm.Params(**KW))
    with pytest.raises(fm.FlowError):
        ctx.set_batched_stage(pairs, 0, 3073, 4, 96, fm.Params(**KW))


def test_graph_replay_reads_new_frames(ctx):
    print("[case] batched graph replay", flush=True)
    fa = frames(MIX[:3])
    fb = frames([(H, W, seed + 100, lv) for H, W, seed, lv in MIX[:3]])
    g = dict(KW, use_graph=1)
    batched(ctx, fa, **g)
    rep = [batched(ctx, fb, **g) for _ in range(3)]        # replays with other frames
    direct = batched(ctx, fb, **dict(KW, use_graph=0))
    for r in rep:
        for x, y in zip(r, direct):
            assert same(x, y)


def test_f16_storage_batch_matches_plain(ctx):
    print("[case] batched f16", flush=True)
    fr = frames(MIX[:3])
    out = batched(ctx, fr, **KW, storage="f16")
    fm.set_tuning("tb_mode", 4)
    for k, (I0, I1, lv, d0, d1) in enumerate(fr):
        u, v, res = ctx.solve(d0, d1, fm.Params(**dict(KW, levels=lv or KW["levels"], storage="f16")))
        assert same(out[k], (u, v, res)), f"pair {k}"


@pytest.mark.parametrize("scheme,beta,storage", [("pdr", 0.0, "f32"), ("pdr", 0.05, "f32"), ("alg1", 0.0, "f32"),
                                                 ("alg1", 0.05, "f32"), ("pdr", 0.0, "f16")])
def test_pd_batch_equals_plain_tile_solves(ctx, scheme, beta, storage):
    """Batched pDR and ALG1: stages of table-order tile launches over all pairs; every pair is
    bitwise its plain tile solve (every tile shape and K computes a cell the same way), alone and in
    a mix, direct and replayed from a graph."""
    print(f"[case] batched {scheme} beta {beta} {storage}", flush=True)
    fr = frames(MIX)
    kw = dict(KW, scheme=scheme, beta=beta, storage=storage)
    out = batched(ctx, fr, **kw)
    rep = batched(ctx, fr, **dict(kw, use_graph=1))
    for k, (I0, I1, lv, d0, d1) in enumerate(fr):
        u, v, res = ctx.solve(d0, d1, fm.Params(**dict(kw, levels=lv or KW["levels"])))
        assert same(out[k], (u, v, res)), f"pair {k}"
        assert same(rep[k], (u, v, res)), f"pair {k} (graph)"
    alone = batched(ctx, fr[3:4], **kw)
    assert same(alone[0], out[3])
    # stage choices measured by the batched autotuner (work-group shape and K per stage) change
    # speed only
    rep = ctx.autotune_batched([(d0, d1, lv) for _, _, lv, d0, d1 in fr], fm.Params(**kw))
    assert len(rep["stages"]) == 3 and all(st["K"] >= 1 for st in rep["stages"])
    tuned = batched(ctx, fr, **kw)
    for a, b in zip(out, tuned):
        assert same(a, b)


@pytest.mark.parametrize("scheme,beta,pins", [
    ("pdr", 0.0, ((0, 3074, 3), (1, 2050, 2), (2, 512, 30))),
    ("pdr", 0.0, ((0, 4098, 1), (1, 6145, 2), (2, 2048, 4))),
    ("pdr", 0.05, ((0, 2050, 2), (1, 4098, 1), (2, 1024, 3))),
    ("alg1", 0.0, ((0, 3074, 5), (1, 2050, 10), (2, 512, 30))),
    ("alg1", 0.05, ((0, 2050, 6), (1, 1024, 3), (2, 2050, 30)))])
def test_pinned_pd_stage_choices_keep_results(ctx, scheme, beta, pins):
    """pDR / ALG1 stage choices set by hand (the work-group code and K the batched autotuner's
    report lists) change speed only: the batch stays bitwise the same; a code the scheme does not
    run, or one whose region the level cannot hold, is refused."""
    print(f"[case] batched {scheme} beta {beta} pinned {pins}", flush=True)
    fr = frames(MIX)
    kw = dict(KW, scheme=scheme, beta=beta)
    pairs = [(d0, d1, lv) for _, _, lv, d0, d1 in fr]
    c = fm.Context(0)
    try:
        before = batched(c, fr, **kw)
        for level, nt, K in pins:
            c.set_batched_stage(pairs, level, nt, K, 64, fm.Params(**kw))
        after = batched(c, fr, **kw)
        for a, b in zip(before, after):
            assert same(a, b)
        bad = 4098 if scheme == "alg1" else 1025           # a code of another scheme
        with pytest.raises(fm.FlowError):
            c.set_batched_stage(pairs, 0, bad, 2, 64, fm.Params(**kw))
        if beta > 0:                                      # the 48-row one-cell tiles need beta = 0
            with pytest.raises(fm.FlowError):
                c.set_batched_stage(pairs, 0, 3074, 2, 64, fm.Params(**kw))
    finally:
        c.close()


def test_pd_batch_matches_the_oracle(ctx):
    """Batched pDR pairs against the FP64 oracle under the parity bar."""
    print("[case] batched pdr vs oracle", flush=True)
    fr = frames(MIX[:3])
    kw = dict(KW, scheme="pdr")
    out = batched(ctx, fr, **kw)
    jobs = [(I0, I1, dict(scheme="pdr", levels=lv or KW["levels"], warps=KW["warps"], iters=KW["iters"]))
            for I0, I1, lv, _, _ in fr]
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        refs = oracle_refs(jobs, pool)(900)
    for k, ((u, v, res), ref) in enumerate(zip(out, refs)):
        assert_parity(f"batched pdr pair {k}", to_np(u), to_np(v), res, ref, job=jobs[k])


def test_invalid_pairs_are_rejected_before_anything_runs(ctx):
    print("[case] batched errors", flush=True)
    fr = frames(MIX[:2])
    good = (fr[0][3], fr[0][4])
    tiny = torch.zeros((1, 40), device="cuda")
    with pytest.raises(fm.FlowError, match="pair 1"):
        ctx.solve_batched([good, (tiny, tiny)], fm.Params(**KW))
    with pytest.raises(fm.FlowError, match="pair 0"):
        ctx.solve_batched([(fr[0][3], fr[0][4], 9)], fm.Params(**KW))   # 70x90 has no 9-level pyramid
    assert ctx.solve_batched([], fm.Params(**KW)) == []
    # the context still works afterwards
    out = batched(ctx, fr, **KW)
    assert all(np.isfinite(r["energy"]) for _, _, r in out)


def test_levels_narrower_than_a_tile_width(ctx):
    """Pairs whose coarse levels are narrower than 8 pixels (75 x 5, 5 x 100, 88 x 5): batched and
    served, their tiles span the level's width; bitwise equal to the plain solve on the same tile
    kernel, and within the FP32 bar of the oracle."""
    print("[case] narrow coarse levels", flush=True)
    spec = [(150, 10, 41, 2), (9, 200, 42, 2), (700, 40, 43, 4)]
    fr = frames(spec)
    jobs = [(I0, I1, dict(KW, levels=lv)) for I0, I1, lv, _, _ in fr]
    with mp.get_context("fork").Pool(3) as pool:
        get = oracle_refs(jobs, pool)
        out = batched(ctx, fr, **KW)
        srv = fm.Server(ctx, fm.Params(**KW), budget_bytes=64 << 20, max_active=3)
        tick = [srv.submit(d0, d1, lv) for _, _, lv, d0, d1 in fr]
        srv.drain()
        served = [srv.poll(t) for t in tick]
        srv.close()
        fm.set_tuning("tb_mode", 4)
        for k, (_, _, lv, d0, d1) in enumerate(fr):
            plain = ctx.solve(d0, d1, fm.Params(**dict(KW, levels=lv)))
            assert same(out[k], plain) and same(served[k], plain), spec[k]
        refs = get(600)
    for k, (u, v, res) in enumerate(out):
        assert_parity(f"narrow pair {spec[k][:2]}", to_np(u), to_np(v), res, refs[k], job=jobs[k])
