"""Parity at the full sizes of the benchmark workloads, in the launch configurations the benchmark
times, against the full FP64 oracle solve.

  1920x1080, 6 levels x 5 warps x 50 iterations (rotation + zoom up to 20 px with occluding
  boxes): the built-in plan, the autotuned plan, small 1024-thread tiles at every level (the
  batched and served kernel) and the pair served through the serving engine, each within the FP32
  bar; FP16-stored pyramids against the oracle's FP16 storage form and against the FP32 form;
  the 64-pair batch of uneven sizes: every batched pair bitwise equal to its plain tile solve, the
  largest pair and the two smallest against the oracle;
  one pair of every serving size through the serving engine, bitwise equal to the batched solve.
"""
import multiprocessing as mp

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2011_10979_amd as fm  # noqa: E402
import synth  # noqa: E402
from helpers import to_dev, to_np, f32, oracle_refs, assert_parity  # noqa: E402

HD_KW = dict(levels=6, warps=5, iters=50)


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
    fm.set_tuning("tb_mode", 0)


@pytest.fixture(scope="module")
def hd():
    """The 1920x1080 pair and its oracle solves (FP32 form and FP16 storage form), started in
    worker processes when the first 1080p test begins, so they run while the GPU works."""
    pair = synth.hd_pair(seed=2)
    I0, I1 = f32(pair.I0), f32(pair.I1)
    pool = mp.get_context("fork").Pool(2)
    get = oracle_refs([(I0, I1, HD_KW), (I0, I1, dict(HD_KW, storage="f16"))], pool)
    cache = {}

    def refs():
        if not cache:
            cache["r"] = get(1200)
        return cache["r"]
    yield I0, I1, refs
    pool.terminate()


@pytest.mark.parametrize("plan", ["builtin", "autotuned", "small tiles"])
def test_hd_1080p_fp32_against_the_oracle(ctx, hd, plan):
    print(f"[case] 1920x1080 6x5x50 fp32 plan {plan}", flush=True)
    I0, I1, refs = hd
    c = ctx
    if plan == "autotuned":
        c = fm.Context(0)
        rep = c.autotune(1080, 1920, fm.Params(**HD_KW))
        print(f"[parity] 1080p autotuned plan: { {k: e['choice'] for k, e in rep.items()} }", flush=True)
    elif plan == "small tiles":
        fm.set_tuning("tb_mode", 4)
    try:
        u, v, res = c.solve(to_dev(I0), to_dev(I1), fm.Params(**HD_KW, use_graph=1))
    finally:
        if c is not ctx:
            c.close()
    assert_parity(f"1080p fp32 {plan}", to_np(u), to_np(v), res, refs()[0], mean_tol=1e-5)


def test_hd_1080p_served_against_the_oracle(ctx, hd):
    print("[case] 1920x1080 served", flush=True)
    I0, I1, refs = hd
    srv = fm.Server(ctx, fm.Params(warps=5, iters=50), budget_bytes=1 << 30, max_active=4)
    try:
        t = srv.submit(to_dev(I0), to_dev(I1), HD_KW["levels"])
        srv.drain()
        out = srv.poll(t)
    finally:
        srv.close()
    assert out is not None
    u, v, res = out
    assert_parity("1080p served", to_np(u), to_np(v), res, refs()[0], mean_tol=1e-5)


def test_hd_1080p_fp16_storage(ctx, hd):
    """FP16-stored pyramids with FP32 arithmetic.  Against the oracle's FP16 storage form (the same
    binary16 pyramid planes, FP64 solve) the flow meets the FP32 bar; against the FP32 form its
    endpoint-error difference is the storage form's own: mean <= 1e-2 px (the contract), and the
    worst pixels are those where the oracle's two forms differ most."""
    print("[case] 1920x1080 fp16 storage", flush=True)
    I0, I1, refs = hd
    u, v, res = ctx.solve(to_dev(I0), to_dev(I1), fm.Params(**HD_KW, storage="f16"))
    u, v = to_np(u), to_np(v)
    r32, r16 = refs()
    assert_parity("1080p fp16 vs the oracle's fp16 form", u, v, res, r16, mean_tol=1e-5)
    epe = np.hypot(u - r32["u"], v - r32["v"])
    form = np.hypot(r16["u"] - r32["u"], r16["v"] - r32["v"])
    i, j = np.unravel_index(int(np.argmax(epe)), epe.shape)
    print(f"[parity] 1080p fp16 storage: EPE vs the FP32 form mean {epe.mean():.3e} p99.9 "
          f"{np.quantile(epe, 0.999):.3e} max {epe.max():.3e} at ({i},{j}); the oracle's fp16 form: mean "
          f"{form.mean():.3e} p99.9 {np.quantile(form, 0.999):.3e} max {form.max():.3e}", flush=True)
    assert epe.mean() <= 1e-2
    # |gpu - fp32 form| <= |gpu - fp16 form| + |fp16 form - fp32 form|, and the first is within
    # sqrt(2) x 1e-4 px at every pixel (asserted above)
    assert np.quantile(epe, 0.999) <= np.quantile(form, 0.999) + 1.5e-4
    assert epe.max() <= form.max() + 1.5e-4


def _gen(k):
    p = synth.batch_pair(k)
    return f32(p.I0), f32(p.I1)


def test_batch_of_64_uneven_pairs(ctx):
    print("[case] batch of 64", flush=True)
    with mp.get_context("fork").Pool(16) as pool:
        host = pool.map(_gen, range(64))
    kw = dict(warps=5, iters=50)
    by_size = sorted(range(64), key=lambda k: host[k][0].size)
    picked = [by_size[-1]] + by_size[:2]            # the largest pair and the two smallest
    jobs = [(host[k][0], host[k][1], dict(kw, levels=synth.levels_by_size(*host[k][0].shape))) for k in picked]
    with mp.get_context("fork").Pool(3) as pool:
        get = oracle_refs(jobs, pool)
        frames = [(to_dev(a), to_dev(b), synth.levels_by_size(*a.shape)) for a, b in host]
        out = ctx.solve_batched(frames, fm.Params(**kw, use_graph=1))
        # the stage choice the benchmark times (autotuned) gives the same results bit for bit
        tuned = fm.Context(0)
        try:
            tuned.autotune_batched(frames, fm.Params(**kw))
            out_t = tuned.solve_batched(frames, fm.Params(**kw, use_graph=1))
        finally:
            tuned.close()
        for k in range(64):
            assert torch.equal(out_t[k][0], out[k][0]) and torch.equal(out_t[k][1], out[k][1]), k
            assert out_t[k][2]["energy"] == out[k][2]["energy"], k
        fm.set_tuning("tb_mode", 4)
        for k, (I0, I1, lv) in enumerate(frames):
            u, v, res = ctx.solve(I0, I1, fm.Params(**kw, levels=lv))
            assert torch.equal(u, out[k][0]) and torch.equal(v, out[k][1]) and res["energy"] == out[k][2]["energy"], k
        refs = get(1200)
    for i, k in enumerate(picked):
        assert_parity(f"batch pair {k} {host[k][0].shape}", to_np(out[k][0]), to_np(out[k][1]), out[k][2], refs[i],
                      mean_tol=1e-5)


def test_serving_sizes_through_the_engine(ctx):
    print("[case] serving sizes", flush=True)
    frames = []
    for si, (H, W) in enumerate(synth.SERVING_SIZES):
        p = synth.vga_pair(7000 + si, H, W)
        frames.append((to_dev(f32(p.I0)), to_dev(f32(p.I1)), synth.levels_by_size(H, W)))
    kw = dict(warps=5, iters=50)
    srv = fm.Server(ctx, fm.Params(**kw), budget_bytes=2 << 30, max_active=16)
    tick = []
    for f in frames:
        tick.append(srv.submit(*f))
        srv.step()
    srv.drain()
    served = [srv.poll(t) for t in tick]
    srv.close()
    batched = ctx.solve_batched(frames, fm.Params(**kw))
    for k in range(len(frames)):
        assert torch.equal(served[k][0], batched[k][0]) and torch.equal(served[k][1], batched[k][1]), k
        assert served[k][2]["energy"] == batched[k][2]["energy"]
