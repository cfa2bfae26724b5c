"""Serving engine (continuous batching): requests admitted as slots and budget free up, every
admitted pair advanced one warp per epoch in shared launches.

Checks: a served pair's results are bitwise the same alone, in a mix that changes while it runs, and
as a batched solve (pDR and ALG1: as the plain tile solve); the budget and slot limits hold; served
flows match the FP64 oracle; bad requests are refused; a pair with a non-finite frame is reported once and leaves the others
untouched.
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
SPEC = [(70, 90, 41, 0), (45, 130, 42, 0), (33, 35, 43, 2), (96, 128, 44, 0), (20, 300, 45, 2), (60, 61, 46, 0)]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fm.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def frames():
    out = []
    for H, W, seed, lv in SPEC:
        p = synth.vga_pair(seed=seed, H=H, W=W)
        out.append((f32(p.I0), f32(p.I1), lv, to_dev(f32(p.I0), 1), to_dev(f32(p.I1), 1)))
    return out


def same(a, b):
    return torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2]["energy"] == b[2]["energy"] \
        and a[2]["gap"] == b[2]["gap"]


def serve_all(srv, tickets):
    srv.drain()
    out = {}
    for k, t in tickets.items():
        r = srv.poll(t)
        assert r is not None, k
        out[k] = r
    return out


def test_served_results_are_the_same_alone_in_a_mix_and_batched(ctx, frames):
    print("[case] serve alone vs mix", flush=True)
    alone = {}
    for k in (0, 3):
        srv = fm.Server(ctx, fm.Params(**KW), budget_bytes=64 << 20, max_active=8)
        t = srv.submit(frames[k][3], frames[k][4], frames[k][2])
        alone[k] = serve_all(srv, {k: t})[k]
        srv.close()
    srv = fm.Server(ctx, fm.Params(**KW), budget_bytes=64 << 20, max_active=8)
    tick = {}
    tick[1] = srv.submit(frames[1][3], frames[1][4], frames[1][2])
    tick[2] = srv.submit(frames[2][3], frames[2][4], frames[2][2])
    for _ in range(2):
        srv.step()
    tick[0] = srv.submit(frames[0][3], frames[0][4], frames[0][2])      # joins mid-flight
    srv.step()
    tick[4] = srv.submit(frames[4][3], frames[4][4], frames[4][2])
    for _ in range(3):
        srv.step()
    tick[3] = srv.submit(frames[3][3], frames[3][4], frames[3][2])
    tick[5] = srv.submit(frames[5][3], frames[5][4], frames[5][2])
    out = serve_all(srv, tick)
    st = srv.stats()
    srv.close()
    assert st["completed"] == 6 and st["peak_active"] >= 3
    assert same(out[0], alone[0]) and same(out[3], alone[3])
    batched = ctx.solve_batched([(f[3], f[4], f[2]) for f in frames], fm.Params(**KW))
    for k in range(len(SPEC)):
        assert same(out[k], batched[k]), k


@pytest.mark.parametrize("order", [0, 1])
def test_graph_replayed_epochs_equal_direct_launches(ctx, frames, order):
    """An epoch's tile launches replayed from a captured graph (fixed tables, device tile count,
    persistent grid) give bitwise the same served results as direct launches, in both tile orders,
    and few graphs serve many epochs."""
    print(f"[case] serve graph replay order {order}", flush=True)
    fm.set_tuning("batch_order", order)
    try:
        out = {}
        stats = {}
        for g in (0, 1):
            fm.set_tuning("serve_graph", g)
            srv = fm.Server(ctx, fm.Params(**KW), budget_bytes=64 << 20, max_active=8)
            tick = {k: srv.submit(f[3], f[4], f[2]) for k, f in enumerate(frames[:4])}
            srv.step()
            tick.update({k + 4: srv.submit(f[3], f[4], f[2]) for k, f in enumerate(frames[4:])})
            out[g] = serve_all(srv, tick)
            stats[g] = srv.stats()
            srv.close()
    finally:
        fm.set_tuning("serve_graph", 1)
        fm.set_tuning("batch_order", -1)
    for k in range(len(SPEC)):
        assert same(out[0][k], out[1][k]), k
    assert stats[0]["graphs_captured"] == 0
    assert 1 <= stats[1]["graphs_captured"] < stats[1]["epochs"]


def test_budget_and_slots_bound_what_is_in_flight(ctx, frames):
    print("[case] serve admission", flush=True)
    p = fm.Params(**KW)
    sizes = [fm.working_set_bytes(f[0].shape[0], f[0].shape[1], p, f[2]) for f in frames]
    budget = sorted(sizes)[-1] + sorted(sizes)[-2]          # room for about two pairs at a time
    srv = fm.Server(ctx, p, budget_bytes=budget, max_active=8)
    tick = {k: srv.submit(f[3], f[4], f[2]) for k, f in enumerate(frames)}
    peak = 0
    while True:
        a, q = srv.step()
        peak = max(peak, a)
        if a == 0 and q == 0:
            break
    out = serve_all(srv, tick)
    st = srv.stats()
    srv.close()
    assert st["peak_bytes_in_use"] <= budget and st["completed"] == len(frames)
    assert 1 <= st["peak_active"] <= 3
    srv1 = fm.Server(ctx, p, budget_bytes=64 << 20, max_active=1)     # one slot: strictly one at a time
    tick1 = {k: srv1.submit(f[3], f[4], f[2]) for k, f in enumerate(frames)}
    out1 = serve_all(srv1, tick1)
    assert srv1.stats()["peak_active"] == 1
    srv1.close()
    for k in range(len(frames)):
        assert same(out[k], out1[k]), k


@pytest.mark.parametrize("scheme,relax,beta", [("padmm", 1.0, 0.0), ("rpadmm2", 1.9, 0.05)])
def test_served_flows_match_the_oracle(ctx, frames, scheme, relax, beta):
    print(f"[case] serve parity {scheme} {beta}", flush=True)
    kw = dict(KW, scheme=scheme, relax=relax, beta=beta)
    jobs = [(f[0], f[1], dict(kw, levels=f[2] or KW["levels"])) for f in frames[:3]]
    with mp.get_context("fork").Pool(3) as pool:
        fut = oracle_refs(jobs, pool)
        srv = fm.Server(ctx, fm.Params(**kw), budget_bytes=64 << 20, max_active=4)
        tick = {}
        for k in range(3):
            tick[k] = srv.submit(frames[k][3], frames[k][4], frames[k][2])
            srv.step()
        out = serve_all(srv, tick)
        srv.close()
        refs = fut(900)
    for k in range(3):
        u, v, res = out[k]
        assert_parity(f"served pair {k}", to_np(u), to_np(v), res, refs[k])


def test_bad_requests_are_refused(ctx, frames):
    print("[case] serve errors", flush=True)
    p = fm.Params(**KW)
    small = fm.working_set_bytes(frames[2][0].shape[0], frames[2][0].shape[1], p, frames[2][2])
    srv = fm.Server(ctx, p, budget_bytes=small, max_active=2)
    with pytest.raises(fm.FlowError, match="budget"):
        srv.submit(frames[3][3], frames[3][4], frames[3][2])               # can never fit
    tiny = torch.zeros((1, 40), device="cuda")
    with pytest.raises(fm.FlowError):
        srv.submit(tiny, tiny)
    with pytest.raises(fm.FlowError):
        srv.poll(12345)
    t = srv.submit(frames[2][3], frames[2][4], frames[2][2])              # exactly fits
    out = serve_all(srv, {0: t})
    assert np.isfinite(out[0][2]["energy"])
    srv.close()
    with pytest.raises(fm.FlowError):
        fm.Server(ctx, fm.Params(**dict(KW, tol=1e-3)))                  # fixed iteration counts only
    srv = fm.Server(ctx, fm.Params(**dict(KW, scheme="pdr", gs_sweeps=40)), budget_bytes=64 << 20)
    with pytest.raises(fm.FlowError, match="halo"):                        # no tile holds this halo
        srv.submit(frames[3][3], frames[3][4], frames[3][2])
    srv.close()


@pytest.mark.parametrize("scheme,beta", [("pdr", 0.0), ("pdr", 0.05), ("alg1", 0.0), ("alg1", 0.05)])
def test_served_pd_pairs_equal_their_plain_solves(ctx, frames, scheme, beta):
    """pDR and ALG1 served in a mix that changes while they run (pairs at different levels share the
    table-order tile launches): every result is bitwise the plain tile solve of the pair."""
    print(f"[case] serve {scheme} beta {beta}", flush=True)
    kw = dict(KW, scheme=scheme, beta=beta)
    srv = fm.Server(ctx, fm.Params(**kw), budget_bytes=64 << 20, max_active=4)
    tick = {}
    for k in range(len(frames)):
        tick[k] = srv.submit(frames[k][3], frames[k][4], frames[k][2])
        srv.step()
    out = serve_all(srv, tick)
    srv.close()
    for k, (I0, I1, lv, d0, d1) in enumerate(frames):
        ref = ctx.solve(d0, d1, fm.Params(**dict(kw, levels=lv or KW["levels"])))
        assert same(out[k], ref), f"pair {k}"


def test_served_pdr_flows_match_the_oracle(ctx, frames):
    print("[case] serve pdr vs oracle", flush=True)
    kw = dict(KW, scheme="pdr")
    srv = fm.Server(ctx, fm.Params(**kw), budget_bytes=64 << 20, max_active=8)
    tick = {k: srv.submit(frames[k][3], frames[k][4], frames[k][2]) for k in (0, 2, 5)}
    out = serve_all(srv, tick)
    srv.close()
    jobs = {k: (frames[k][0], frames[k][1], dict(scheme="pdr", levels=frames[k][2] or KW["levels"], warps=KW["warps"],
                                                 iters=KW["iters"])) for k in tick}
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        refs = oracle_refs(list(jobs.values()), pool)(900)
    for (k, job), ref in zip(jobs.items(), refs):
        u, v, res = out[k]
        assert_parity(f"served pdr pair {k}", to_np(u), to_np(v), res, ref, job=job)


def test_non_finite_pair_is_reported_and_leaves_the_others_untouched(ctx, frames):
    """A frame holding a NaN gives that pair a non-finite energy: its poll raises FLOW_E_NONFINITE
    once (outputs attached) and collects the ticket; a pair served beside it is bitwise the same as
    served alone."""
    print("[case] serve non-finite pair", flush=True)
    srv = fm.Server(ctx, fm.Params(**KW), budget_bytes=64 << 20, max_active=8)
    alone = serve_all(srv, {0: srv.submit(frames[0][3], frames[0][4], frames[0][2])})[0]
    bad = frames[1][3].contiguous().clone()
    bad[5, 7] = float("nan")
    tick = {"bad": srv.submit(bad, frames[1][4].contiguous(), frames[1][2]),
            "good": srv.submit(frames[0][3], frames[0][4], frames[0][2])}
    srv.drain()
    with pytest.raises(fm.FlowError) as e:
        srv.poll(tick["bad"])
    assert e.value.status == fm.FLOW_E_NONFINITE
    u, v, res = e.value.result
    assert u.shape == bad.shape and not np.isfinite(res["energy"])
    with pytest.raises(fm.FlowError) as e:
        srv.poll(tick["bad"])                                               # collected
    assert e.value.status == fm.FLOW_E_NOTFOUND
    assert same(srv.poll(tick["good"]), alone)
    st = srv.stats()
    srv.close()
    assert st["completed"] == 3 and st["bytes_in_use"] == 0
