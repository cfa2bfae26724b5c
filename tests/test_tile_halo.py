"""The halo of the K-iteration tile kernels is sufficient and tight, checked on the CPU with the oracle.

A tile kernel loads an output tile plus a halo and advances that extended region by K iterations
without seeing anything outside it.  Here the same is done with the oracle's steps on the whole
image, after replacing every value outside the extended region (state and linearisation) by
random garbage: inside the output tile the result must equal the undisturbed run bit for bit.  With
one row or column less on any side (away from the image border) some output value must change, so
the halo is also the smallest one that works.  The halo sizes are the ones the tile planner and
kernels use:

  ADMM family (Sec. 3.1.1)        K + 1 above / left,    K below / right
  pDR with n sweeps (Sec. 3.1.2)  (2n+1) K above / left, (2n+1) K + 1 below / right
  ALG1 (Sec. 4)                   K on every side
"""
import zlib

import numpy as np
import pytest

from oracle import schemes

SHAPE = (41, 47)
LAM, C = 0.05, 0.05


def _admm_state(rng, beta):
    st = {k: rng.normal(scale=2.0, size=SHAPE) for k in ("u", "v")}
    for k in ("q1x", "q1y", "q2x", "q2y"):
        st[k] = rng.uniform(-0.5, 0.5, size=SHAPE)
    st["s"] = rng.uniform(-0.05, 0.05, size=SHAPE)
    st["w"] = rng.normal(scale=0.5, size=SHAPE) if beta > 0 else np.zeros(SHAPE)
    for k in ("px", "py"):
        st[k] = rng.uniform(-0.6, 0.6, size=SHAPE) if beta > 0 else np.zeros(SHAPE)
    return st


def _pd_state(rng, beta):
    st = {k: rng.normal(scale=1.5, size=SHAPE) for k in ("u", "v", "ub", "vb")}
    for k in ("qb1x", "qb1y", "qb2x", "qb2y"):
        st[k] = rng.uniform(-0.6, 0.6, size=SHAPE)
    for k in ("w", "wb"):
        st[k] = rng.normal(scale=0.5, size=SHAPE) if beta > 0 else np.zeros(SHAPE)
    for k in ("pbx", "pby"):
        st[k] = rng.uniform(-0.6, 0.6, size=SHAPE) if beta > 0 else np.zeros(SHAPE)
    return st


def _lin(rng, beta):
    L = {k: rng.normal(0, s, size=SHAPE) for k, s in (("Ix", 20), ("Iy", 20), ("It", 15))}
    L["at"] = float(np.max(beta * beta + L["Ix"] ** 2 + L["Iy"] ** 2))
    return L


def _scheme(name, beta, n):
    if name == "admm":
        return _admm_state, lambda st, L: schemes.rpadmm1_step(st, L, beta, LAM, C, 1.0)
    if name == "rpadmm2":
        return _admm_state, lambda st, L: schemes.rpadmm2_step(st, L, beta, LAM, C, 1.9)
    if name == "pdr":
        return _pd_state, lambda st, L: schemes.pdr_step(st, L, beta, LAM, 2.0, 0.4, n)[0]
    return _pd_state, lambda st, L: schemes.alg1_step(st, L, beta, LAM, 0.1, 1.25)[0]


def _halo(name, K, n):
    if name in ("admm", "rpadmm2"):
        return K + 1, K
    if name == "pdr":
        return (2 * n + 1) * K, (2 * n + 1) * K + 1
    return K, K


def _tile_result(step, st, L, K, tile, lo, hi, rng):
    """K steps with everything outside the extended region (lo = (top, left), hi = (bottom,
    right)) replaced by garbage; returns the output tile of every state field."""
    y0, x0, th, tw = tile
    H, W = SHAPE
    ey0, ex0 = max(y0 - lo[0], 0), max(x0 - lo[1], 0)
    ey1, ex1 = min(y0 + th + hi[0], H), min(x0 + tw + hi[1], W)

    def cut(a):
        b = rng.normal(scale=3.0, size=SHAPE)
        b[ey0:ey1, ex0:ex1] = a[ey0:ey1, ex0:ex1]
        return b

    s = {k: cut(v) for k, v in st.items()}
    lin = {k: (cut(v) if np.ndim(v) else v) for k, v in L.items()}
    for _ in range(K):
        s = step(s, lin)
    return {k: v[y0:y0 + th, x0:x0 + tw] for k, v in s.items()}


def _setup(name, beta, n, K, seed):
    rng = np.random.default_rng(seed)
    make, step = _scheme(name, beta, n)
    st, L = make(rng, beta), _lin(rng, beta)
    full = dict(st)
    for _ in range(K):
        full = step(full, L)
    return rng, step, st, L, full


CASES = [("admm", 0.0, 1, 1), ("admm", 0.05, 1, 3), ("rpadmm2", 0.05, 1, 2), ("pdr", 0.0, 1, 1),
         ("pdr", 0.05, 1, 2), ("pdr", 0.0, 2, 1), ("alg1", 0.0, 1, 2), ("alg1", 0.05, 1, 4)]


@pytest.mark.parametrize("name,beta,n,K", CASES)
def test_tile_halo_is_sufficient(name, beta, n, K):
    rng, step, st, L, full = _setup(name, beta, n, K, seed=zlib.crc32(repr((name, beta, n, K)).encode()))
    lo, hi = _halo(name, K, n)
    # interior tiles, tiles on every border and a corner, odd and even offsets
    for tile in [(15, 17, 7, 9), (16, 18, 6, 5), (0, 0, 8, 8), (SHAPE[0] - 6, SHAPE[1] - 7, 6, 7),
                 (0, 20, 5, 9), (21, 0, 9, 6)]:
        got = _tile_result(step, st, L, K, tile, (lo, lo), (hi, hi), rng)
        y0, x0, th, tw = tile
        for k, v in got.items():
            assert np.array_equal(v, full[k][y0:y0 + th, x0:x0 + tw]), (tile, k)


@pytest.mark.parametrize("name,beta,n,K", CASES)
@pytest.mark.parametrize("side", ["top", "left", "bottom", "right"])
def test_tile_halo_is_tight(name, beta, n, K, side):
    rng, step, st, L, full = _setup(name, beta, n, K, seed=zlib.crc32(repr((name, beta, n, K, side)).encode()))
    lo, hi = _halo(name, K, n)
    lo2, hi2 = [lo, lo], [hi, hi]
    {"top": lo2, "left": lo2, "bottom": hi2, "right": hi2}[side][0 if side in ("top", "bottom") else 1] -= 1
    tile = (16, 17, 8, 9)   # far enough from every border for the largest halo here
    got = _tile_result(step, st, L, K, tile, tuple(lo2), tuple(hi2), rng)
    y0, x0, th, tw = tile
    assert any(not np.array_equal(v, full[k][y0:y0 + th, x0:x0 + tw]) for k, v in got.items()), side


# The kernels go further than the halo: after iteration m of a launch only the extended region
# shrunk by m rows on every side that has a halo can still reach the output, so rows outside that
# band skip the iteration and keep stale values (a whole wavefront's rows in the general ADMM
# tiles, single rows in the ADMM and ALG1 wave-row tiles).  Stale values are one kind of garbage;
# here the rows
# outside the band are replaced by random values after every iteration, and the output tile must
# still equal the undisturbed run bit for bit.  With a band one row narrower on either side some
# output value changes (for K >= 2: with one iteration the row above the output tile can no longer
# reach it), so the band is the narrowest that works.

def _band_result(step, st, L, K, tile, lo, hi, rng, extra=(0, 0)):
    """Like _tile_result, and after iteration m (1-based) every row outside the extended region
    shrunk by m rows (plus extra = (top, bottom)) on the top and bottom, where the region does not
    meet the image border, is overwritten with garbage."""
    y0, x0, th, tw = tile
    H, W = SHAPE
    ey0, ex0 = max(y0 - lo[0], 0), max(x0 - lo[1], 0)
    ey1, ex1 = min(y0 + th + hi[0], H), min(x0 + tw + hi[1], W)

    def cut(a, r0, r1):
        b = rng.normal(scale=3.0, size=SHAPE)
        b[r0:r1, ex0:ex1] = a[r0:r1, ex0:ex1]
        return b

    s = {k: cut(v, ey0, ey1) for k, v in st.items()}
    lin = {k: (cut(v, ey0, ey1) if np.ndim(v) else v) for k, v in L.items()}
    for m in range(1, K + 1):
        s = step(s, lin)
        r0 = ey0 + m + extra[0] if ey0 > 0 else 0
        r1 = ey1 - m - extra[1] if ey1 < H else H
        s = {k: cut(v, r0, r1) for k, v in s.items()}
    return {k: v[y0:y0 + th, x0:x0 + tw] for k, v in s.items()}


BAND_CASES = [c for c in CASES if c[0] in ("admm", "rpadmm2", "alg1")] + [("admm", 0.0, 1, 5), ("admm", 0.05, 1, 6),
                                                                            ("alg1", 0.0, 1, 5)]


@pytest.mark.parametrize("name,beta,n,K", BAND_CASES)
def test_rows_outside_the_shrinking_band_may_hold_anything(name, beta, n, K):
    rng, step, st, L, full = _setup(name, beta, n, K, seed=zlib.crc32(repr(("band", name, beta, n, K)).encode()))
    lo, hi = _halo(name, K, n)
    for tile in [(15, 17, 7, 9), (16, 18, 6, 5), (0, 0, 8, 8), (SHAPE[0] - 6, SHAPE[1] - 7, 6, 7),
                 (0, 20, 5, 9), (21, 0, 9, 6)]:
        got = _band_result(step, st, L, K, tile, (lo, lo), (hi, hi), rng)
        y0, x0, th, tw = tile
        for k, v in got.items():
            assert np.array_equal(v, full[k][y0:y0 + th, x0:x0 + tw]), (tile, k)


@pytest.mark.parametrize("name,beta,n,K", [c for c in BAND_CASES if c[3] >= 2])
@pytest.mark.parametrize("extra", [(1, 0), (0, 1)], ids=["top", "bottom"])
def test_shrinking_band_is_tight(name, beta, n, K, extra):
    rng, step, st, L, full = _setup(name, beta, n, K,
                                    seed=zlib.crc32(repr(("band-tight", name, beta, n, K, extra)).encode()))
    lo, hi = _halo(name, K, n)
    tile = (16, 17, 8, 9)
    got = _band_result(step, st, L, K, tile, (lo, lo), (hi, hi), rng, extra)
    y0, x0, th, tw = tile
    assert any(not np.array_equal(v, full[k][y0:y0 + th, x0:x0 + tw]) for k, v in got.items())


# The pDR wave-row tiles skip rows in every phase of an iteration (b, the half sweeps, the resolvent
# and dual step): a skipped row keeps its state and its neighbours in the band read that state.
# Modelled here phase by phase with the oracle's operators: at iteration m (0-based) only the rows
# of the extended region shrunk by (2n + 1) m + 1 rows on every side with a halo are computed, and
# the output tile still equals the undisturbed run bit for bit; one row more on either side changes
# it.

def _pdr_step_rows(st, L, beta, n, rows):
    """schemes.pdr_step where only the rows flagged in `rows` are computed, phase by phase."""
    sigma, tau = 2.0, 0.4
    Ix, Iy, It = L["Ix"], L["Iy"], L["It"]
    stt = sigma * tau
    has_w = beta != 0.0
    M = rows[:, None]
    red = schemes.red_mask(SHAPE)
    black = ~red

    def sweep(x, b):
        for _ in range(n):
            for col in (red, black, black, red):
                x = np.where(M, schemes.gs_colour_update(x, b, stt, col), x)
        return x

    w = sweep(st["w"], st["wb"] + sigma * schemes.div(st["pbx"], st["pby"])) if has_w else st["w"]
    u = sweep(st["u"], st["ub"] + sigma * schemes.div(st["qb1x"], st["qb1y"]))
    v = sweep(st["v"], st["vb"] + sigma * schemes.div(st["qb2x"], st["qb2y"]))
    Jw, Ju, Jv, _ = schemes.resolvent(2 * w - st["wb"], 2 * u - st["ub"], 2 * v - st["vb"], Ix, Iy, It, beta, LAM,
                                      sigma)

    def keep(new, old):
        return np.where(M, new, old)
    gwx, gwy = schemes.grad(w)
    gux, guy = schemes.grad(u)
    gvx, gvy = schemes.grad(v)
    ppx, ppy = (schemes.proj_p(st["pbx"] + 2 * tau * gwx, st["pby"] + 2 * tau * gwy) if has_w
                else (st["pbx"], st["pby"]))
    q1x, q1y, q2x, q2y = schemes.proj_q(st["qb1x"] + 2 * tau * gux, st["qb1y"] + 2 * tau * guy,
                                        st["qb2x"] + 2 * tau * gvx, st["qb2y"] + 2 * tau * gvy)
    return dict(w=w, u=u, v=v, wb=keep(st["wb"] + Jw - w, st["wb"]) if has_w else st["wb"],
                ub=keep(st["ub"] + Ju - u, st["ub"]), vb=keep(st["vb"] + Jv - v, st["vb"]),
                pbx=keep(ppx - tau * gwx, st["pbx"]) if has_w else st["pbx"],
                pby=keep(ppy - tau * gwy, st["pby"]) if has_w else st["pby"],
                qb1x=keep(q1x - tau * gux, st["qb1x"]), qb1y=keep(q1y - tau * guy, st["qb1y"]),
                qb2x=keep(q2x - tau * gvx, st["qb2x"]), qb2y=keep(q2y - tau * gvy, st["qb2y"]))


def _pdr_row_band_result(st, L, beta, n, K, tile, rng, extra=(0, 0)):
    lo, hi = _halo("pdr", K, n)
    y0, x0, th, tw = tile
    H, W = SHAPE
    ey0, ex0 = max(y0 - lo, 0), max(x0 - lo, 0)
    ey1, ex1 = min(y0 + th + hi, H), min(x0 + tw + hi, W)

    def cut(a):
        b = rng.normal(scale=3.0, size=SHAPE)
        b[ey0:ey1, ex0:ex1] = a[ey0:ey1, ex0:ex1]
        return b

    s = {k: cut(v) for k, v in st.items()}
    lin = {k: (cut(v) if np.ndim(v) else v) for k, v in L.items()}
    for m in range(K):
        d = (2 * n + 1) * m + 1
        rows = np.zeros(H, bool)
        rows[ey0 + d + extra[0] if ey0 > 0 else 0:ey1 - d - extra[1] if ey1 < H else H] = True
        s = _pdr_step_rows(s, lin, beta, n, rows)
    return {k: v[y0:y0 + th, x0:x0 + tw] for k, v in s.items()}


PDR_ROW_CASES = [(0.0, 1, 1), (0.0, 1, 2), (0.05, 1, 3), (0.0, 2, 2), (0.0, 1, 3)]


@pytest.mark.parametrize("beta,n,K", PDR_ROW_CASES)
def test_pdr_rows_outside_the_band_may_skip_every_phase(beta, n, K):
    rng, step, st, L, full = _setup("pdr", beta, n, K, seed=zlib.crc32(repr(("pdr-rows", beta, n, K)).encode()))
    if K == 1:                                       # with every row computed the model is pdr_step itself
        one = _pdr_step_rows(st, L, beta, n, np.ones(SHAPE[0], bool))
        assert all(np.array_equal(v, full[k]) for k, v in one.items())
    for tile in [(15, 17, 7, 9), (16, 18, 6, 5), (0, 0, 8, 8), (SHAPE[0] - 6, SHAPE[1] - 7, 6, 7),
                 (0, 20, 5, 9), (21, 0, 9, 6)]:
        got = _pdr_row_band_result(st, L, beta, n, K, tile, rng)
        y0, x0, th, tw = tile
        for k, v in got.items():
            assert np.array_equal(v, full[k][y0:y0 + th, x0:x0 + tw]), (tile, k)


@pytest.mark.parametrize("beta,n,K", PDR_ROW_CASES)
@pytest.mark.parametrize("extra", [(1, 0), (0, 1)], ids=["top", "bottom"])
def test_pdr_row_band_is_tight(beta, n, K, extra):
    rng, step, st, L, full = _setup("pdr", beta, n, K,
                                    seed=zlib.crc32(repr(("pdr-rows-tight", beta, n, K, extra)).encode()))
    tile = (16, 17, 8, 9)
    got = _pdr_row_band_result(st, L, beta, n, K, tile, rng, extra)
    y0, x0, th, tw = tile
    assert any(not np.array_equal(v, full[k][y0:y0 + th, x0:x0 + tw]) for k, v in got.items())


def _tile_regions(shape, tile, lo, hi):
    """Extended regions (clipped) of every tile of a regular tiling: (ey0, ex0, ey1, ex1)."""
    H, W = shape
    for y0 in range(0, H, tile[0]):
        for x0 in range(0, W, tile[1]):
            th, tw = min(tile[0], H - y0), min(tile[1], W - x0)
            yield y0 - lo, x0 - lo, y0 + th + hi, x0 + tw + hi


def _kinds(shape, regions):
    """Which kinds of tile occur: an interior region (no image edge inside it), and regions that
    reach each of the four image edges."""
    H, W = shape
    kinds = set()
    for ey0, ex0, ey1, ex1 in regions:
        edges = {"top": ey0 <= 0, "left": ex0 <= 0, "bottom": ey1 >= H, "right": ex1 >= W}
        kinds |= {k for k, v in edges.items() if v}
        if not any(edges.values()):
            kinds.add("interior")
    return kinds


def test_wave_row_parity_cases_cover_interior_and_edge_tiles():
    """The wave-row tiles take a branch of their own where the extended region holds no image edge
    (every neighbour coefficient 1); the GPU cases that compare them bitwise with the general tiles
    run both branches: tiles inside the image and tiles at each of its edges."""
    import test_gpu_ops as g
    admm, pdr = set(), set()
    for shape, tile, K, _ in g._row_cases():
        admm |= _kinds(shape, _tile_regions(shape, tile, K + 1, K))
    for shape, tile, K, n, _, _ in g._pdr_row_cases():
        pdr |= _kinds(shape, _tile_regions(shape, tile, (2 * n + 1) * K, (2 * n + 1) * K + 1))
    want = {"interior", "top", "left", "bottom", "right"}
    assert admm >= want, admm
    assert pdr >= want, pdr
