"""Operator-level parity: one GPU step against the FP64 oracle on identical inputs.

Shapes span several wavefront strips (61 columns) and row segments with ragged tails, pitches
padded beyond W, and the degenerate 2 x N / N x 2 frames.
"""
import zlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2011_10979_amd as fm  # noqa: E402
from oracle import ops, pyramid, schemes, energy  # noqa: E402
from helpers import to_dev, to_np, f32, random_admm_state, random_lin, max_abs  # noqa: E402

ROW_CODES = (2049, 3073, 4097)   # wave-row tile codes: 64 columns x 32 / 48 / 64 rows

SHAPES = [(2, 2), (2, 67), (67, 2), (3, 5), (17, 61), (70, 130), (129, 200), (240, 320)]


@pytest.fixture(autouse=True, scope="module")
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fm.lib()


def print_case(name, **kw):
    print(f"[case] {name} {kw}", flush=True)


@pytest.mark.parametrize("shape", SHAPES)
def test_downsample_and_derivatives(shape):
    print_case("downsample", shape=shape)
    rng = np.random.default_rng(1)
    I = f32(rng.uniform(size=shape))
    d = to_np(fm.downsample(to_dev(I, pad=5)))
    assert max_abs(d, pyramid.downsample(I)) < 1e-6
    Dx, Dy = fm.derivatives(to_dev(I, pad=3))
    ox, oy = pyramid.derivatives(I)
    assert max_abs(to_np(Dx), ox) < 1e-6
    assert max_abs(to_np(Dy), oy) < 1e-6


@pytest.mark.parametrize("shape", [(2, 2), (5, 7), (70, 130), (240, 320)])
@pytest.mark.parametrize("beta", [0.0, 0.05])
def test_linearize(shape, beta):
    print_case("linearize", shape=shape, beta=beta)
    rng = np.random.default_rng(2)
    H, W = shape
    I0 = f32(rng.uniform(size=shape))
    I1 = f32(rng.uniform(size=shape))
    Dx, Dy = (f32(a) for a in pyramid.derivatives(I1))
    u0 = f32(rng.normal(scale=3.0, size=shape))
    v0 = f32(rng.normal(scale=3.0, size=shape))
    u0[0, 0], v0[0, 0] = 2.0 * W, -2.0 * H          # far outside: clamped
    if H > 1 and W > 1:
        u0[-1, -1], v0[-1, -1] = 0.0, 0.0           # exactly on the last node
    g = fm.linearize(*(to_dev(a, pad=7) for a in (I0, I1, Dx, Dy, u0, v0)), kappa=255.0, beta=beta)
    Ix, Iy, It, at = pyramid.linearize(I0, I1, Dx, Dy, u0, v0, 255.0, beta)
    assert max_abs(to_np(g[0]), Ix) < 2e-4
    assert max_abs(to_np(g[1]), Iy) < 2e-4
    assert max_abs(to_np(g[2]), It) < 5e-4 * max(1.0, np.abs(It).max() / 100)
    assert abs(float(g[3].item()) - at) <= 2e-6 * at


@pytest.mark.parametrize("shape", [(3, 3), (5, 8), (60, 80), (121, 161)])
def test_upsample(shape):
    print_case("upsample", shape=shape)
    rng = np.random.default_rng(3)
    Hf, Wf = shape
    C = f32(rng.normal(size=((Hf + 1) // 2, (Wf + 1) // 2)))
    got = to_np(fm.upsample(to_dev(C), (Hf, Wf), 2.0))
    assert max_abs(got, pyramid.upsample(C, (Hf, Wf), 2.0)) < 2e-6


def _dev_state(st, pad):
    return {k: to_dev(v, pad=pad) for k, v in st.items()}


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("scheme,relax,beta", [("padmm", 1.0, 0.0), ("padmm", 1.618, 0.0), ("padmm", 1.0, 0.05),
                                               ("rpadmm2", 1.9, 0.0), ("rpadmm2", 1.9, 0.05)])
def test_admm_iteration(shape, scheme, relax, beta):
    print_case("admm_iter", shape=shape, scheme=scheme, relax=relax, beta=beta)
    rng = np.random.default_rng(zlib.crc32(repr((shape, scheme, relax, beta)).encode()))
    st = random_admm_state(rng, shape, beta)
    Ix, Iy, It, at = random_lin(rng, shape, beta)
    L = dict(Ix=Ix, Iy=Iy, It=It, at=at)
    p = fm.Params(scheme=scheme, relax=relax, beta=beta)
    gst = _dev_state(st, pad=11)
    at_t = torch.tensor([at], dtype=torch.float32, device="cuda")
    out = fm.admm_iter(gst, to_dev(Ix, 11), to_dev(Iy, 11), to_dev(It, 11), at_t, p)
    if scheme == "padmm":
        ref = schemes.rpadmm1_step(st, L, beta, 0.05, 0.05, relax)
    else:
        ref = schemes.rpadmm2_step(st, L, beta, 0.05, 0.05, relax)
    keys = ["u", "v", "q1x", "q1y", "q2x", "q2y", "s"] + (["w", "px", "py"] if beta > 0 else [])
    for k in keys:
        tol = 2e-5 if k in ("s",) else 1e-4
        assert max_abs(to_np(out[k]), ref[k]) < tol, (k, max_abs(to_np(out[k]), ref[k]))


def test_admm_iteration_chain_matches_oracle():
    """25 chained iterations on a 129 x 200 random linearisation (no divergence of the streams)."""
    rng = np.random.default_rng(7)
    shape = (129, 200)
    st = random_admm_state(rng, shape, 0.0)
    Ix, Iy, It, at = random_lin(rng, shape, 0.0)
    L = dict(Ix=Ix, Iy=Iy, It=It, at=at)
    p = fm.Params()
    g = _dev_state(st, pad=0)
    dI = [to_dev(a) for a in (Ix, Iy, It)]
    at_t = torch.tensor([at], dtype=torch.float32, device="cuda")
    for _ in range(25):
        g = fm.admm_iter(g, *dI, at_t, p)
        st = schemes.rpadmm1_step(st, L, 0.0, 0.05, 0.05, 1.0)
    for k in ("u", "v", "s", "q1x"):
        assert max_abs(to_np(g[k]), st[k]) < 2e-4, k


def random_pdr_state(rng, shape, beta):
    st = {k: f32(rng.normal(scale=1.5, size=shape)) for k in ("u", "v", "ub", "vb")}
    for k in ("qb1x", "qb1y", "qb2x", "qb2y"):
        st[k] = f32(rng.uniform(-0.6, 0.6, size=shape))
    if beta > 0:
        st["w"] = f32(rng.normal(scale=0.5, size=shape))
        st["wb"] = f32(rng.normal(scale=0.5, size=shape))
        st["pbx"] = f32(rng.uniform(-0.6, 0.6, size=shape))
        st["pby"] = f32(rng.uniform(-0.6, 0.6, size=shape))
    else:
        for k in ("w", "wb", "pbx", "pby"):
            st[k] = np.zeros(shape)
    return st


@pytest.mark.parametrize("shape", [(2, 2), (3, 5), (17, 61), (70, 130)])
@pytest.mark.parametrize("sweeps,beta", [(1, 0.0), (2, 0.0), (1, 0.05), (3, 0.05)])
def test_pdr_iteration(shape, sweeps, beta):
    print_case("pdr_iter", shape=shape, sweeps=sweeps, beta=beta)
    rng = np.random.default_rng(17)
    st = random_pdr_state(rng, shape, beta)
    Ix, Iy, It, _ = random_lin(rng, shape, beta)
    p = fm.Params(scheme="pdr", gs_sweeps=sweeps, beta=beta)
    g = {k: to_dev(v, pad=4) for k, v in st.items()}
    s_out = to_dev(np.zeros(shape), pad=4)
    fm.pdr_iter(g, to_dev(Ix, 4), to_dev(Iy, 4), to_dev(It, 4), p, s_out=s_out)
    ref, duals = schemes.pdr_step(st, dict(Ix=Ix, Iy=Iy, It=It), beta, 0.05, 2.0, 0.4, sweeps)
    keys = ["u", "v", "ub", "vb", "qb1x", "qb1y", "qb2x", "qb2y"] + (["w", "wb", "pbx", "pby"] if beta > 0 else [])
    for k in keys:
        assert max_abs(to_np(g[k]), ref[k]) < 1e-4, (k, max_abs(to_np(g[k]), ref[k]))
    assert max_abs(to_np(s_out), duals["s"]) < 1e-5


@pytest.mark.parametrize("shape,tile,K", [((7, 5), (7, 5), 6), ((37, 130), (8, 30), 2), ((101, 250), (12, 20), 1),
                                          ((40, 45), (40, 45), 9), ((64, 64), (10, 18), 2), ((33, 47), (5, 9), 3),
                                          ((101, 250), (40, 40), 2), ((64, 64), (51, 51), 2), ((130, 140), (30, 50), 3),
                                          ((60, 61), (60, 61), 4)])
@pytest.mark.parametrize("sweeps,beta", [(1, 0.0), (1, 0.05), (2, 0.0)])
def test_pdr_tiles_match_k_oracle_steps(shape, tile, K, sweeps, beta):
    """K pDR iterations of the tile kernel (halo (2n+1)K / (2n+1)K + 1, ragged tiles, resident levels;
    extended regions above 2048 cells run the large tiles, beta = 0) against K steps of the oracle on
    the same state, I_t relative to (u0, v0)."""
    print_case("pdr_tb", shape=shape, tile=tile, K=K, sweeps=sweeps, beta=beta)
    halo = (4 * sweeps + 2) * K + 1
    oversized = min(shape[0], tile[0] + halo) * min(shape[1], tile[1] + halo) > (4096 if beta == 0 else 2048)
    rng = np.random.default_rng(zlib.crc32(repr(("pdrtb", shape, tile, K, sweeps, beta)).encode()))
    st = random_pdr_state(rng, shape, beta)
    Ix, Iy, Itr, _ = random_lin(rng, shape, beta)
    u0 = f32(rng.normal(scale=3.0, size=shape))
    v0 = f32(rng.normal(scale=3.0, size=shape))
    g = {k: to_dev(v, pad=3) for k, v in st.items()}

    def call():
        return fm.pdr_tb(g, to_dev(Ix, 3), to_dev(Iy, 3), to_dev(Itr, 3), to_dev(u0, 3), to_dev(v0, 3),
                         fm.Params(scheme="pdr", gs_sweeps=sweeps, beta=beta), iters=K, tile_h=tile[0], tile_w=tile[1])
    if oversized:                                    # refused before any launch
        with pytest.raises(fm.FlowError, match="capacity") as e:
            call()
        assert e.value.status == fm.FLOW_E_INVAL
        return
    L = dict(Ix=Ix, Iy=Iy, It=Itr - Ix * u0 - Iy * v0)
    ref = dict(st)
    for _ in range(K):
        ref, duals = schemes.pdr_step(ref, L, beta, 0.05, 2.0, 0.4, sweeps)
    out, s_out = call()
    keys = ["u", "v", "ub", "vb", "qb1x", "qb1y", "qb2x", "qb2y"] + (["w", "wb", "pbx", "pby"] if beta > 0 else [])
    tol = 1e-4 * max(1, K)
    for k in keys:
        assert max_abs(to_np(out[k]), ref[k]) < tol, (k, max_abs(to_np(out[k]), ref[k]))
    assert max_abs(to_np(s_out), duals["s"]) < tol
    for k in keys:                                   # the input state is left as it was
        assert np.array_equal(to_np(g[k]), f32(st[k]))


@pytest.mark.parametrize("shape,tile,K,small", [((101, 250), (40, 40), 2, (12, 20)), ((64, 64), (51, 51), 2, (10, 18)),
                                                ((60, 61), (60, 61), 4, (5, 9)), ((130, 140), (30, 50), 3, (7, 11))])
def test_large_pdr_tiles_equal_the_1024_thread_tiles(shape, tile, K, small):
    """A large tile (1024 threads, two cells of each colour per thread) computes each cell with the
    same expression on the same operands as the 1024-thread tiles: K iterations of both tilings of
    the same state agree bit for bit."""
    print_case("pdr_tb large vs small", shape=shape, tile=tile, K=K, small=small)
    rng = np.random.default_rng(zlib.crc32(repr(("pdrtb2", shape, tile, K)).encode()))
    st = random_pdr_state(rng, shape, 0.0)
    Ix, Iy, Itr, _ = random_lin(rng, shape, 0.0)
    u0 = f32(rng.normal(scale=3.0, size=shape))
    v0 = f32(rng.normal(scale=3.0, size=shape))
    g = {k: to_dev(v, pad=3) for k, v in st.items()}
    outs = [fm.pdr_tb(g, to_dev(Ix, 3), to_dev(Iy, 3), to_dev(Itr, 3), to_dev(u0, 3), to_dev(v0, 3),
                      fm.Params(scheme="pdr"), iters=K, tile_h=t[0], tile_w=t[1]) for t in (tile, small)]
    for k in ["u", "v", "ub", "vb", "qb1x", "qb1y", "qb2x", "qb2y"]:
        assert torch.equal(outs[0][0][k], outs[1][0][k]), k
    assert torch.equal(outs[0][1], outs[1][1])


def _pdr_row_cases():
    """(shape, tile, K, sweeps, beta, mode): wave-row pDR tiles (mode 12: 128 x 32 cells, 13: 128 x 48,
    14: 64 x 48 with one cell per lane, 15: 64 x 32) whose extended region also fits the general
    tiles used as reference (4096 cells, 2048 with w)."""
    cases = []
    for shape, tile, K, n in [((101, 250), (19, 50), 2, 1), ((130, 140), (17, 80), 3, 1), ((60, 61), (60, 61), 4, 1),
                              ((45, 200), (20, 115), 1, 1), ((90, 170), (10, 90), 1, 2), ((33, 128), (33, 128), 6, 1),
                              ((28, 100), (28, 100), 5, 1), ((40, 60), (10, 30), 1, 1), ((70, 300), (15, 40), 2, 1)]:
        halo = (2 * n + 1) * K * 2 + 1
        eh, ew = min(shape[0], tile[0] + halo), min(shape[1], tile[1] + halo)
        for beta in (0.0, 0.05):
            for mode, rows, cols in ((12, 32, 128), (13, 48, 128), (14, 48, 64), (15, 32, 64)):
                if ew <= cols and eh <= rows and eh * ew <= (2048 if beta > 0 else 4096):
                    cases.append((shape, tile, K, n, beta, mode))
    return cases


def _alg1_row_cases():
    """(shape, tile, K, beta, mode): ALG1 wave-row tiles (mode 14: 64 x 48 cells, beta = 0; 15: 64 x 32)
    whose extended region (halo K on every side) also fits the general ALG1 tiles (2048 cells)."""
    cases = []
    for shape, tile, K in [((101, 250), (12, 44), 4), ((130, 140), (10, 40), 10), ((30, 61), (30, 61), 3),
                           ((45, 200), (20, 50), 1), ((70, 300), (15, 40), 2), ((32, 64), (32, 64), 6),
                           ((2, 67), (2, 40), 2), ((67, 2), (20, 2), 2)]:
        eh, ew = min(shape[0], tile[0] + 2 * K), min(shape[1], tile[1] + 2 * K)
        for beta in (0.0, 0.05):
            for mode, rows in ((14, 48), (15, 32)):
                if mode == 14 and beta > 0:
                    continue
                if ew <= 64 and eh <= rows and eh * ew <= 2048:
                    cases.append((shape, tile, K, beta, mode))
    return cases


def _alg1_call(g, lin, beta, K, tile):
    return fm.alg1_tb(g, *lin, fm.Params(scheme="alg1", beta=beta), iters=K, tile_h=tile[0], tile_w=tile[1])


@pytest.mark.parametrize("shape,tile,K,beta,mode", _alg1_row_cases())
def test_alg1_row_tiles_equal_the_general_tiles(shape, tile, K, beta, mode):
    """The ALG1 wave-row tiles (one cell per lane and row, registers per row, DPP neighbours, the
    shrinking band) evaluate the general ALG1 tiles' operations in the same order: K iterations of
    the same tiles of the same state agree bit for bit, Theta included."""
    print_case("alg1 rows vs general tiles", shape=shape, tile=tile, K=K, beta=beta, mode=mode)
    rng = np.random.default_rng(zlib.crc32(repr(("alg1rows", shape, tile, K, beta)).encode()))
    st = random_pdr_state(rng, shape, beta)
    Ix, Iy, Itr, _ = random_lin(rng, shape, beta)
    u0 = f32(rng.normal(scale=3.0, size=shape))
    v0 = f32(rng.normal(scale=3.0, size=shape))
    g = {k: to_dev(v, pad=3) for k, v in st.items()}
    lin = (to_dev(Ix, 3), to_dev(Iy, 3), to_dev(Itr, 3), to_dev(u0, 3), to_dev(v0, 3))
    ref, ref_s = _alg1_call(g, lin, beta, K, tile)
    fm.set_tuning("pdr_mode", mode)
    try:
        out, out_s = _alg1_call(g, lin, beta, K, tile)
    finally:
        fm.set_tuning("pdr_mode", 0)
    keys = ["u", "v", "ub", "vb", "qb1x", "qb1y", "qb2x", "qb2y"] + (["w", "wb", "pbx", "pby"] if beta > 0 else [])
    for k in keys:
        assert torch.equal(out[k], ref[k]), k
    assert torch.equal(out_s, ref_s)


@pytest.mark.parametrize("shape,tile,K,beta,mode", [((120, 130), (28, 40), 10, 0.0, 14), ((140, 200), (30, 44), 9, 0.0, 14),
                                                    ((90, 150), (12, 40), 10, 0.05, 15), ((48, 64), (48, 64), 7, 0.0, 14)])
def test_alg1_row_tiles_match_k_oracle_steps(shape, tile, K, beta, mode):
    """ALG1 wave-row tiles whose extended regions fill every row of the shape (64 x 48 with beta = 0,
    64 x 32 with w), beyond the general tiles' capacity, against K steps of the oracle."""
    print_case("alg1 rows vs oracle", shape=shape, tile=tile, K=K, beta=beta, mode=mode)
    rng = np.random.default_rng(zlib.crc32(repr(("alg1rowsor", shape, tile, K, beta)).encode()))
    st = random_pdr_state(rng, shape, beta)
    Ix, Iy, Itr, _ = random_lin(rng, shape, beta)
    u0 = f32(rng.normal(scale=3.0, size=shape))
    v0 = f32(rng.normal(scale=3.0, size=shape))
    g = {k: to_dev(v, pad=3) for k, v in st.items()}
    lin = (to_dev(Ix, 3), to_dev(Iy, 3), to_dev(Itr, 3), to_dev(u0, 3), to_dev(v0, 3))
    fm.set_tuning("pdr_mode", mode)
    try:
        out, s_out = _alg1_call(g, lin, beta, K, tile)
    finally:
        fm.set_tuning("pdr_mode", 0)
    L = dict(Ix=Ix, Iy=Iy, It=Itr - Ix * u0 - Iy * v0)
    ref = dict(st)
    for _ in range(K):
        ref, duals = schemes.alg1_step(ref, L, beta, 0.05, 0.1, 1.25)
    keys = ["u", "v", "ub", "vb", "qb1x", "qb1y", "qb2x", "qb2y"] + (["w", "wb", "pbx", "pby"] if beta > 0 else [])
    tol = 1e-4 * max(1, K)
    for k in keys:
        assert max_abs(to_np(out[k]), ref[k]) < tol, (k, max_abs(to_np(out[k]), ref[k]))
    assert max_abs(to_np(s_out), duals["s"]) < tol


@pytest.mark.parametrize("shape,tile,K,sweeps,beta,mode", _pdr_row_cases())
def test_pdr_row_tiles_equal_the_general_tiles(shape, tile, K, sweeps, beta, mode):
    """The wave-row pDR tiles (cell pairs per lane, registers per row, DPP neighbours) evaluate the
    general pDR tiles' operations in the same order: K iterations of the same tiles of the same state
    agree bit for bit (with w, modes 13 and 14 run the 128 x 32 and 64 x 32 shapes)."""
    print_case("pdr rows vs general tiles", shape=shape, tile=tile, K=K, sweeps=sweeps, beta=beta, mode=mode)
    rng = np.random.default_rng(zlib.crc32(repr(("pdrrows", shape, tile, K, sweeps, beta)).encode()))
    st = random_pdr_state(rng, shape, beta)
    Ix, Iy, Itr, _ = random_lin(rng, shape, beta)
    u0 = f32(rng.normal(scale=3.0, size=shape))
    v0 = f32(rng.normal(scale=3.0, size=shape))
    g = {k: to_dev(v, pad=3) for k, v in st.items()}
    lin = (to_dev(Ix, 3), to_dev(Iy, 3), to_dev(Itr, 3), to_dev(u0, 3), to_dev(v0, 3))
    p = fm.Params(scheme="pdr", beta=beta, gs_sweeps=sweeps)
    ref = fm.pdr_tb(g, *lin, p, iters=K, tile_h=tile[0], tile_w=tile[1])
    fm.set_tuning("pdr_mode", mode)
    try:
        out = fm.pdr_tb(g, *lin, p, iters=K, tile_h=tile[0], tile_w=tile[1])
    finally:
        fm.set_tuning("pdr_mode", 0)
    keys = ["u", "v", "ub", "vb", "qb1x", "qb1y", "qb2x", "qb2y"] + (["w", "wb", "pbx", "pby"] if beta > 0 else [])
    for k in keys:
        assert torch.equal(out[0][k], ref[0][k]), k
    assert torch.equal(out[1], ref[1])


@pytest.mark.parametrize("shape,tile,K", [((7, 5), (7, 5), 9), ((37, 130), (8, 30), 4), ((101, 250), (12, 20), 1),
                                          ((40, 45), (40, 45), 20), ((64, 64), (10, 18), 6), ((33, 47), (5, 9), 3)])
@pytest.mark.parametrize("beta", [0.0, 0.05])
def test_alg1_tiles_match_k_oracle_steps(shape, tile, K, beta):
    """K ALG1 iterations of its tile kernel (halo K on each side, ragged tiles, a resident level)
    against K steps of the oracle on the same state, I_t relative to (u0, v0)."""
    print_case("alg1_tb", shape=shape, tile=tile, K=K, beta=beta)
    oversized = min(shape[0], tile[0] + 2 * K) * min(shape[1], tile[1] + 2 * K) > 2048
    rng = np.random.default_rng(zlib.crc32(repr(("alg1tb", shape, tile, K, beta)).encode()))
    st = random_pdr_state(rng, shape, beta)
    Ix, Iy, Itr, _ = random_lin(rng, shape, beta)
    u0 = f32(rng.normal(scale=3.0, size=shape))
    v0 = f32(rng.normal(scale=3.0, size=shape))
    g = {k: to_dev(v, pad=3) for k, v in st.items()}

    def call():
        return fm.alg1_tb(g, to_dev(Ix, 3), to_dev(Iy, 3), to_dev(Itr, 3), to_dev(u0, 3), to_dev(v0, 3),
                          fm.Params(scheme="alg1", beta=beta), iters=K, tile_h=tile[0], tile_w=tile[1])
    if oversized:                                    # refused before any launch
        with pytest.raises(fm.FlowError, match="capacity") as e:
            call()
        assert e.value.status == fm.FLOW_E_INVAL
        return
    L = dict(Ix=Ix, Iy=Iy, It=Itr - Ix * u0 - Iy * v0)
    ref = dict(st)
    for _ in range(K):
        ref, duals = schemes.alg1_step(ref, L, beta, 0.05, 0.1, 1.25)
    out, s_out = call()
    keys = ["u", "v", "ub", "vb", "qb1x", "qb1y", "qb2x", "qb2y"] + (["w", "wb", "pbx", "pby"] if beta > 0 else [])
    tol = 1e-4 * max(1, K)
    for k in keys:
        assert max_abs(to_np(out[k]), ref[k]) < tol, (k, max_abs(to_np(out[k]), ref[k]))
    assert max_abs(to_np(s_out), duals["s"]) < tol


@pytest.mark.parametrize("shape", [(2, 2), (70, 130), (240, 320)])
@pytest.mark.parametrize("beta", [0.0, 0.05])
def test_energy_terms(shape, beta):
    print_case("energy", shape=shape, beta=beta)
    rng = np.random.default_rng(5)
    st = random_admm_state(rng, shape, beta)
    Ix, Iy, It, _ = random_lin(rng, shape, beta)
    g = _dev_state(st, pad=2)
    r = fm.energy(g, to_dev(Ix, 2), to_dev(Iy, 2), to_dev(It, 2), lam=0.05, beta=beta)
    t = energy.terms(st["u"], st["v"], st["w"], st["px"], st["py"], st["q1x"], st["q1y"], st["q2x"], st["q2y"],
                     st["s"], Ix, Iy, It, beta, 0.05)
    for k in ("energy", "dual", "gap", "residual", "tv", "data"):
        scale = max(1.0, abs(t["energy"]), abs(t["dual"]))
        assert abs(r[k] - t[k]) <= 1e-5 * scale, (k, r[k], t[k])


@pytest.mark.parametrize("shape", [(3, 5), (70, 130), (240, 320)])
@pytest.mark.parametrize("scheme,relax,beta", [("padmm", 1.0, 0.0), ("rpadmm2", 1.9, 0.05)])
def test_admm_iteration_increment_form(shape, scheme, relax, beta):
    """The solver's increment form: multipliers u0 + du with I_t relative to (u0, v0) give the same
    iterate as the absolute form (the oracle step on u = u0 + du, I_t = I_t' - I_x u0 - I_y v0)."""
    print_case("admm_iter_increment", shape=shape, scheme=scheme, relax=relax, beta=beta)
    rng = np.random.default_rng(zlib.crc32(repr(("inc", shape, scheme)).encode()))
    st = random_admm_state(rng, shape, beta)
    Ix, Iy, Itr, at = random_lin(rng, shape, beta)
    u0 = f32(rng.normal(scale=6.0, size=shape))
    v0 = f32(rng.normal(scale=6.0, size=shape))
    du = f32(rng.normal(scale=0.3, size=shape))
    dv = f32(rng.normal(scale=0.3, size=shape))
    full = dict(st, u=u0 + du, v=v0 + dv)
    L = dict(Ix=Ix, Iy=Iy, It=Itr - Ix * u0 - Iy * v0, at=at)
    if scheme == "padmm":
        ref = schemes.rpadmm1_step(full, L, beta, 0.05, 0.05, relax)
    else:
        ref = schemes.rpadmm2_step(full, L, beta, 0.05, 0.05, relax)
    g = _dev_state(dict(st, u=du, v=dv, u0=u0, v0=v0), pad=3)
    at_t = torch.tensor([at], dtype=torch.float32, device="cuda")
    out = fm.admm_iter(g, to_dev(Ix, 3), to_dev(Iy, 3), to_dev(Itr, 3), at_t, fm.Params(scheme=scheme, relax=relax,
                                                                                        beta=beta))
    assert max_abs(to_np(out["u"]), ref["u"] - u0) < 1e-4
    assert max_abs(to_np(out["v"]), ref["v"] - v0) < 1e-4
    for k in ("q1x", "q1y", "q2x", "q2y", "s"):
        assert max_abs(to_np(out[k]), ref[k]) < 1e-4, k


def _ulps(a, b):
    """Distance in units in the last place between float32 arrays (the order-preserving integer
    image of each value's bits)."""
    def key(x):
        i = np.ascontiguousarray(x, dtype=np.float32).view(np.int32).astype(np.int64)
        return np.where(i < 0, -(i & 0x7FFFFFFF), i)
    return np.abs(key(a) - key(b))


@pytest.mark.parametrize("threads", [1025, 1026, 256, 3073])
@pytest.mark.parametrize("beta", [0.0, 0.05])
def test_tiles_and_one_pass_iterations_agree_to_the_ulp(threads, beta):
    """K = 6 iterations of a tile kernel against 6 one-pass iterations from the same increment-form
    state: the two kernels evaluate the same expressions in their own order, so they may differ by
    rounding only.  Per field, the largest difference is measured in units of the FP32 spacing at the
    field's magnitude (its largest value) and bounded by 16 (measured: at most 7.5, in p_x with beta >
    0); the ulps of the values above a tenth of that magnitude are printed beside it (at most 34)."""
    shape, K = (70, 90), 6
    print_case("tile vs one-pass", threads=threads, beta=beta)
    rng = np.random.default_rng(zlib.crc32(repr(("ulp", threads, beta)).encode()))
    st = random_admm_state(rng, shape, beta)
    Ix, Iy, Itr, at = random_lin(rng, shape, beta)
    u0 = f32(rng.normal(scale=4.0, size=shape))
    v0 = f32(rng.normal(scale=4.0, size=shape))
    du = f32(rng.normal(scale=0.3, size=shape))
    dv = f32(rng.normal(scale=0.3, size=shape))
    init = dict(st, u=du, v=dv, u0=u0, v0=v0)
    at_t = torch.tensor([at, 0.0], dtype=torch.float32, device="cuda")
    p = fm.Params(beta=beta)
    lin = (to_dev(Ix, 2), to_dev(Iy, 2), to_dev(Itr, 2))
    tile = fm.admm_tb(_dev_state(init, pad=2), *lin, at_t, p, iters=K, threads=threads, tile_h=12, tile_w=20, order=0)
    g = _dev_state(init, pad=2)
    for _ in range(K):
        out = fm.admm_iter(g, *lin, at_t[:1], p)
        g = dict(g, **{k: v for k, v in out.items() if v is not None})
    keys = ["u", "v", "q1x", "q1y", "q2x", "q2y", "s"] + (["w", "px", "py"] if beta > 0 else [])
    spacings, ulps = {}, {}
    for k in keys:
        a, b = to_np(tile[k]), to_np(g[k])
        scale = float(np.abs(b).max())
        spacings[k] = round(float(np.abs(a - b).max() / np.spacing(np.float32(scale))), 2)
        large = np.abs(b) >= 0.1 * scale
        ulps[k] = int(_ulps(a, b)[large].max())
    print(f"[ulps] threads {threads} beta {beta}: max difference in spacings at each field's magnitude "
          f"{spacings}; ulps of values above a tenth of it {ulps}", flush=True)
    assert max(spacings.values()) <= 16, spacings


@pytest.mark.parametrize("rows", [2, 4, 8])
@pytest.mark.parametrize("shape", [(7, 5), (37, 130), (101, 250)])
@pytest.mark.parametrize("beta", [0.0, 0.05])
def test_admm_iteration_every_strip_height(rows, shape, beta):
    """Each compiled strip height R, on row counts that leave a ragged last strip."""
    print_case("admm_rows", rows=rows, shape=shape, beta=beta)
    rng = np.random.default_rng(rows * 1000 + shape[0])
    st = random_admm_state(rng, shape, beta)
    Ix, Iy, It, at = random_lin(rng, shape, beta)
    ref = schemes.rpadmm1_step(st, dict(Ix=Ix, Iy=Iy, It=It, at=at), beta, 0.05, 0.05, 1.0)
    fm.set_tuning("admm_rows", rows)
    try:
        out = fm.admm_iter(_dev_state(st, pad=1), to_dev(Ix, 1), to_dev(Iy, 1), to_dev(It, 1),
                           torch.tensor([at], dtype=torch.float32, device="cuda"), fm.Params(beta=beta))
        torch.cuda.synchronize()
    finally:
        fm.set_tuning("admm_rows", 0)
    for k in ["u", "v", "q1x", "q1y", "q2x", "q2y", "s"] + (["w", "px", "py"] if beta > 0 else []):
        assert max_abs(to_np(out[k]), ref[k]) < 1e-4, k


@pytest.mark.parametrize("shape,tile,K", [((7, 5), (7, 5), 6), ((37, 130), (8, 30), 3), ((101, 250), (12, 20), 4),
                                          ((60, 80), (60, 80), 9), ((64, 64), (10, 18), 1), ((33, 47), (33, 47), 20)])
@pytest.mark.parametrize("threads,order", [(256, 0), (1024, 0), (1025, 0), (256, 1), (1024, 1), (1025, 2),
                                           (1025, 3), (256, 2), (513, 0), (257, 0), (1026, 0), (514, 0),
                                           (2049, 0), (3073, 0), (3073, 3), (4097, 0)])
@pytest.mark.parametrize("scheme,relax,beta", [("padmm", 1.0, 0.0), ("rpadmm2", 1.9, 0.05)])
def test_admm_tiles_match_k_oracle_steps(shape, tile, K, threads, order, scheme, relax, beta):
    """K iterations of the temporally blocked tile kernel (halo K + 1 / K, ragged tiles, resident
    levels) against K steps of the oracle on the same increment-form state; a tile whose extended
    region exceeds the kernel's capacity is refused before any launch."""
    print_case("admm_tb", shape=shape, tile=tile, K=K, threads=threads, order=order, scheme=scheme, beta=beta)
    eh, ew = min(shape[0], tile[0] + 2 * K + 1), min(shape[1], tile[1] + 2 * K + 1)
    if threads in ROW_CODES:                         # wave-row tiles: at most 64 columns, (code - 1) / 64 rows
        oversized = ew > 64 or eh * 64 > threads - 1
    else:
        cap = {1025: 2048, 513: 1024, 257: 512, 1026: 1024, 514: 512}.get(threads) or (
            1024 * (3 if beta > 0 else 4) if threads == 1024 else 256 * (4 if beta > 0 else 6))
        oversized = eh * ew > cap
    rng = np.random.default_rng(zlib.crc32(repr(("tb", shape, tile, K, threads, scheme)).encode()))
    st = random_admm_state(rng, shape, beta)
    Ix, Iy, Itr, at = random_lin(rng, shape, beta)
    u0 = f32(rng.normal(scale=4.0, size=shape))
    v0 = f32(rng.normal(scale=4.0, size=shape))
    du = f32(rng.normal(scale=0.3, size=shape))
    dv = f32(rng.normal(scale=0.3, size=shape))
    g = _dev_state(dict(st, u=du, v=dv, u0=u0, v0=v0), pad=2)
    at_t = torch.tensor([at, 0.0], dtype=torch.float32, device="cuda")

    def call():
        return fm.admm_tb(g, to_dev(Ix, 2), to_dev(Iy, 2), to_dev(Itr, 2), at_t,
                          fm.Params(scheme=scheme, relax=relax, beta=beta), iters=K, threads=threads,
                          tile_h=tile[0], tile_w=tile[1], order=order)
    if oversized:                                    # refused before any launch
        with pytest.raises(fm.FlowError, match="capacity") as e:
            call()
        assert e.value.status == fm.FLOW_E_INVAL
        return
    full = dict(st, u=u0 + du, v=v0 + dv)
    L = dict(Ix=Ix, Iy=Iy, It=Itr - Ix * u0 - Iy * v0, at=at)
    for _ in range(K):
        full = (schemes.rpadmm1_step(full, L, beta, 0.05, 0.05, relax) if scheme == "padmm"
                else schemes.rpadmm2_step(full, L, beta, 0.05, 0.05, relax))
    out = call()
    tol = 1e-4 * max(1, K)
    assert max_abs(to_np(out["u"]), full["u"] - u0) < tol
    assert max_abs(to_np(out["v"]), full["v"] - v0) < tol
    for k in ["q1x", "q1y", "q2x", "q2y", "s"] + (["w", "px", "py"] if beta > 0 else []):
        assert max_abs(to_np(out[k]), full[k]) < tol, k


def _row_cases():
    """(shape, tile, K, code) with the tile's extended region within the wave-row shape."""
    cases = []
    for shape, tile, K in [((101, 250), (12, 20), 4), ((300, 200), (27, 53), 5), ((96, 130), (17, 43), 10),
                           ((45, 64), (45, 64), 7), ((70, 33), (20, 33), 3)]:
        eh, ew = min(shape[0], tile[0] + 2 * K + 1), min(shape[1], tile[1] + 2 * K + 1)
        cases += [(shape, tile, K, nt) for nt in ROW_CODES if ew <= 64 and eh * 64 <= nt - 1]
    return cases


@pytest.mark.parametrize("shape,tile,K,threads", _row_cases())
@pytest.mark.parametrize("beta", [0.0, 0.05])
def test_row_tiles_equal_the_general_tiles(shape, tile, K, threads, beta):
    """The wave-row tiles (registers per row, DPP neighbours) evaluate the general tile kernel's
    operations in the same order: the same tiles give bitwise the same iterates, in direct and in
    table order."""
    print_case("rows vs general tiles", shape=shape, tile=tile, K=K, threads=threads, beta=beta)
    eh, ew = min(shape[0], tile[0] + 2 * K + 1), min(shape[1], tile[1] + 2 * K + 1)
    rng = np.random.default_rng(zlib.crc32(repr(("rows", shape, tile, K, threads, beta)).encode()))
    st = random_admm_state(rng, shape, beta)
    Ix, Iy, Itr, at = random_lin(rng, shape, beta)
    init = dict(st, u=f32(rng.normal(scale=0.3, size=shape)), v=f32(rng.normal(scale=0.3, size=shape)),
                u0=f32(rng.normal(scale=4.0, size=shape)), v0=f32(rng.normal(scale=4.0, size=shape)))
    at_t = torch.tensor([at, 0.0], dtype=torch.float32, device="cuda")
    lin = (to_dev(Ix, 2), to_dev(Iy, 2), to_dev(Itr, 2))
    p = fm.Params(beta=beta)
    ref = fm.admm_tb(_dev_state(init, pad=2), *lin, at_t, p, iters=K, threads=1025 if eh * ew <= 2048 else 1024,
                     tile_h=tile[0], tile_w=tile[1], order=0)
    keys = ["u", "v", "q1x", "q1y", "q2x", "q2y", "s"] + (["w", "px", "py"] if beta > 0 else [])
    for order in (0, 3):
        out = fm.admm_tb(_dev_state(init, pad=2), *lin, at_t, p, iters=K, threads=threads, tile_h=tile[0],
                         tile_w=tile[1], order=order)
        for k in keys:
            assert np.array_equal(to_np(out[k]), to_np(ref[k])), (order, k)
