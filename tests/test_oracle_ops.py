"""Pins of the oracle's operators against the mathematics (no GPU).

Each check is written so that a plausible slip (sign, boundary row, transposed axis, separate
instead of joint projection, swapped resolvent case) fails it.
"""
import json
import os

import numpy as np
import pytest
import scipy.ndimage
import scipy.optimize
import scipy.sparse
import scipy.sparse.csgraph

from oracle import ops

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SHAPES = [(2, 2), (2, 7), (7, 2), (3, 3), (5, 8), (17, 13), (64, 48)]


def check_adjoint(grad, div, shape, seed=0):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=shape)
    px, py = rng.normal(size=shape), rng.normal(size=shape)
    gx, gy = grad(u)
    lhs = float((gx * px + gy * py).sum())
    rhs = -float((u * div(px, py)).sum())
    scale = float(np.abs(gx * px).sum() + np.abs(gy * py).sum() + np.abs(u * div(px, py)).sum())
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)


@pytest.mark.parametrize("shape", SHAPES)
def test_adjoint_identity(shape):
    """<grad u, p>_Y = -<u, div p>_X (Sec. 2.2) on random FP64 arrays."""
    check_adjoint(ops.grad, ops.div, shape, seed=shape[0] * 100 + shape[1])


def test_hand_worked_grad_div():
    g = json.load(open(os.path.join(GOLD, "grad_div_3x3.json")))
    f = np.array(g["f"], float)
    gx, gy = ops.grad(f)
    np.testing.assert_array_equal(gx, g["grad_x"])
    np.testing.assert_array_equal(gy, g["grad_y"])
    d = ops.div(np.array(g["px"], float), np.array(g["py"], float))
    np.testing.assert_array_equal(d, g["div_p"])
    assert float((gx * np.array(g["px"]) + gy * np.array(g["py"])).sum()) == g["inner_grad_f_p"]
    np.testing.assert_array_equal(ops.laplacian(f), g["laplacian_f"])


def test_divergence_sums_to_zero():
    rng = np.random.default_rng(3)
    for shape in SHAPES:
        d = ops.div(rng.normal(size=shape), rng.normal(size=shape))
        assert abs(d.sum()) < 1e-11


def grid_graph_laplacian(M, N):
    """L = D - A of the 4-neighbour grid graph, via scipy's csgraph (an independent routine)."""
    idx = np.arange(M * N).reshape(M, N)
    rows = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    cols = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    A = scipy.sparse.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(M * N, M * N))
    A = (A + A.T).tocsr()
    return scipy.sparse.csgraph.laplacian(A).toarray()


@pytest.mark.parametrize("shape", [(2, 2), (3, 5), (6, 4), (9, 9)])
def test_laplacian_is_neumann_graph_laplacian(shape):
    """div o grad is minus the grid graph Laplacian, i.e. the 5-point Neumann Laplacian."""
    M, N = shape
    Lg = grid_graph_laplacian(M, N)
    rng = np.random.default_rng(1)
    f = rng.normal(size=shape)
    np.testing.assert_allclose(ops.laplacian(f).ravel(), -(Lg @ f.ravel()), rtol=0, atol=1e-12)


def test_grad_gradstar_norm_at_most_8():
    """||grad grad^*|| <= 8 (the bound behind a = 8, eq:stepsize:constraint / Prop. 3.1)."""
    rng = np.random.default_rng(2)
    for shape in [(4, 4), (16, 16), (33, 20)]:
        px, py = rng.normal(size=shape), rng.normal(size=shape)
        lam = 0.0
        for _ in range(400):
            n = np.sqrt((px * px + py * py).sum())
            px, py = px / n, py / n
            px, py = ops.grad_gradstar(px, py)
            lam = np.sqrt((px * px + py * py).sum())
        assert lam <= 8.0 + 1e-9
        if shape == (33, 20):
            assert lam > 7.5       # the bound is nearly attained on larger grids


def test_grad_gradstar_is_psd():
    rng = np.random.default_rng(4)
    px, py = rng.normal(size=(9, 7)), rng.normal(size=(9, 7))
    gx, gy = ops.grad_gradstar(px, py)
    assert float((gx * px + gy * py).sum()) >= 0.0
    # <z, grad grad^* z> = ||div z||^2
    assert np.isclose(float((gx * px + gy * py).sum()), float((ops.div(px, py) ** 2).sum()), rtol=1e-12)


# --- projections ---------------------------------------------------------------------------------
def _rand_vectors(rng, n, k, scale=2.0):
    return [rng.normal(size=n) * scale for _ in range(k)]


def test_proj_p_feasible_idempotent_nearest():
    rng = np.random.default_rng(5)
    px, py = _rand_vectors(rng, 500, 2)
    qx, qy = ops.proj_p(px, py)
    assert np.all(ops.norm_p(qx, qy) <= 1 + 1e-15)
    rx, ry = ops.proj_p(qx, qy)
    np.testing.assert_allclose(rx, qx, rtol=0, atol=4 * np.finfo(float).eps)
    np.testing.assert_allclose(ry, qy, rtol=0, atol=4 * np.finfo(float).eps)
    # brute force: no sampled point of the unit disc is nearer than the projection
    ang = rng.uniform(0, 2 * np.pi, 4000)
    rad = np.sqrt(rng.uniform(0, 1, 4000))
    cx, cy = rad * np.cos(ang), rad * np.sin(ang)
    for k in range(50):
        dproj = np.hypot(px[k] - qx[k], py[k] - qy[k])
        dmin = np.min(np.hypot(px[k] - cx, py[k] - cy))
        assert dproj <= dmin + 1e-12


def test_proj_q_joint_feasible_idempotent_nearest():
    rng = np.random.default_rng(6)
    q = _rand_vectors(rng, 400, 4)
    pq = ops.proj_q(*q)
    assert np.all(ops.norm_q(*pq) <= 1 + 1e-15)
    ppq = ops.proj_q(*pq)
    for a, b in zip(ppq, pq):
        np.testing.assert_allclose(a, b, rtol=0, atol=4 * np.finfo(float).eps)
    samples = rng.normal(size=(4, 6000))
    samples /= np.maximum(1.0, np.linalg.norm(samples, axis=0)) * (1 + 1e-12)
    samples *= rng.uniform(0, 1, 6000) ** 0.25
    for k in range(40):
        x = np.array([c[k] for c in q])
        p = np.array([c[k] for c in pq])
        assert np.linalg.norm(x - p) <= np.min(np.linalg.norm(samples - x[:, None], axis=0)) + 1e-12


def test_proj_q_is_joint_not_two_discs():
    """|q| couples all four components (eq:euclid:norm): two halves inside their discs can still
    need scaling."""
    q = [np.array([0.6]), np.array([0.6]), np.array([0.6]), np.array([0.6])]   # |q1| = |q2| = 0.85, |q| = 1.2
    out = ops.proj_q(*q)
    np.testing.assert_allclose([o[0] for o in out], [0.5] * 4, rtol=1e-15)


def test_proj_s_is_clamp():
    s = np.array([-1.0, -0.05, -0.01, 0.0, 0.03, 0.05, 2.0])
    np.testing.assert_array_equal(ops.proj_s(s, 0.05), [-0.05, -0.05, -0.01, 0.0, 0.03, 0.05, 0.05])


# --- bilinear sampling ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(2, 2), (5, 9), (31, 17)])
def test_bilinear_matches_scipy_linear_interpolation(shape):
    rng = np.random.default_rng(7)
    F = rng.normal(size=shape)
    M, N = shape
    y = rng.uniform(-3, M + 2, 2000)
    x = rng.uniform(-3, N + 2, 2000)
    ref = scipy.ndimage.map_coordinates(F, [np.clip(y, 0, M - 1), np.clip(x, 0, N - 1)], order=1, mode="nearest")
    np.testing.assert_allclose(ops.bilinear(F, y, x), ref, rtol=0, atol=1e-12)


def test_bilinear_exact_at_nodes_and_edges():
    F = np.arange(12.0).reshape(3, 4)
    ii, jj = np.indices(F.shape)
    np.testing.assert_array_equal(ops.bilinear(F, ii.astype(float), jj.astype(float)), F)
    assert ops.bilinear(F, np.array([10.0]), np.array([-5.0]))[0] == F[2, 0]


# --- resolvent -----------------------------------------------------------------------------------
def test_resolvent_hand_cases():
    g = json.load(open(os.path.join(GOLD, "resolvent_cases.json")))
    for c in g["cases"]:
        a = lambda k: np.array([c[k]], float)  # noqa: E731
        w, u, v, _ = ops.resolvent(a("w"), a("u"), a("v"), a("Ix"), a("Iy"), a("It"), c["beta"],
                                   g["lambda"], g["sigma"])
        np.testing.assert_allclose([w[0], u[0], v[0]], [c["expect_w"], c["expect_u"], c["expect_v"]],
                                   rtol=0, atol=1e-14, err_msg=c["name"])


def test_resolvent_is_the_prox_brute_force():
    """argmin_X lambda|rho(X)| + |X - X~|^2 / (2 sigma), minimised numerically per pixel."""
    rng = np.random.default_rng(8)
    sigma, lam = 2.0, 0.05
    for k in range(60):
        beta = [0.0, 0.05, 0.5][k % 3]
        Ix, Iy, It = rng.normal(0, 3), rng.normal(0, 3), rng.normal(0, 2)
        wt, ut, vt = rng.normal(size=3)
        w, u, v, _ = ops.resolvent(np.array(wt), np.array(ut), np.array(vt), np.array(Ix),
                                   np.array(Iy), np.array(It), beta, lam, sigma)
        e = np.array([beta, Ix, Iy])
        xt = np.array([wt, ut, vt])

        def obj(x):
            return lam * abs(It + e @ x) + ((x - xt) ** 2).sum() / (2 * sigma)
        # the minimiser lies on xt + t e; search t by bounded scalar minimisation, then polish in 3-D
        r = scipy.optimize.minimize_scalar(lambda t: obj(xt + t * e), bounds=(-50, 50), method="bounded",
                                           options=dict(xatol=1e-13))
        xs = xt + r.x * e
        r3 = scipy.optimize.minimize(obj, xs, method="Nelder-Mead",
                                     options=dict(xatol=1e-13, fatol=1e-16, maxiter=20000))
        best = r3.x if r3.fun < obj(xs) else xs
        got = np.array([float(w), float(u), float(v)])
        assert obj(got) <= obj(best) + 1e-12
        np.testing.assert_allclose(got, best, atol=5e-6)


def test_resolvent_continuous_at_thresholds():
    sigma, lam, Ix, Iy = 2.0, 0.05, 1.5, -0.5
    e2 = Ix * Ix + Iy * Iy
    thr = sigma * lam * e2
    for sgn in (1, -1):
        base = sgn * thr
        its = np.array([base - 1e-9, base, base + 1e-9])
        w, u, v, th = ops.resolvent(np.zeros(3), np.zeros(3), np.zeros(3), np.full(3, Ix), np.full(3, Iy), its,
                                    0.0, lam, sigma)
        assert np.ptp(u) < 1e-8 and np.ptp(v) < 1e-8
        assert np.allclose(np.abs(th), lam, atol=1e-8)
