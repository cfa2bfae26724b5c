"""Pins of the solver iterations (no GPU).

* the dual (y) and s steps of rpADMMI equal a numerical argmax of the preconditioned augmented
  Lagrangian (eq:aug:pre1:vector, with the objective of eq:dual:optic) on tiny grids;
* scheme algebra: rpADMMII(rho = 1) = rpADMMI(r = 1); Zach-pADMM = rpADMMI(beta = 0, r = 1);
* SRBGS is a symmetric, feasible preconditioner (M >= T, Sec. 3.1.2) and converges to the solve;
* convergence statements (Prop. 3.1, Prop. 3.2): gap and residual fall towards zero and every
  scheme reaches the same minimum energy;
* the gap decomposition E - D = G_TV + G_data + <Lambda, r> holds for arbitrary states.
"""
import numpy as np
import pytest
import scipy.optimize

import synth
from oracle import ops, schemes, energy
from oracle.solve import Params, zeros_admm, zeros_pdr, step
from oracle.pyramid import build_pyramid, linearize


def random_state(rng, shape, beta):
    st = {k: rng.normal(scale=0.4, size=shape) for k in ("w", "u", "v", "px", "py", "q1x", "q1y", "q2x", "q2y")}
    st["s"] = rng.uniform(-0.05, 0.05, size=shape)
    if beta == 0.0:
        st["w"][:] = 0.0
        st["px"][:] = 0.0
        st["py"][:] = 0.0
    return st


def random_lin(rng, shape, beta):
    Ix, Iy, It = rng.normal(0, 3, shape), rng.normal(0, 3, shape), rng.normal(0, 2, shape)
    at = float(np.max(beta * beta + Ix * Ix + Iy * Iy))
    return dict(Ix=Ix, Iy=Iy, It=It, at=at)


def residual_blocks(s, ys, L, beta):
    """A s + B y = (beta s - div p, I_x s - div q1, I_y s - div q2)."""
    px, py, q1x, q1y, q2x, q2y = ys
    return (beta * s - ops.div(px, py), L["Ix"] * s - ops.div(q1x, q1y), L["Iy"] * s - ops.div(q2x, q2y))


def lagrangian(st, s, ys, L, beta, c):
    """L_c of eq:dual:optic without its indicator terms (the constraint sets are imposed separately)."""
    r = residual_blocks(s, ys, L, beta)
    lam_r = sum(float((m * x).sum()) for m, x in zip((st["w"], st["u"], st["v"]), r))
    return float((L["It"] * s).sum()) + lam_r - 0.5 * c * sum(float((x * x).sum()) for x in r)


@pytest.mark.parametrize("beta", [0.0, 0.3])
def test_y_step_is_preconditioned_argmax(beta):
    """p+, q+ of rpADMMI maximise L_c(Lambda; y, s) - 1/2 |y - y^k|^2_{acI - c grad grad^*} over
    |p_ij| <= 1, |q_ij| <= 1 (eq:aug:pre1:vector, first line)."""
    rng = np.random.default_rng(11)
    shape, c, a = (3, 3), 0.05, 8.0
    st = random_state(rng, shape, beta)
    L = random_lin(rng, shape, beta)
    new = schemes.rpadmm1_step(st, L, beta, 0.05, c, 1.0)
    n = 9
    yk = [st[k] for k in ("px", "py", "q1x", "q1y", "q2x", "q2y")]

    def unpack(z):
        return [z[i * n:(i + 1) * n].reshape(shape) for i in range(6)]

    def neg_obj(z):
        ys = unpack(z)
        d = [y - y0 for y, y0 in zip(ys, yk)]
        # |z|^2_{acI - c grad grad^*} = ac |z|^2 - c |div z|^2 per block
        prox = a * c * sum(float((x * x).sum()) for x in d)
        prox -= c * sum(float((ops.div(d[2 * b], d[2 * b + 1]) ** 2).sum()) for b in range(3))
        return -(lagrangian(st, st["s"], ys, L, beta, c) - 0.5 * prox)

    cons = []
    for k in range(n):
        cons.append(dict(type="ineq", fun=lambda z, k=k: 1.0 - z[k] ** 2 - z[n + k] ** 2))
        cons.append(dict(type="ineq", fun=lambda z, k=k: 1.0 - sum(z[(2 + b) * n + k] ** 2 for b in range(4))))
    z0 = np.concatenate([np.clip(y, -0.4, 0.4).ravel() for y in yk])
    res = scipy.optimize.minimize(neg_obj, z0, method="SLSQP", constraints=cons,
                                  options=dict(ftol=1e-15, maxiter=2000))
    got = np.concatenate([new[k].ravel() for k in ("px", "py", "q1x", "q1y", "q2x", "q2y")])
    assert neg_obj(got) <= res.fun + 1e-9
    if beta == 0.0:   # the p block is not coupled to anything: only q is compared
        got, ref = got[2 * n:], res.x[2 * n:]
    else:
        ref = res.x
    np.testing.assert_allclose(got, ref, atol=2e-5)


@pytest.mark.parametrize("beta", [0.0, 0.3])
def test_s_step_is_preconditioned_argmax(beta):
    """s+ of rpADMMI maximises L_c(Lambda; y+, s) - 1/2 |s - s^k|^2_{a~cI - cM_s} over |s| <= lambda
    (eq:aug:pre1:vector, second line; the indicator bound is lambda, as in eq:ofc-dual)."""
    rng = np.random.default_rng(12)
    shape, c, lam = (4, 3), 0.05, 0.05
    st = random_state(rng, shape, beta)
    L = random_lin(rng, shape, beta)
    new = schemes.rpadmm1_step(st, L, beta, lam, c, 1.0)
    ys = [new[k] for k in ("px", "py", "q1x", "q1y", "q2x", "q2y")]
    Ms = beta * beta + L["Ix"] ** 2 + L["Iy"] ** 2

    def neg_obj(z):
        s = z.reshape(shape)
        prox = float(((L["at"] * c - c * Ms) * (s - st["s"]) ** 2).sum())
        return -(lagrangian(st, s, ys, L, beta, c) - 0.5 * prox)

    res = scipy.optimize.minimize(neg_obj, np.zeros(12), method="L-BFGS-B", bounds=[(-lam, lam)] * 12,
                                  options=dict(ftol=1e-16, gtol=1e-12, maxiter=5000))
    assert neg_obj(new["s"].ravel()) <= res.fun + 1e-10
    np.testing.assert_allclose(new["s"].ravel(), res.x, atol=1e-6)


def test_rpadmm2_at_rho_1_is_rpadmm1_at_r_1():
    rng = np.random.default_rng(13)
    st = random_state(rng, (7, 9), 0.2)
    L = random_lin(rng, (7, 9), 0.2)
    a = schemes.rpadmm1_step(st, L, 0.2, 0.05, 0.05, 1.0)
    b = schemes.rpadmm2_step(st, L, 0.2, 0.05, 0.05, 1.0)
    for k in a:
        np.testing.assert_allclose(a[k], b[k], rtol=0, atol=1e-13, err_msg=k)


def test_zach_is_rpadmm1_with_beta_0():
    rng = np.random.default_rng(14)
    st = random_state(rng, (6, 5), 0.0)
    L = random_lin(rng, (6, 5), 0.0)
    a = schemes.rpadmm1_step(st, L, 0.0, 0.05, 0.05, 1.0)
    b = schemes.zach_padmm_step(st, L, 0.05, 0.05)
    for k in ("q1x", "q1y", "q2x", "q2y", "s", "u", "v"):
        np.testing.assert_allclose(a[k], b[k], rtol=0, atol=1e-13, err_msg=k)
    for k in ("w", "px", "py"):
        assert np.all(a[k] == 0.0)


def test_relaxation_changes_only_the_multipliers():
    """rpADMMI's r enters only the multiplier update (eq:aug:pre1:vector, third line)."""
    rng = np.random.default_rng(15)
    st = random_state(rng, (5, 6), 0.1)
    L = random_lin(rng, (5, 6), 0.1)
    a = schemes.rpadmm1_step(st, L, 0.1, 0.05, 0.05, 1.0)
    b = schemes.rpadmm1_step(st, L, 0.1, 0.05, 0.05, 1.618)
    for k in ("px", "py", "q1x", "q1y", "q2x", "q2y", "s"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_allclose(b["u"] - st["u"], 1.618 * (a["u"] - st["u"]), atol=1e-14)


# --- SRBGS ---------------------------------------------------------------------------------------
def build_T(shape, stt):
    """The matrix of T = I - st Delta, from the operator applied to unit vectors."""
    n = shape[0] * shape[1]
    T = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        T[:, k] = schemes.pdr_T(e.reshape(shape), stt).ravel()
    return T


def build_Minv(shape, stt, sweeps):
    n = shape[0] * shape[1]
    Mi = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        Mi[:, k] = schemes.srbgs(np.zeros(shape), e.reshape(shape), stt, sweeps).ravel()
    return Mi


@pytest.mark.parametrize("shape,sweeps", [((3, 4), 1), ((4, 5), 1), ((5, 5), 2), ((2, 6), 3)])
def test_srbgs_is_symmetric_feasible_preconditioner(shape, sweeps):
    stt = 2.0 * 0.4
    T = build_T(shape, stt)
    Mi = build_Minv(shape, stt, sweeps)
    np.testing.assert_allclose(Mi, Mi.T, atol=1e-13)
    # M >= T  <=>  T^{-1} - M^{-1} >= 0 for SPD T, M
    ev = np.linalg.eigvalsh(np.linalg.inv(T) - Mi)
    assert ev.min() >= -1e-12
    assert np.linalg.eigvalsh(Mi).min() > 0


def test_srbgs_one_sweep_equals_sequential_gauss_seidel():
    """One symmetric sweep = plain Gauss-Seidel on the matrix T visiting red cells, then black,
    then black and red again in reverse order (brute force, Python loops on a tiny grid)."""
    shape, stt = (4, 5), 0.8
    T = build_T(shape, stt)
    rng = np.random.default_rng(16)
    x0, b = rng.normal(size=shape), rng.normal(size=shape)
    red = [k for k in range(20) if sum(divmod(k, 5)) % 2 == 0]
    black = [k for k in range(20) if sum(divmod(k, 5)) % 2 == 1]
    order = red + black + black[::-1] + red[::-1]
    x = x0.ravel().copy()
    bb = b.ravel()
    for k in order:
        x[k] = (bb[k] - T[k] @ x + T[k, k] * x[k]) / T[k, k]
    np.testing.assert_allclose(schemes.srbgs(x0, b, stt, 1).ravel(), x, atol=1e-13)


def test_srbgs_converges_to_linear_solve():
    shape, stt = (6, 7), 0.8
    T = build_T(shape, stt)
    rng = np.random.default_rng(17)
    b = rng.normal(size=shape)
    x = schemes.srbgs(np.zeros(shape), b, stt, 60)
    np.testing.assert_allclose(x.ravel(), np.linalg.solve(T, b.ravel()), atol=1e-11)


# --- gap identity --------------------------------------------------------------------------------
@pytest.mark.parametrize("beta", [0.0, 0.2])
def test_gap_decomposition_identity(beta):
    rng = np.random.default_rng(18)
    st = random_state(rng, (8, 9), beta)
    L = random_lin(rng, (8, 9), beta)
    t = energy.terms(st["u"], st["v"], st["w"], st["px"], st["py"], st["q1x"], st["q1y"], st["q2x"],
                     st["q2y"], st["s"], L["Ix"], L["Iy"], L["It"], beta, 0.05)
    assert np.isclose(t["gap"], t["g_tv"] + t["g_data"] + t["lam_r"], rtol=1e-12, atol=1e-10)


def test_gap_parts_nonnegative_for_feasible_duals():
    rng = np.random.default_rng(19)
    st = random_state(rng, (8, 9), 0.2)
    st["px"], st["py"] = ops.proj_p(st["px"], st["py"])
    st["q1x"], st["q1y"], st["q2x"], st["q2y"] = ops.proj_q(st["q1x"], st["q1y"], st["q2x"], st["q2y"])
    L = random_lin(rng, (8, 9), 0.2)
    t = energy.terms(st["u"], st["v"], st["w"], st["px"], st["py"], st["q1x"], st["q1y"], st["q2x"],
                     st["q2y"], st["s"], L["Ix"], L["Iy"], L["It"], 0.2, 0.05)
    assert t["g_tv"] >= 0 and t["g_data"] >= 0


# --- convergence ---------------------------------------------------------------------------------
def small_problem(beta):
    pair = synth.translation_pair(0)
    I0 = pair.I0[20:40, 18:42]
    I1 = pair.I1[20:40, 18:42]
    a, b, dx, dy = build_pyramid(I0, I1, 1)[0]
    z = np.zeros(a.shape)
    Ix, Iy, It, at = linearize(a, b, dx, dy, z, z, 255.0, beta)
    return a.shape, dict(Ix=Ix, Iy=Iy, It=It, at=at)


def run(scheme, relax, beta, iters, checkpoints):
    shape, L = small_problem(beta)
    p = Params(scheme=scheme, relax=relax, beta=beta)
    z = np.zeros(shape)
    st = zeros_pdr(shape, z, z, z) if scheme in ("pdr", "alg1") else zeros_admm(shape, z.copy(), z.copy(), z.copy())
    out = []
    for k in range(1, iters + 1):
        st, duals = step(scheme, st, L, p)
        if k in checkpoints:
            t = energy.terms(st["u"], st["v"], st["w"], duals["px"], duals["py"], duals["q1x"], duals["q1y"],
                             duals["q2x"], duals["q2y"], duals["s"], L["Ix"], L["Iy"], L["It"], beta, 0.05)
            out.append(t)
    return out


@pytest.mark.parametrize("beta", [0.0, 0.05])
def test_all_schemes_reach_the_same_minimum(beta):
    """Prop. 3.1 / 3.2: gap and feasibility residual fall towards zero; the limit is the (unique)
    minimum energy of the convex linearised problem, the same for every scheme."""
    cps = (100, 3000)
    finals = {}
    schemes_ = [("padmm", 1.0), ("padmm", 1.618), ("rpadmm2", 1.9), ("pdr", 1.0)]
    if beta == 0.0:
        schemes_.append(("zach", 1.0))
    for scheme, relax in schemes_:
        tr = run(scheme, relax, beta, 3000, cps)
        first, last = tr[0], tr[-1]
        assert abs(last["gap"]) < 0.25 * abs(first["gap"]) + 1e-9, (scheme, first["gap"], last["gap"])
        assert abs(last["gap"]) / last["energy"] < 2e-3, (scheme, last)
        assert last["residual"] < 0.05 * max(first["residual"], 1.0), (scheme, last)
        finals[(scheme, relax)] = last["energy"]
    e = np.array(list(finals.values()))
    assert np.ptp(e) / e.mean() < 2e-3, finals


# --- ALG1 (the primal-dual comparison algorithm of Sec. 4) --------------------------------------
def random_pd_state(rng, shape, beta):
    st = {k: rng.normal(scale=0.5, size=shape) for k in ("w", "u", "v", "wb", "ub", "vb")}
    for k in ("pbx", "pby", "qb1x", "qb1y", "qb2x", "qb2y"):
        st[k] = rng.uniform(-0.5, 0.5, size=shape)
    if beta == 0.0:
        for k in ("w", "wb", "pbx", "pby"):
            st[k][:] = 0.0
    return st


@pytest.mark.parametrize("beta", [0.0, 0.3])
def test_alg1_dual_step_is_the_projected_ascent(beta):
    """y+ is the nearest point of the dual set to y + tau K X bar: feasible, and the variational
    inequality <z - y+, (y + tau K X bar) - y+> <= 0 holds for feasible z."""
    rng = np.random.default_rng(31)
    shape = (6, 7)
    st = random_pd_state(rng, shape, beta)
    L = random_lin(rng, shape, beta)
    new, _ = schemes.alg1_step(st, L, beta, 0.05, 0.1, 1.25)
    tau = 0.1
    g = [ops.grad(st["ub"]), ops.grad(st["vb"])]
    a = [st["qb1x"] + tau * g[0][0], st["qb1y"] + tau * g[0][1], st["qb2x"] + tau * g[1][0], st["qb2y"] + tau * g[1][1]]
    y = [new["qb1x"], new["qb1y"], new["qb2x"], new["qb2y"]]
    assert np.all(ops.norm_q(*y) <= 1 + 1e-12)
    for _ in range(20):
        z = [rng.normal(size=shape) for _ in range(4)]
        z = list(ops.proj_q(*z))
        vi = sum(((zi - yi) * (ai - yi)).sum() for zi, yi, ai in zip(z, y, a))
        assert vi <= 1e-10
    if beta > 0:
        gw = ops.grad(st["wb"])
        assert np.all(ops.norm_p(new["pbx"], new["pby"]) <= 1 + 1e-12)
        assert np.allclose(np.hypot(*ops.proj_p(st["pbx"] + tau * gw[0], st["pby"] + tau * gw[1])),
                           np.hypot(new["pbx"], new["pby"]))


@pytest.mark.parametrize("beta", [0.0, 0.3])
def test_alg1_primal_step_is_the_proximal_descent(beta):
    """X+ minimises lambda |rho(X)| + <K X, y+> + |X - X^k|^2 / (2 sigma) (numerically, per pixel:
    <K X, y> = -<X, div y> is separable), i.e. the primal step uses K^* = -div."""
    rng = np.random.default_rng(32)
    shape = (3, 4)
    st = random_pd_state(rng, shape, beta)
    L = random_lin(rng, shape, beta)
    lam, tau, sigma = 0.05, 0.1, 1.25
    new, _ = schemes.alg1_step(st, L, beta, lam, tau, sigma)
    dq1 = ops.div(new["qb1x"], new["qb1y"])
    dq2 = ops.div(new["qb2x"], new["qb2y"])
    dp = ops.div(new["pbx"], new["pby"])
    for i in range(shape[0]):
        for j in range(shape[1]):
            x0 = np.array([st["w"][i, j], st["u"][i, j], st["v"][i, j]])
            lin = np.array([dp[i, j], dq1[i, j], dq2[i, j]])
            e = np.array([beta, L["Ix"][i, j], L["Iy"][i, j]])

            def f(x):
                xx = x if beta > 0 else np.array([0.0, x[1], x[2]])
                return (lam * abs(L["It"][i, j] + e @ xx) - lin @ xx + ((xx - x0) ** 2).sum() / (2 * sigma))
            best = min((scipy.optimize.minimize(f, x0 + rng.normal(scale=0.3, size=3), method="Nelder-Mead",
                                                options=dict(xatol=1e-11, fatol=1e-14, maxiter=20000)) for _ in range(3)),
                       key=lambda r: r.fun)
            got = np.array([new["w"][i, j], new["u"][i, j], new["v"][i, j]])
            assert f(got) <= best.fun + 1e-9
            assert np.allclose(got[1:], best.x[1:], atol=2e-4)
    # extrapolation: X bar+ = 2 X+ - X
    assert np.allclose(new["ub"], 2 * new["u"] - st["u"]) and np.allclose(new["vb"], 2 * new["v"] - st["v"])


def test_alg1_reaches_the_minimum_of_the_preconditioned_schemes():
    """ALG1 converges (O(1/k)) to the same minimum energy as pADMM on the same linearised problem."""
    ref = run("padmm", 1.0, 0.05, 3000, (3000,))[-1]
    tr = run("alg1", 1.0, 0.05, 6000, (200, 6000))
    first, last = tr
    assert abs(last["gap"]) < 0.25 * abs(first["gap"])
    assert abs(last["gap"]) / last["energy"] < 5e-3, last
    assert abs(last["energy"] - ref["energy"]) / ref["energy"] < 5e-3, (last["energy"], ref["energy"])
