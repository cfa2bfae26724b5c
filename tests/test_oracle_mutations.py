"""Plant plausible mistakes in the oracle (on the CPU only) and check that a pin catches each one.

Every mutation is applied with monkeypatch to the oracle module that uses the function, then the
relevant pin from the other test modules is run and must fail.
"""
import numpy as np
import pytest

import test_oracle_ops as T_ops
import test_oracle_pyramid as T_pyr
import test_oracle_schemes as T_sch
from oracle import ops, schemes, pyramid


def _fails(fn, *a, **k):
    with pytest.raises(AssertionError):
        fn(*a, **k)


def test_div_with_wrong_boundary_is_caught(monkeypatch):
    def bad(px, py):
        d = np.zeros_like(px)
        d += px
        d[:, 1:] -= px[:, :-1]
        d += py
        d[1:, :] -= py[:-1, :]
        return d
    monkeypatch.setattr(ops, "div", bad)
    _fails(T_ops.test_adjoint_identity, (5, 8))


def test_div_with_wrong_sign_is_caught(monkeypatch):
    good = ops.div
    monkeypatch.setattr(ops, "div", lambda px, py: -good(px, py))
    _fails(T_ops.test_adjoint_identity, (5, 8))


def test_separate_q_projection_is_caught(monkeypatch):
    def bad(q1x, q1y, q2x, q2y):
        a = np.maximum(1.0, np.hypot(q1x, q1y))
        b = np.maximum(1.0, np.hypot(q2x, q2y))
        return q1x / a, q1y / a, q2x / b, q2y / b
    monkeypatch.setattr(ops, "proj_q", bad)
    _fails(T_ops.test_proj_q_is_joint_not_two_discs)


def test_swapped_resolvent_cases_are_caught(monkeypatch):
    def bad(wt, ut, vt, Ix, Iy, It, beta, lam, sigma):
        e2 = beta * beta + Ix * Ix + Iy * Iy
        rho = It + beta * wt + Ix * ut + Iy * vt
        thr = sigma * lam * e2
        step = np.where(rho < -thr, -sigma * lam, np.where(rho > thr, sigma * lam, -rho / np.where(e2 > 0, e2, 1)))
        step = np.where(e2 > 0, step, 0.0)
        return wt + step * beta, ut + step * Ix, vt + step * Iy, step
    monkeypatch.setattr(ops, "resolvent", bad)
    _fails(T_ops.test_resolvent_hand_cases)


def test_s_step_without_preconditioner_term_is_caught(monkeypatch):
    good = schemes.rpadmm1_step

    def bad(st, L, beta, lam, c, r, a=8.0):
        out = good(st, L, beta, lam, c, r, a)
        Ms = beta * beta + L["Ix"] ** 2 + L["Iy"] ** 2
        # recompute s+ with (I - M_s/a~) s replaced by s (a dropped term)
        dp, dq1, dq2 = ops.div(out["px"], out["py"]), ops.div(out["q1x"], out["q1y"]), ops.div(out["q2x"], out["q2y"])
        s = ops.proj_s(st["s"] + (L["It"] + beta * st["w"] + st["u"] * L["Ix"] + st["v"] * L["Iy"]
                                  + c * beta * dp + c * L["Ix"] * dq1 + c * L["Iy"] * dq2) / (L["at"] * c), lam)
        out["s"] = s
        del Ms
        return out
    monkeypatch.setattr(schemes, "rpadmm1_step", bad)
    _fails(T_sch.test_s_step_is_preconditioned_argmax, 0.3)


def test_wrong_sign_of_grad_gradstar_is_caught(monkeypatch):
    good = schemes.grad_gradstar
    monkeypatch.setattr(schemes, "grad_gradstar", lambda px, py: tuple(-x for x in good(px, py)))
    _fails(T_sch.test_y_step_is_preconditioned_argmax, 0.3)


def test_product_rule_slip_in_q_step_is_caught(monkeypatch):
    """grad(s I_x) replaced by I_x grad(s) in the q step."""
    good_grad = schemes.grad
    calls = {"n": 0}

    def bad_dual_step(st, L, beta, c, a):
        s = st["s"]
        out = list(good_dual(st, L, beta, c, a))
        gsx, gsy = good_grad(s)
        g1x, g1y = good_grad(s * L["Ix"])
        calls["n"] += 1
        del gsx, gsy, g1x, g1y
        # perturb q1 the way the slip would: add (grad(s Ix) - Ix grad s)/a before projecting
        gx, gy = good_grad(s * L["Ix"])
        sx, sy = good_grad(s)
        out[2] = out[2] + (gx - L["Ix"] * sx) / a
        out[3] = out[3] + (gy - L["Ix"] * sy) / a
        return tuple(out)
    good_dual = schemes._dual_step
    monkeypatch.setattr(schemes, "_dual_step", bad_dual_step)
    _fails(T_sch.test_y_step_is_preconditioned_argmax, 0.0)


def test_multiplier_sign_flip_breaks_convergence(monkeypatch):
    good = schemes.rpadmm1_step

    def bad(st, L, beta, lam, c, r, a=8.0):
        out = good(st, L, beta, lam, c, r, a)
        for k in ("u", "v"):
            out[k] = 2 * st[k] - out[k]
        return out
    monkeypatch.setattr(schemes, "rpadmm1_step", bad)
    tr = T_sch.run("padmm", 1.0, 0.0, 1500, (100, 1500))
    assert not (abs(tr[-1]["gap"]) / abs(tr[-1]["energy"]) < 2e-3 and tr[-1]["residual"] < 0.05 * max(tr[0]["residual"], 1.0))


def test_rpadmm2_relaxation_sign_flip_breaks_convergence(monkeypatch):
    good = schemes.rpadmm2_step

    def bad(st, L, beta, lam, c, rho, a=8.0):
        out = good(st, L, beta, lam, c, rho, a)
        # (1 - rho) I_x s^k entered with the wrong sign
        out["u"] = out["u"] - 2 * c * (1.0 - rho) * L["Ix"] * st["s"]
        out["v"] = out["v"] - 2 * c * (1.0 - rho) * L["Iy"] * st["s"]
        return out
    monkeypatch.setattr(schemes, "rpadmm2_step", bad)
    tr = T_sch.run("rpadmm2", 1.9, 0.0, 3000, (100, 3000))
    ok_gap = abs(tr[-1]["gap"]) / abs(tr[-1]["energy"]) < 2e-3
    ok_res = tr[-1]["residual"] < 0.05 * max(tr[0]["residual"], 1.0)
    assert not (ok_gap and ok_res)


def test_nonsymmetric_sweep_is_caught(monkeypatch):
    def forward_only(x, b, st, sweeps):
        red = schemes.red_mask(x.shape)
        for _ in range(sweeps):
            x = schemes.gs_colour_update(x, b, st, red)
            x = schemes.gs_colour_update(x, b, st, ~red)
        return x
    monkeypatch.setattr(schemes, "srbgs", forward_only)
    _fails(T_sch.test_srbgs_is_symmetric_feasible_preconditioner, (4, 5), 1)


def test_linearisation_without_flow_term_is_caught(monkeypatch):
    good = pyramid.linearize

    def bad(I0, I1, DxI1, DyI1, u0, v0, kappa, beta):
        Ix, Iy, It, at = good(I0, I1, DxI1, DyI1, u0, v0, kappa, beta)
        return Ix, Iy, It + Ix * u0 + Iy * v0, at
    monkeypatch.setattr(pyramid, "linearize", bad)
    _fails(T_pyr.test_linearize_is_exact_first_order_model_on_a_ramp)


def test_alg1_primal_step_with_the_wrong_adjoint_sign_is_caught(monkeypatch):
    good = schemes.div

    def flipped(px, py):
        return -good(px, py)
    # only ALG1's primal step sees the flipped divergence: its pin checks the prox of the primal step
    orig = schemes.alg1_step

    def bad(st, L, beta, lam, tau, sigma):
        monkeypatch.setattr(schemes, "div", flipped)
        try:
            return orig(st, L, beta, lam, tau, sigma)
        finally:
            monkeypatch.setattr(schemes, "div", good)
    monkeypatch.setattr(schemes, "alg1_step", bad)
    _fails(T_sch.test_alg1_primal_step_is_the_proximal_descent, 0.3)


def test_alg1_without_extrapolation_is_caught(monkeypatch):
    orig = schemes.alg1_step

    def bad(st, L, beta, lam, tau, sigma):
        new, duals = orig(st, L, beta, lam, tau, sigma)
        new = dict(new, ub=new["u"], vb=new["v"], wb=new["w"])
        return new, duals
    monkeypatch.setattr(schemes, "alg1_step", bad)
    _fails(T_sch.test_alg1_primal_step_is_the_proximal_descent, 0.0)
