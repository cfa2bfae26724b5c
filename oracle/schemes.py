"""One iteration of each solver in the paper's component form, FP64 (oracle; test infrastructure).

State dictionaries hold full-size float64 arrays:
  ADMM family:  w, u, v (multipliers = primal flow and illumination), px, py (p), q1x, q1y, q2x,
                q2y (q), s (data dual).
  pDR:          w, u, v (X), wb, ub, vb (X bar), pbx, pby, qb1x, qb1y, qb2x, qb2y (y bar).
  ALG1:         the pDR layout: X, X bar (the extrapolated primal point) and y = (p, q) in the y bar
                slots.
Linearisation L holds Ix, Iy, It and at (a~).  With beta = 0 the (w, p) block never leaves zero.
"""
from __future__ import annotations

import numpy as np

from .ops import grad, div, grad_gradstar, proj_p, proj_q, proj_s, resolvent, laplacian

A_TV = 8.0   # a = 8 >= ||grad grad^*|| (Prop. 3.1, eq:stepsize:constraint)


def _dual_step(st, L, beta, c, a):
    """p and q updates shared by rpADMMI and rpADMMII (first four lines of both component forms).

    p_t = (I - grad grad^*/a) p + (grad w / c - beta grad s) / a,       p+ = P_p(p_t)
    q1_t = (I - grad grad^*/a) q1 + (grad u / c - grad(s I_x)) / a,      likewise q2 with v, I_y
    (q1+, q2+) = P_q(q1_t, q2_t)
    """
    s = st["s"]
    ggx, ggy = grad_gradstar(st["px"], st["py"])
    gwx, gwy = grad(st["w"])
    gsx, gsy = grad(s)
    ptx = st["px"] - ggx / a + (gwx / c - beta * gsx) / a
    pty = st["py"] - ggy / a + (gwy / c - beta * gsy) / a
    px, py = proj_p(ptx, pty)

    g1x, g1y = grad_gradstar(st["q1x"], st["q1y"])
    g2x, g2y = grad_gradstar(st["q2x"], st["q2y"])
    gux, guy = grad(st["u"])
    gvx, gvy = grad(st["v"])
    gsix, gsiy = grad(s * L["Ix"])
    gsjx, gsjy = grad(s * L["Iy"])
    q1tx = st["q1x"] - g1x / a + (gux / c - gsix) / a
    q1ty = st["q1y"] - g1y / a + (guy / c - gsiy) / a
    q2tx = st["q2x"] - g2x / a + (gvx / c - gsjx) / a
    q2ty = st["q2y"] - g2y / a + (gvy / c - gsjy) / a
    q1x, q1y, q2x, q2y = proj_q(q1tx, q1ty, q2tx, q2ty)
    return px, py, q1x, q1y, q2x, q2y


def rpadmm1_step(st, L, beta, lam, c, r, a=A_TV):
    """rpADMMI (Sec. 3.1.1): dual steps, s step, multipliers relaxed by r in (0, (1+sqrt 5)/2).

    pADMM is r = 1.  s+ = P_s[(I - M_s/a~) s + (I_t + beta w + u I_x + v I_y
                              + c beta div p+ + c I_x div q1+ + c I_y div q2+) / (a~ c)],
    w+ = w - r c (beta s+ - div p+),  u+ = u - r c (I_x s+ - div q1+),  v+ likewise.
    """
    Ix, Iy, It, at = L["Ix"], L["Iy"], L["It"], L["at"]
    px, py, q1x, q1y, q2x, q2y = _dual_step(st, L, beta, c, a)
    dp, dq1, dq2 = div(px, py), div(q1x, q1y), div(q2x, q2y)
    Ms = beta * beta + Ix * Ix + Iy * Iy
    s0, w, u, v = st["s"], st["w"], st["u"], st["v"]
    s = proj_s((1.0 - Ms / at) * s0 + (It + beta * w + u * Ix + v * Iy
                                      + c * beta * dp + c * Ix * dq1 + c * Iy * dq2) / (at * c), lam)
    return dict(px=px, py=py, q1x=q1x, q1y=q1y, q2x=q2x, q2y=q2y, s=s,
                w=w - r * c * (beta * s - dp),
                u=u - r * c * (Ix * s - dq1),
                v=v - r * c * (Iy * s - dq2))


def rpadmm2_step(st, L, beta, lam, c, rho, a=A_TV):
    """rpADMMII (Sec. 3.1.1, the component form of the relaxed ADMM of [SUN], rho in (0, 2)).

    s+ = P_s{(I - rho M_s/a~) s + [I_t + beta w + u I_x + v I_y
                                   + c rho (beta div p+ + I_x div q1+ + I_y div q2+)] / (a~ c)},
    w+ = w - c (beta s+ - rho div p+ - (1 - rho) beta s),  u+, v+ likewise with I_x, I_y.
    """
    Ix, Iy, It, at = L["Ix"], L["Iy"], L["It"], L["at"]
    px, py, q1x, q1y, q2x, q2y = _dual_step(st, L, beta, c, a)
    dp, dq1, dq2 = div(px, py), div(q1x, q1y), div(q2x, q2y)
    Ms = beta * beta + Ix * Ix + Iy * Iy
    s0, w, u, v = st["s"], st["w"], st["u"], st["v"]
    s = proj_s((1.0 - rho * Ms / at) * s0 + (It + beta * w + u * Ix + v * Iy
                                            + c * rho * (beta * dp + Ix * dq1 + Iy * dq2)) / (at * c), lam)
    return dict(px=px, py=py, q1x=q1x, q1y=q1y, q2x=q2x, q2y=q2y, s=s,
                w=w - c * (beta * s - rho * dp - (1.0 - rho) * beta * s0),
                u=u - c * (Ix * s - rho * dq1 - (1.0 - rho) * Ix * s0),
                v=v - c * (Iy * s - rho * dq2 - (1.0 - rho) * Iy * s0))


def zach_padmm_step(st, L, lam, c, a=A_TV):
    """Zach-pADMM (Sec. 3.1.1): the beta = 0 model with only (q, s) and multipliers (u, v).

    q_t as in rpADMMI; s+ = P_s[(I - M_s/a~) s + (I_t + u I_x + v I_y + c I_x div q1+
    + c I_y div q2+)/(a~ c)] with M_s = I_x^2 + I_y^2 (the beta div p term vanishes at beta = 0);
    u+ = u - c (I_x s+ - div q1+), v+ likewise.
    """
    Ix, Iy, It, at = L["Ix"], L["Iy"], L["It"], L["at"]
    s0, u, v = st["s"], st["u"], st["v"]
    g1x, g1y = grad_gradstar(st["q1x"], st["q1y"])
    g2x, g2y = grad_gradstar(st["q2x"], st["q2y"])
    gux, guy = grad(u)
    gvx, gvy = grad(v)
    gsix, gsiy = grad(s0 * Ix)
    gsjx, gsjy = grad(s0 * Iy)
    q1x, q1y, q2x, q2y = proj_q(st["q1x"] - g1x / a + (gux / c - gsix) / a,
                                st["q1y"] - g1y / a + (guy / c - gsiy) / a,
                                st["q2x"] - g2x / a + (gvx / c - gsjx) / a,
                                st["q2y"] - g2y / a + (gvy / c - gsjy) / a)
    dq1, dq2 = div(q1x, q1y), div(q2x, q2y)
    Ms = Ix * Ix + Iy * Iy
    s = proj_s((1.0 - Ms / at) * s0 + (It + u * Ix + v * Iy + c * Ix * dq1 + c * Iy * dq2) / (at * c), lam)
    out = dict(st)
    out.update(q1x=q1x, q1y=q1y, q2x=q2x, q2y=q2y, s=s,
               u=u - c * (Ix * s - dq1), v=v - c * (Iy * s - dq2))
    return out


# --- Sec. 3.1.2: preconditioned Douglas-Rachford ------------------------------------------------
def red_mask(shape):
    """Red cells of the red-black colouring: (i + j) even."""
    i, j = np.indices(shape)
    return (i + j) % 2 == 0


def _neighbour_sum_count(x):
    """Sum of the 4-neighbour values inside the frame and the number of such neighbours."""
    M, N = x.shape
    S = np.zeros_like(x)
    C = np.zeros_like(x)
    S[:, 1:] += x[:, :-1]; C[:, 1:] += 1
    S[:, :-1] += x[:, 1:]; C[:, :-1] += 1
    S[1:, :] += x[:-1, :]; C[1:, :] += 1
    S[:-1, :] += x[1:, :]; C[:-1, :] += 1
    return S, C


def gs_colour_update(x, b, st, mask):
    """Gauss-Seidel update of the cells in `mask` for (I - st Delta) x = b, Neumann boundary.

    Row of T at a cell with n in-frame neighbours: (1 + st n) x_ij - st sum x_nb = b_ij; cells of
    one colour only couple to the other colour, so the whole colour updates at once.
    """
    S, C = _neighbour_sum_count(x)
    return np.where(mask, (b + st * S) / (1.0 + st * C), x)


def srbgs(x, b, st, sweeps):
    """x + M^{-1}(b - T x) for M = `sweeps` symmetric red-black Gauss-Seidel sweeps (eq. neumann:boudary).

    A symmetric sweep is the forward sweep (red, then black) followed by the backward sweep
    (black, then red).
    """
    red = red_mask(x.shape)
    black = ~red
    for _ in range(sweeps):
        x = gs_colour_update(x, b, st, red)
        x = gs_colour_update(x, b, st, black)
        x = gs_colour_update(x, b, st, black)
        x = gs_colour_update(x, b, st, red)
    return x


def pdr_step(st, L, beta, lam, sigma, tau, sweeps):
    """One pDR iteration (Sec. 3.1.2, component form of the preconditioned DR iteration).

    w+ = w + M^{-1}[w_bar + sigma div p_bar - T w] (likewise u with q1_bar, v with q2_bar),
    T = I - sigma tau Delta, M = finitely many SRBGS sweeps;
    (w_bar, d_bar)+ = (w_bar, d_bar) + (I + sigma dF)^{-1}[2 (w+, d+) - (w_bar, d_bar)] - (w+, d+);
    p_bar+ = -tau grad w+ + P_p(p_bar + 2 tau grad w+), q_bar+ likewise with P_q.
    Also returns the dual pair used by the gap: q = P(y_bar + 2 tau grad X+) and s = Theta.
    """
    Ix, Iy, It = L["Ix"], L["Iy"], L["It"]
    stt = sigma * tau
    has_w = beta != 0.0
    w = srbgs(st["w"], st["wb"] + sigma * div(st["pbx"], st["pby"]), stt, sweeps) if has_w else st["w"]
    u = srbgs(st["u"], st["ub"] + sigma * div(st["qb1x"], st["qb1y"]), stt, sweeps)
    v = srbgs(st["v"], st["vb"] + sigma * div(st["qb2x"], st["qb2y"]), stt, sweeps)
    Jw, Ju, Jv, theta = resolvent(2 * w - st["wb"], 2 * u - st["ub"], 2 * v - st["vb"],
                                  Ix, Iy, It, beta, lam, sigma)
    wb = st["wb"] + Jw - w if has_w else st["wb"]
    ub = st["ub"] + Ju - u
    vb = st["vb"] + Jv - v
    gwx, gwy = grad(w)
    gux, guy = grad(u)
    gvx, gvy = grad(v)
    if has_w:
        ppx, ppy = proj_p(st["pbx"] + 2 * tau * gwx, st["pby"] + 2 * tau * gwy)
    else:
        ppx, ppy = st["pbx"], st["pby"]
    q1x, q1y, q2x, q2y = proj_q(st["qb1x"] + 2 * tau * gux, st["qb1y"] + 2 * tau * guy,
                                st["qb2x"] + 2 * tau * gvx, st["qb2y"] + 2 * tau * gvy)
    new = dict(w=w, u=u, v=v, wb=wb, ub=ub, vb=vb,
               pbx=ppx - tau * gwx if has_w else ppx, pby=ppy - tau * gwy if has_w else ppy,
               qb1x=q1x - tau * gux, qb1y=q1y - tau * guy, qb2x=q2x - tau * gvx, qb2y=q2y - tau * gvy)
    gap_duals = dict(px=ppx, py=ppy, q1x=q1x, q1y=q1y, q2x=q2x, q2y=q2y, s=theta)
    return new, gap_duals


def pdr_T(x, st):
    """T x = x - st Delta x (the operator the SRBGS sweeps precondition)."""
    return x - st * laplacian(x)


def alg1_step(st, L, beta, lam, tau, sigma):
    """One iteration of ALG1, the first-order primal-dual method of Chambolle and Pock that Sec. 4
    compares against, on the saddle form eq:primal-dual:optical:o (K = diag(grad, grad), F the data
    term, the dual sets the unit balls of p and of the coupled q), extrapolation weight 1:
      y+     = P(y + tau K X bar)                       (P_p on p, joint P_q on q)
      X+     = (I + sigma dF)^{-1}(X - sigma K^* y+)    with K^* y = -div y   (eq:resolvent)
      X bar+ = 2 X+ - X
    tau is the dual and sigma the primal step (tau sigma |K|^2 <= 1 with |K|^2 <= 8).  Returns the
    new state and the dual pair of the gap: q = y+ and s = Theta of the resolvent.
    """
    Ix, Iy, It = L["Ix"], L["Iy"], L["It"]
    has_w = beta != 0.0
    gwx, gwy = grad(st["wb"])
    gux, guy = grad(st["ub"])
    gvx, gvy = grad(st["vb"])
    if has_w:
        px, py = proj_p(st["pbx"] + tau * gwx, st["pby"] + tau * gwy)
    else:
        px, py = st["pbx"], st["pby"]
    q1x, q1y, q2x, q2y = proj_q(st["qb1x"] + tau * gux, st["qb1y"] + tau * guy,
                                st["qb2x"] + tau * gvx, st["qb2y"] + tau * gvy)
    wt = st["w"] + sigma * div(px, py) if has_w else st["w"]
    ut = st["u"] + sigma * div(q1x, q1y)
    vt = st["v"] + sigma * div(q2x, q2y)
    w, u, v, theta = resolvent(wt, ut, vt, Ix, Iy, It, beta, lam, sigma)
    if not has_w:
        w = st["w"]
    new = dict(w=w, u=u, v=v, wb=2 * w - st["w"] if has_w else st["wb"], ub=2 * u - st["u"], vb=2 * v - st["v"],
               pbx=px, pby=py, qb1x=q1x, qb1y=q1y, qb2x=q2x, qb2y=q2y)
    gap_duals = dict(px=px, py=py, q1x=q1x, q1y=q1y, q2x=q2x, q2y=q2y, s=theta)
    return new, gap_duals
