"""Primal energy, dual objective, gap and feasibility residual, FP64 (oracle; test infrastructure).

The paper states the primal problem (eq:l1:finite, eq:l1:finite:no:w) and its dual
(eq:dual:l1:flow:cons with the constraints eq:dual:l1:flow:constaint) but no stopping test.  The
quantities here are the natural ones: E is the linearised energy of the current warp, D the dual
objective <I_t, s>, gap = E - D, and r = A s + B y the dual feasibility residual.  They satisfy
  E - D = G_TV + G_data + <Lambda, r>,
with G_TV = sum(|grad d| - <grad d, q>) (+ the w, p part) >= 0 and G_data = sum(lambda|rho| - rho s)
>= 0 whenever |q| <= 1 and |s| <= lambda, which fixes every sign convention.
"""
from __future__ import annotations

import numpy as np

from .ops import grad, div


def terms(u, v, w, px, py, q1x, q1y, q2x, q2y, s, Ix, Iy, It, beta, lam):
    """All per-warp scalars as a dict (sums over the whole grid)."""
    ux, uy = grad(u)
    vx, vy = grad(v)
    nd = np.sqrt(ux * ux + uy * uy + vx * vx + vy * vy)
    tv = float(nd.sum())
    g_tv = float((nd - (ux * q1x + uy * q1y + vx * q2x + vy * q2y)).sum())
    if beta != 0.0:
        wx, wy = grad(w)
        nw = np.sqrt(wx * wx + wy * wy)
        tv += float(nw.sum())
        g_tv += float((nw - (wx * px + wy * py)).sum())
    rho = It + beta * w + Ix * u + Iy * v
    data = lam * float(np.abs(rho).sum())
    g_data = float((lam * np.abs(rho) - rho * s).sum())
    dual = float((It * s).sum())
    r_u = Ix * s - div(q1x, q1y)
    r_v = Iy * s - div(q2x, q2y)
    res2 = float((r_u * r_u + r_v * r_v).sum())
    lam_r = float((u * r_u + v * r_v).sum())
    if beta != 0.0:
        r_w = beta * s - div(px, py)
        res2 += float((r_w * r_w).sum())
        lam_r += float((w * r_w).sum())
    energy = tv + data
    return dict(energy=energy, tv=tv, data=data, dual=dual, gap=energy - dual,
                residual=float(np.sqrt(res2)), g_tv=g_tv, g_data=g_data, lam_r=lam_r)
