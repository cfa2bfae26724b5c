"""Coarse-to-fine driver around one solver, FP64 (oracle; test infrastructure).

For level l = L-1 (coarsest) .. 0: bring the flow up from the coarser level (zero at the coarsest),
reset the dual variables, then `warps` times re-linearise around the current flow and run `iters`
iterations of the chosen scheme.  Dual variables (and pDR's X bar, y bar) carry over between warps
of one level.  Sec. 4 fixes the solver parameters used here as defaults (c = 0.05; r = 1.618 for
rpADMMI; rho = 1.9 for rpADMMII; sigma = 2, tau = 0.4 for pDR; ALG1 dual step 0.1 and primal step
1 / (8 x 0.1)); the outer-loop choices are this library's reading of the unspecified "standard
coarse-to-fine framework".
"""
from __future__ import annotations

from dataclasses import dataclass, asdict

import numpy as np

from . import schemes
from .energy import terms
from .pyramid import build_pyramid, linearize, upsample

SCHEMES = ("padmm", "rpadmm2", "zach", "pdr", "alg1")
PDR_STATE = ("pdr", "alg1")     # schemes whose state is (X, X bar, y)


@dataclass
class Params:
    scheme: str = "padmm"      # padmm: rpADMMI with r = relax (pADMM at 1); rpadmm2: rho = relax;
    lam: float = 0.05          # zach: Zach-pADMM (beta = 0); pdr: preconditioned Douglas-Rachford
    beta: float = 0.0
    c: float = 0.05
    relax: float = 1.0
    sigma: float = 2.0
    tau: float = 0.4
    gs_sweeps: int = 1
    alg1_tau: float = 0.1      # ALG1: dual step (Sec. 4); the primal step is 1 / (L^2 tau), L^2 = 8
    alg1_sigma: float = 1.25
    kappa: float = 255.0       # intensity scale applied to frames given in [0, 1]
    storage: str = "f32"       # "f16": the half-precision storage form of the pyramids (build_pyramid)
    levels: int = 1
    warps: int = 1
    iters: int = 200

    def asdict(self):
        return asdict(self)


def zeros_admm(shape, u, v, w):
    z = lambda: np.zeros(shape)  # noqa: E731
    return dict(u=u, v=v, w=w, px=z(), py=z(), q1x=z(), q1y=z(), q2x=z(), q2y=z(), s=z())


def zeros_pdr(shape, u, v, w):
    z = lambda: np.zeros(shape)  # noqa: E731
    return dict(u=u, v=v, w=w, wb=w.copy(), ub=u.copy(), vb=v.copy(),
                pbx=z(), pby=z(), qb1x=z(), qb1y=z(), qb2x=z(), qb2y=z())


def step(scheme, st, L, p: Params):
    """One iteration; returns (new_state, gap_duals) where gap_duals hold (p, q, s) for the gap."""
    if scheme == "padmm":
        new = schemes.rpadmm1_step(st, L, p.beta, p.lam, p.c, p.relax)
        return new, new
    if scheme == "rpadmm2":
        new = schemes.rpadmm2_step(st, L, p.beta, p.lam, p.c, p.relax)
        return new, new
    if scheme == "zach":
        new = schemes.zach_padmm_step(st, L, p.lam, p.c)
        return new, new
    if scheme == "pdr":
        return schemes.pdr_step(st, L, p.beta, p.lam, p.sigma, p.tau, p.gs_sweeps)
    if scheme == "alg1":
        return schemes.alg1_step(st, L, p.beta, p.lam, p.alg1_tau, p.alg1_sigma)
    raise ValueError(scheme)


def warp_terms(st, duals, L, p: Params):
    return terms(st["u"], st["v"], st["w"], duals["px"], duals["py"], duals["q1x"], duals["q1y"],
                 duals["q2x"], duals["q2y"], duals["s"], L["Ix"], L["Iy"], L["It"], p.beta, p.lam)


def solve_pair(I0, I1, p: Params, trace: bool = False, perturb=None):
    """Estimate d = (u, v) with I1(x + d) ~= I0(x).  Returns a dict with u, v, w, the final warp's
    energy terms and, with trace=True, one record of terms per (level, warp).

    `perturb` (tests only; None for the method itself) maps the carried state dict to a perturbed
    copy after every iteration: a probe of how far perturbations of a given size, e.g. the rounding
    of the state to FP32, move the result."""
    if p.scheme not in SCHEMES:
        raise ValueError(p.scheme)
    if p.scheme == "zach" and p.beta != 0.0:
        raise ValueError("Zach-pADMM is the beta = 0 model")
    pyr = build_pyramid(I0, I1, p.levels, p.storage)
    u = v = w = None
    records = []
    last = None
    for lev in range(p.levels - 1, -1, -1):
        a, b, dx, dy = pyr[lev]
        shape = a.shape
        if u is None:
            u, v, w = np.zeros(shape), np.zeros(shape), np.zeros(shape)
        else:
            u, v, w = upsample(u, shape, 2.0), upsample(v, shape, 2.0), upsample(w, shape, 1.0)
        st = zeros_pdr(shape, u, v, w) if p.scheme in PDR_STATE else zeros_admm(shape, u, v, w)
        duals = zeros_admm(shape, u, v, w)
        for wp in range(p.warps):
            Ix, Iy, It, at = linearize(a, b, dx, dy, st["u"], st["v"], p.kappa, p.beta)
            L = dict(Ix=Ix, Iy=Iy, It=It, at=at)
            if p.scheme not in PDR_STATE:
                duals = st
            for _ in range(p.iters):
                st, duals = step(p.scheme, st, L, p)
                if perturb is not None:
                    st = perturb(st)
                    if p.scheme not in PDR_STATE:
                        duals = st
            if trace or (lev == 0 and wp == p.warps - 1):
                t = warp_terms(st, duals, L, p)
                t.update(level=lev, warp=wp, at=at)
                records.append(t)
                last = t
        u, v, w = st["u"], st["v"], st["w"]
    out = dict(u=u, v=v, w=w)
    out.update({k: last[k] for k in ("energy", "dual", "gap", "residual", "tv", "data")})
    if trace:
        out["trace"] = records
    return out
