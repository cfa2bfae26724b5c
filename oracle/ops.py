"""Pointwise and stencil operators of the discrete model, FP64 (oracle; test infrastructure).

Grid: Omega = {0..M-1} x {0..N-1}, arrays indexed [i, j] with i the row (y) and j the column (x).
"""
from __future__ import annotations

import numpy as np


# --- Sec. 2.2: discrete gradient and its negative adjoint --------------------------------------
def grad(f):
    """Forward-difference gradient X -> Y, zero on the last column (x part) / last row (y part).

    Sec. 2.2 takes the gradient of its references [CP, BS]: forward differences with the dual
    variables vanishing on the boundary (Sec. 2.1, eq:tvw).
    """
    f = np.asarray(f, dtype=np.float64)
    gx = np.zeros_like(f)
    gy = np.zeros_like(f)
    gx[:, :-1] = f[:, 1:] - f[:, :-1]
    gy[:-1, :] = f[1:, :] - f[:-1, :]
    return gx, gy


def div(px, py):
    """Discrete divergence Y -> X defined by <grad u, p>_Y = -<u, div p>_X (Sec. 2.2).

    Written out: (div p)_ij = [j<N-1] px_ij - [j>0] px_i,j-1 + [i<M-1] py_ij - [i>0] py_i-1,j.
    """
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    d = np.zeros_like(px)
    d[:, :-1] += px[:, :-1]
    d[:, 1:] -= px[:, :-1]
    d[:-1, :] += py[:-1, :]
    d[1:, :] -= py[:-1, :]
    return d


def laplacian(f):
    """Delta = div o grad: the 5-point Laplacian with Neumann boundary (Sec. 3.1.2, eq. neumann:boudary)."""
    gx, gy = grad(f)
    return div(gx, gy)


def grad_gradstar(px, py):
    """The operator grad grad^* = -grad div on Y, appearing in the proximal weight a c I - c grad grad^*."""
    gx, gy = grad(div(px, py))
    return -gx, -gy


# --- Sec. 3.1, discrete norms (eq:euclid:norm) and the projections P_s, P_p, P_q ----------------
def norm_p(px, py):
    """|p_ij| = sqrt(p1^2 + p2^2) (eq:euclid:norm)."""
    return np.sqrt(px * px + py * py)


def norm_q(q1x, q1y, q2x, q2y):
    """|q_ij| = sqrt of the sum of the four squared components (eq:euclid:norm): TV of d is coupled."""
    return np.sqrt(q1x * q1x + q1y * q1y + q2x * q2x + q2y * q2y)


def proj_p(px, py):
    """P_p: Euclidean projection of each p_ij onto the unit disc, p / max(1, |p|) (Sec. 3.1.1)."""
    n = np.maximum(1.0, norm_p(px, py))
    return px / n, py / n


def proj_q(q1x, q1y, q2x, q2y):
    """P_q: joint projection of the 4-vector q_ij onto the unit ball, q / max(1, |q|) (Sec. 3.1.1)."""
    n = np.maximum(1.0, norm_q(q1x, q1y, q2x, q2y))
    return q1x / n, q1y / n, q2x / n, q2y / n


def proj_s(s, lam):
    """P_s: projection onto {|s_ij| <= lambda} (eq:ofc-dual), i.e. clamping to [-lambda, lambda]."""
    return np.clip(s, -lam, lam)


# --- coarse-to-fine sampling -------------------------------------------------------------------
def bilinear(F, y, x):
    """Bilinear sample of F at real (y, x) with coordinates clamped into the frame.

    i0 = min(floor(y), M-2), j0 = min(floor(x), N-2); the four-tap weights are (1-fy)(1-fx), ...
    Requires M, N >= 2.
    """
    F = np.asarray(F, dtype=np.float64)
    M, N = F.shape
    y = np.clip(np.asarray(y, dtype=np.float64), 0.0, M - 1.0)
    x = np.clip(np.asarray(x, dtype=np.float64), 0.0, N - 1.0)
    i0 = np.minimum(np.floor(y).astype(np.int64), M - 2)
    j0 = np.minimum(np.floor(x).astype(np.int64), N - 2)
    fy = y - i0
    fx = x - j0
    return ((1.0 - fy) * ((1.0 - fx) * F[i0, j0] + fx * F[i0, j0 + 1])
            + fy * ((1.0 - fx) * F[i0 + 1, j0] + fx * F[i0 + 1, j0 + 1]))


# --- Sec. 3.1.2, eq:resolvent: proximal step of the data term ----------------------------------
def resolvent(wt, ut, vt, Ix, Iy, It, beta, lam, sigma):
    """(I + sigma dF)^{-1} for F = lambda |rho(w, d)|_1, rho = I_t + beta w + I_x u + I_y v.

    Three cases on rho~ = rho(w~, d~) against sigma lambda |e|^2 with e = (beta, I_x, I_y)
    (eq:resolvent, proved in the Appendix).  Where |e|^2 = 0 the data term is constant and the
    resolvent is the identity.  Returns (w, u, v) and the dual value Theta of the prox subproblem,
    the projection of rho~ / (sigma |e|^2) onto [-lambda, lambda] (Appendix).
    """
    e2 = beta * beta + Ix * Ix + Iy * Iy
    rho = It + beta * wt + Ix * ut + Iy * vt
    thr = sigma * lam * e2
    safe = np.where(e2 > 0, e2, 1.0)
    step = np.where(rho < -thr, sigma * lam,                 # move along +e
                    np.where(rho > thr, -sigma * lam,        # move along -e
                             -rho / safe))                   # land on rho = 0
    step = np.where(e2 > 0, step, 0.0)
    theta = np.where(e2 > 0, np.clip(rho / (sigma * safe), -lam, lam), 0.0)
    return wt + step * beta, ut + step * Ix, vt + step * Iy, theta
