"""Coarse-to-fine framework around the solvers, FP64 (oracle; test infrastructure).

Sec. 4 only says the solvers run inside a standard coarse-to-fine (multiscale pyramid) framework;
it gives no filter, factor, derivative or interpolation.  The definitions below are this library's
reading (factor 1/2, 2x2 box average with edge replication, ceil sizes, central differences with
replicated neighbours, bilinear warping with clamped coordinates, centre-aligned bilinear
upsampling).  They are "parity unpinned" by the paper: they are pinned only by exactness properties
(constants, linear ramps, integer shifts, scipy's linear interpolation) in the tests.
"""
from __future__ import annotations

import numpy as np

from .ops import bilinear


def downsample(I, dtype=np.float64):
    """Next pyramid level: mean of the 2x2 block at (2i, 2j), rows/columns past the edge replicated
    (the four taps summed in row-major order, in `dtype` arithmetic)."""
    I = np.asarray(I, dtype=dtype)
    M, N = I.shape
    Mc, Nc = (M + 1) // 2, (N + 1) // 2
    r0 = 2 * np.arange(Mc)
    r1 = np.minimum(r0 + 1, M - 1)
    c0 = 2 * np.arange(Nc)
    c1 = np.minimum(c0 + 1, N - 1)
    return 0.25 * (I[np.ix_(r0, c0)] + I[np.ix_(r0, c1)] + I[np.ix_(r1, c0)] + I[np.ix_(r1, c1)])


def level_shapes(M, N, levels):
    shapes = [(M, N)]
    for _ in range(levels - 1):
        m, n = shapes[-1]
        shapes.append(((m + 1) // 2, (n + 1) // 2))
    return shapes


def derivatives(F, dtype=np.float64):
    """Central differences (F[j+1] - F[j-1]) / 2 with neighbour indices clamped into the frame."""
    F = np.asarray(F, dtype=dtype)
    M, N = F.shape
    jp = np.minimum(np.arange(N) + 1, N - 1)
    jm = np.maximum(np.arange(N) - 1, 0)
    ip = np.minimum(np.arange(M) + 1, M - 1)
    im = np.maximum(np.arange(M) - 1, 0)
    Dx = 0.5 * (F[:, jp] - F[:, jm])
    Dy = 0.5 * (F[ip, :] - F[im, :])
    return Dx, Dy


def build_pyramid(I0, I1, levels, storage="f32"):
    """Per level l = 0 (finest) .. levels-1: (I0, I1, D_x I1, D_y I1).

    storage="f16" is the half-precision storage form of the pyramids.  The frames (binary32) are
    stored centred, minus 1/2; every stored plane -- each image level, computed from the stored
    level above it, and each derivative plane -- is evaluated in binary32 arithmetic from stored
    operands and rounded once to binary16.  The centring cancels in the linearisation, which only
    uses differences of images and the derivatives.  The planes are returned as float64."""
    if storage == "f32":
        out = []
        a, b = np.asarray(I0, np.float64), np.asarray(I1, np.float64)
        for lev in range(levels):
            if lev > 0:
                a, b = downsample(a), downsample(b)
            dx, dy = derivatives(b)
            out.append((a, b, dx, dy))
        return out
    if storage != "f16":
        raise ValueError(storage)
    f32, half = np.float32, (lambda F: np.asarray(F, np.float32).astype(np.float16).astype(np.float32))
    a = half(np.asarray(I0, f32) - f32(0.5))
    b = half(np.asarray(I1, f32) - f32(0.5))
    out = []
    for lev in range(levels):
        if lev > 0:
            a, b = half(downsample(a, f32)), half(downsample(b, f32))
        dx, dy = derivatives(b, f32)
        out.append(tuple(np.asarray(x, np.float64) for x in (a, b, half(dx), half(dy))))
    return out


def linearize(I0, I1, DxI1, DyI1, u0, v0, kappa, beta):
    """Linearise the constancy constraint around d0 = (u0, v0) (Sec. 1, rho(d) = grad I^T d + I_t).

    I1 and its derivatives are sampled at x + d0; with intensities scaled by kappa,
      I_x = kappa D_xI1(x + d0),  I_y = kappa D_yI1(x + d0),
      I_t = kappa (I1(x + d0) - I0(x)) - I_x u0 - I_y v0,
    so that rho(d) = I_x u + I_y v + I_t is the first-order model of kappa (I1(x + d) - I0(x)).
    Also returns a~ = max over pixels of M_s = beta^2 + I_x^2 + I_y^2 (Prop. 3.1: a~ = ||M_s||),
    floored at 1e-12.
    """
    M, N = I0.shape
    ii, jj = np.meshgrid(np.arange(M, dtype=np.float64), np.arange(N, dtype=np.float64), indexing="ij")
    y = ii + v0
    x = jj + u0
    I1w = bilinear(I1, y, x)
    Ix = kappa * bilinear(DxI1, y, x)
    Iy = kappa * bilinear(DyI1, y, x)
    It = kappa * (I1w - I0) - Ix * u0 - Iy * v0
    at = max(float(np.max(beta * beta + Ix * Ix + Iy * Iy)), 1e-12)
    return Ix, Iy, It, at


def upsample(F, shape, scale):
    """Sample a coarse field at the fine grid's centres mapped to coarse coordinates, times scale.

    Fine pixel (i, j) of the 2x finer grid sits at coarse coordinate (i/2 - 1/4, j/2 - 1/4): the
    coarse pixel a is the mean of fine rows 2a and 2a+1, centred at fine coordinate 2a + 1/2.
    Flow components use scale 2 (pixel units halve), the illumination field scale 1.
    """
    M, N = shape
    ii, jj = np.meshgrid(np.arange(M, dtype=np.float64), np.arange(N, dtype=np.float64), indexing="ij")
    return scale * bilinear(F, 0.5 * ii - 0.25, 0.5 * jj - 0.25)
