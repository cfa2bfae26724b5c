"""Seeded synthetic frame pairs with known motion (inputs for both the solver and its checker).

Frames are sampled from an analytic texture: a sum of isotropic Gaussian blobs plus a band-limited
random-phase plane-wave field.  The second frame is the same texture evaluated at displaced
coordinates, so the ground-truth motion is exact and no image resampling (bilinear warping,
pyramids, derivative filters) enters the data.  This module holds none of the flow solver's
arithmetic; it only draws random numbers and evaluates the texture.

Conventions: pixel (i, j) sits at y = i (row), x = j (column).  Motion d = (u, v) has u along x and
v along y.  Frame 1 is built by backward warping, I1(y) = T(y - d(y)), so that
I1(x + d(x)) ~= I0(x) = T(x) where d is locally constant.  Both frames are mapped by the same affine
map that sends I0's range to [0, 1]; frame 1 then receives additive N(0, noise^2) noise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Texture", "Pair", "make_pair", "texture_blobs", "texture_rich", "flow_constant",
    "flow_piecewise", "flow_affine_occluded", "translation_pair", "vga_pair", "hd_pair",
    "batch_pair", "batch_pairs", "levels_by_size", "serving_trace", "SERVING_SIZES", "SERVING_PROBS",
]


@dataclass
class Texture:
    """Analytic intensity field T(y, x) = sum_k A_k exp(-|p - c_k|^2 / (2 s_k^2)) + waves."""
    centers: np.ndarray          # (K, 2) blob centres (y, x)
    sigmas: np.ndarray           # (K,)
    amps: np.ndarray             # (K,)
    wave_freq: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))  # (M, 2) cycles/px (fy, fx)
    wave_phase: np.ndarray = field(default_factory=lambda: np.zeros(0))
    wave_amp: float = 0.0
    cutoff: float = 5.0          # blobs are evaluated within cutoff * sigma of their centre

    def eval(self, Y: np.ndarray, X: np.ndarray, margin: float = 0.0) -> np.ndarray:
        """Evaluate T at real coordinates (Y, X), arrays shaped like the pixel grid.

        `margin` bounds |Y - i| and |X - j| over the grid; it widens each blob's evaluation window
        so that displaced coordinates are still covered.
        """
        H, W = Y.shape
        out = np.zeros((H, W), dtype=np.float64)
        for (cy, cx), s, a in zip(self.centers, self.sigmas, self.amps):
            r = self.cutoff * s + margin + 1.0
            i0, i1 = max(0, int(math.floor(cy - r))), min(H, int(math.ceil(cy + r)) + 1)
            j0, j1 = max(0, int(math.floor(cx - r))), min(W, int(math.ceil(cx + r)) + 1)
            if i0 >= i1 or j0 >= j1:
                continue
            dy = Y[i0:i1, j0:j1] - cy
            dx = X[i0:i1, j0:j1] - cx
            out[i0:i1, j0:j1] += a * np.exp(-(dy * dy + dx * dx) / (2.0 * s * s))
        if self.wave_amp != 0.0 and len(self.wave_phase):
            for (fy, fx), ph in zip(self.wave_freq, self.wave_phase):
                out += self.wave_amp * np.cos(2.0 * np.pi * (fy * Y + fx * X) + ph)
        return out


@dataclass
class Pair:
    I0: np.ndarray
    I1: np.ndarray
    u: np.ndarray                # ground-truth motion along x (columns)
    v: np.ndarray                # ground-truth motion along y (rows)
    meta: dict


def _grid(H, W):
    Y, X = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    return Y, X


def texture_blobs(rng: np.random.Generator, H: int, W: int, n: int = 20,
                  sigma=(3.0, 10.0), amp=(0.0, 1.0)) -> Texture:
    """n Gaussians, centres uniform over the frame, sigma ~ U[sigma], amplitude ~ U[amp]."""
    centers = np.stack([rng.uniform(0, H, n), rng.uniform(0, W, n)], axis=1)
    sig = rng.uniform(sigma[0], sigma[1], n)
    amps = rng.uniform(amp[0], amp[1], n)
    return Texture(centers, sig, amps)


def texture_rich(rng: np.random.Generator, H: int, W: int, n: int = 200, n_waves: int = 48,
                 noise_sigma: float = 1.5, noise_rel: float = 0.1) -> Texture:
    """200 Gaussians (sigma ~ U[3,20], A ~ U[-1,1]) plus band-limited noise.

    The noise is a random-phase sum of plane waves whose frequencies are drawn from the power
    spectrum of white noise blurred by a Gaussian of std `noise_sigma` px (a Gaussian in frequency
    with per-axis std 1/(2*sqrt(2)*pi*noise_sigma)); its std is `noise_rel` times the blob field's
    std measured on the pixel grid.
    """
    tex = texture_blobs(rng, H, W, n, sigma=(3.0, 20.0), amp=(-1.0, 1.0))
    fstd = 1.0 / (2.0 * math.sqrt(2.0) * math.pi * noise_sigma)
    tex.wave_freq = rng.normal(0.0, fstd, size=(n_waves, 2))
    tex.wave_phase = rng.uniform(0.0, 2.0 * math.pi, n_waves)
    Y, X = _grid(H, W)
    blob_std = float(np.std(tex.eval(Y, X)))
    # a sum of M unit cosines with random phases has variance M/2
    tex.wave_amp = noise_rel * blob_std / math.sqrt(n_waves / 2.0)
    return tex


def flow_constant(H, W, u0, v0):
    return np.full((H, W), float(u0)), np.full((H, W), float(v0))


def _rects(rng, H, W, n, dmax, u, v):
    for _ in range(n):
        w = int(rng.uniform(W / 8.0, W / 3.0))
        h = int(rng.uniform(H / 8.0, H / 3.0))
        x0 = int(rng.integers(0, max(1, W - w)))
        y0 = int(rng.integers(0, max(1, H - h)))
        du, dv = rng.uniform(-dmax, dmax, 2)
        u[y0:y0 + h, x0:x0 + w] = du
        v[y0:y0 + h, x0:x0 + w] = dv
    return u, v


def flow_piecewise(rng, H, W, n_rect=3, background=(1.0, 0.0), dmax=8.0):
    """Background motion plus n_rect rectangles (later ones overwrite) with d ~ U[-dmax, dmax]^2."""
    u, v = flow_constant(H, W, *background)
    return _rects(rng, H, W, n_rect, dmax, u, v)


def flow_affine_occluded(rng, H, W, max_mag=20.0, n_rect=5, dmax=8.0):
    """Rotation + zoom about the frame centre, scaled to max |d| = max_mag, then occluding boxes."""
    theta = math.radians(rng.uniform(-3.0, 3.0))
    s = rng.uniform(0.97, 1.03)
    A = s * np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]]) - np.eye(2)
    Y, X = _grid(H, W)
    yc, xc = (H - 1) / 2.0, (W - 1) / 2.0
    dy = A[0, 0] * (Y - yc) + A[0, 1] * (X - xc)
    dx = A[1, 0] * (Y - yc) + A[1, 1] * (X - xc)
    mag = np.sqrt(dx * dx + dy * dy).max()
    scale = max_mag / mag if mag > 0 else 0.0
    u, v = dx * scale, dy * scale
    return _rects(rng, H, W, n_rect, dmax, u, v)


def make_pair(tex: Texture, u: np.ndarray, v: np.ndarray, rng: np.random.Generator,
              noise_std: float = 0.01, meta: dict | None = None) -> Pair:
    """I0 = T on the grid; I1(y) = T(y - d(y)); both mapped by I0's min-max; noise added to I1."""
    H, W = u.shape
    Y, X = _grid(H, W)
    margin = float(max(np.abs(u).max(), np.abs(v).max())) + 1.0
    T0 = tex.eval(Y, X)
    T1 = tex.eval(Y - v, X - u, margin=margin)
    lo, hi = T0.min(), T0.max()
    span = hi - lo if hi > lo else 1.0
    I0 = (T0 - lo) / span
    I1 = (T1 - lo) / span
    if noise_std > 0:
        I1 = I1 + rng.normal(0.0, noise_std, size=I1.shape)
    return Pair(I0, I1, u.copy(), v.copy(), dict(meta or {}))


def translation_pair(seed: int = 0, H: int = 64, W: int = 64, d=(0.3, -0.2), noise_std: float = 0.01) -> Pair:
    """64x64, 20 blobs (sigma 3-10, A in [0,1]), constant motion d = (u, v), N(0, 0.01^2) noise."""
    rng = np.random.default_rng(seed)
    tex = texture_blobs(rng, H, W, 20)
    u, v = flow_constant(H, W, *d)
    return make_pair(tex, u, v, rng, noise_std,
                     dict(recipe="translation", seed=seed, H=H, W=W, d=list(d)))


def vga_pair(seed: int = 1, H: int = 480, W: int = 640, noise_std: float = 0.01) -> Pair:
    """Rich texture, piecewise-constant motion: background (1, 0) plus 3 boxes d ~ U[-8, 8]^2."""
    rng = np.random.default_rng(seed)
    tex = texture_rich(rng, H, W)
    u, v = flow_piecewise(rng, H, W)
    return make_pair(tex, u, v, rng, noise_std, dict(recipe="piecewise", seed=seed, H=H, W=W))


def hd_pair(seed: int = 2, H: int = 1080, W: int = 1920, noise_std: float = 0.01) -> Pair:
    """Rich texture, rotation + zoom (max 20 px) with 5 occluding boxes."""
    rng = np.random.default_rng(seed)
    tex = texture_rich(rng, H, W)
    u, v = flow_affine_occluded(rng, H, W)
    return make_pair(tex, u, v, rng, noise_std, dict(recipe="affine", seed=seed, H=H, W=W))


def batch_pair(k: int, seed0: int = 1000, size_scale: float = 1.0) -> Pair:
    """Pair k of `batch_pairs` (seeded seed0 + k): W ~ U_int[128, 1280], H ~ U_int[96, 720]; even k
    use the piecewise-motion recipe, odd k the rotation + zoom recipe.  `size_scale` shrinks both
    sides (for quick tests) without changing the draws."""
    rng = np.random.default_rng(seed0 + k)
    W = int(rng.integers(128, 1281))
    H = int(rng.integers(96, 721))
    W = max(16, int(W * size_scale))
    H = max(16, int(H * size_scale))
    if k % 2 == 0:
        return vga_pair(seed0 + k, H, W)
    return hd_pair(seed0 + k, H, W)


def batch_pairs(n: int = 64, seed0: int = 1000, size_scale: float = 1.0):
    """n pairs of uneven sizes (see batch_pair)."""
    return [batch_pair(k, seed0, size_scale) for k in range(n)]


def levels_by_size(H: int, W: int) -> int:
    """Pyramid depth for mixed-size workloads: 1 + floor(log2(min(H, W) / 16)), clamped to [1, 6]
    (5 levels at 640 x 480, 6 at 1920 x 1080, coarsest side about 16 to 30 pixels)."""
    return int(min(6, max(1, 1 + math.floor(math.log2(min(H, W) / 16.0)))))


SERVING_SIZES = [(240, 320), (480, 640), (436, 1024), (720, 1280), (1080, 1920)]
SERVING_PROBS = [0.3, 0.3, 0.2, 0.1, 0.1]


def serving_trace(n_requests: int = 2000, rate: float = 200.0, seed: int = 7):
    """Poisson arrivals: returns (arrival_times_s, size_index) with exponential gaps of mean 1/rate."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps)
    idx = rng.choice(len(SERVING_SIZES), size=n_requests, p=SERVING_PROBS)
    return t, idx
