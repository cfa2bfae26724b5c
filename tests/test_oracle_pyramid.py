"""Pins of the coarse-to-fine definitions (no GPU).

The paper leaves the pyramid open ("parity unpinned" by the paper); these tests pin the chosen
definitions to exactness properties and to independent library routines.
"""
import numpy as np
import pytest

from oracle import pyramid, ops


@pytest.mark.parametrize("shape", [(2, 2), (3, 5), (8, 6), (9, 11)])
def test_downsample_matches_padded_block_mean(shape):
    rng = np.random.default_rng(0)
    I = rng.normal(size=shape)
    M, N = shape
    P = np.pad(I, ((0, M % 2), (0, N % 2)), mode="edge")
    ref = P.reshape(P.shape[0] // 2, 2, P.shape[1] // 2, 2).mean(axis=(1, 3))
    np.testing.assert_allclose(pyramid.downsample(I), ref, rtol=0, atol=1e-15)


def test_downsample_constant_and_ramp():
    assert np.all(pyramid.downsample(np.full((7, 9), 3.25)) == 3.25)
    i, j = np.indices((8, 10)).astype(float)
    ramp = 0.5 * i - 2.0 * j + 1.0
    ii, jj = np.indices((4, 5)).astype(float)
    np.testing.assert_allclose(pyramid.downsample(ramp), 0.5 * (2 * ii + 0.5) - 2.0 * (2 * jj + 0.5) + 1.0,
                               atol=1e-13)


def test_level_shapes_ceil():
    assert pyramid.level_shapes(480, 640, 5) == [(480, 640), (240, 320), (120, 160), (60, 80), (30, 40)]
    assert pyramid.level_shapes(1080, 1920, 6)[-1] == (34, 60)
    assert pyramid.level_shapes(135, 7, 2)[-1] == (68, 4)


def test_derivatives_exact_for_quadratics_inside():
    i, j = np.indices((9, 12)).astype(float)
    F = 0.3 * j * j - 1.1 * i * j + 2.0 * i + 0.7
    Dx, Dy = pyramid.derivatives(F)
    np.testing.assert_allclose(Dx[:, 1:-1], (0.6 * j - 1.1 * i)[:, 1:-1], atol=1e-12)
    np.testing.assert_allclose(Dy[1:-1, :], (-1.1 * j + 2.0)[1:-1, :], atol=1e-12)
    # at the frame edge the replicated neighbour halves a one-sided difference
    np.testing.assert_allclose(Dx[:, 0], 0.5 * (F[:, 1] - F[:, 0]), atol=1e-12)


def test_linearize_zero_flow():
    rng = np.random.default_rng(1)
    I0, I1 = rng.uniform(size=(6, 7)), rng.uniform(size=(6, 7))
    Dx, Dy = pyramid.derivatives(I1)
    z = np.zeros((6, 7))
    Ix, Iy, It, at = pyramid.linearize(I0, I1, Dx, Dy, z, z, 255.0, 0.0)
    np.testing.assert_allclose(Ix, 255 * Dx, atol=1e-12)
    np.testing.assert_allclose(Iy, 255 * Dy, atol=1e-12)
    np.testing.assert_allclose(It, 255 * (I1 - I0), atol=1e-12)
    assert np.isclose(at, np.max(Ix ** 2 + Iy ** 2))


def test_linearize_is_exact_first_order_model_on_a_ramp():
    """For a linear I1 and an interior linearisation point d0, rho(d) = kappa (I1(x + d) - I0(x))."""
    M, N = 20, 24
    i, j = np.indices((M, N)).astype(float)
    I1 = 0.01 * j + 0.02 * i + 0.1
    I0 = np.full((M, N), 0.3)
    Dx, Dy = pyramid.derivatives(I1)
    u0 = np.full((M, N), 1.5)
    v0 = np.full((M, N), 0.6)   # I_x u0 + I_y v0 != 0, so a dropped flow term shows
    kappa = 255.0
    Ix, Iy, It, _ = pyramid.linearize(I0, I1, Dx, Dy, u0, v0, kappa, 0.0)
    du, dv = 0.4, 0.3
    rho = Ix * (u0 + du) + Iy * (v0 + dv) + It
    target = kappa * (0.01 * (j + u0 + du) + 0.02 * (i + v0 + dv) + 0.1 - I0)
    sl = (slice(2, M - 3), slice(2, N - 4))
    np.testing.assert_allclose(rho[sl], target[sl], atol=1e-11)


def test_linearize_integer_shift_samples_exactly():
    rng = np.random.default_rng(2)
    I1 = rng.uniform(size=(10, 12))
    I0 = np.zeros_like(I1)
    Dx, Dy = pyramid.derivatives(I1)
    u0 = np.full(I1.shape, 2.0)
    v0 = np.full(I1.shape, 1.0)
    Ix, Iy, It, _ = pyramid.linearize(I0, I1, Dx, Dy, u0, v0, 1.0, 0.0)
    I1w = It + Ix * u0 + Iy * v0
    np.testing.assert_allclose(I1w[:-1, :-2], I1[1:, 2:], atol=1e-14)


def test_upsample_constant_and_linear():
    c = np.full((5, 6), 1.25)
    np.testing.assert_allclose(pyramid.upsample(c, (10, 12), 2.0), 2.5, atol=1e-15)
    a, b = np.indices((6, 8)).astype(float)
    lin = 3.0 * a - b
    fine = pyramid.upsample(lin, (12, 16), 1.0)
    i, j = np.indices((12, 16)).astype(float)
    ref = 3.0 * (0.5 * i - 0.25) - (0.5 * j - 0.25)
    np.testing.assert_allclose(fine[1:-1, 1:-1], ref[1:-1, 1:-1], atol=1e-12)


def test_upsample_inverts_downsample_geometry():
    """A flow that is a linear function of position survives downsample -> upsample (x2 scaling)."""
    i, j = np.indices((16, 20)).astype(float)
    u = 0.1 * j + 0.05 * i
    uc = pyramid.downsample(u) * 0.5          # coarse pixel units
    back = pyramid.upsample(uc, u.shape, 2.0)
    np.testing.assert_allclose(back[1:-1, 1:-1], u[1:-1, 1:-1], atol=1e-12)


def test_bilinear_used_by_warp_clamps():
    F = np.arange(6.0).reshape(2, 3)
    assert ops.bilinear(F, np.array([-1.0]), np.array([5.0]))[0] == F[0, 2]


def _is_half(x):
    return np.array_equal(np.asarray(x, np.float64).astype(np.float16).astype(np.float64), x)


def test_f16_storage_form_planes_are_binary16_and_centred():
    """The half-precision storage form: every stored plane holds binary16 values; the images are
    the frames minus 1/2 to within half a binary16 spacing at the finest level, and each coarse
    level is the binary16 value nearest the 2x2 mean of the stored level above it (checked against
    the exact FP64 mean of those stored values: at most half a binary16 spacing away; the binary32
    sum of four binary16 operands in [-1/2, 1/2] only rounds when it reaches 1 in magnitude with an
    operand below 2^-13, which these inputs never combine)."""
    rng = np.random.default_rng(11)
    I0 = rng.uniform(0, 1, (23, 30)).astype(np.float32).astype(np.float64)
    I1 = rng.uniform(0, 1, (23, 30)).astype(np.float32).astype(np.float64)
    p16 = pyramid.build_pyramid(I0, I1, 4, storage="f16")
    p32 = pyramid.build_pyramid(I0, I1, 4)
    for lev, planes in enumerate(p16):
        assert all(_is_half(x) for x in planes)
        assert all(np.abs(x).max() <= 0.5 for x in planes[:2])
    spacing = lambda x: np.spacing(np.abs(x).astype(np.float16)).astype(np.float64)  # noqa: E731
    for k, I in ((0, I0), (1, I1)):
        assert np.all(np.abs(p16[0][k] - (I - 0.5)) <= 0.5 * spacing(p16[0][k]))
    for lev in range(1, 4):
        for k in (0, 1):
            exact = pyramid.downsample(p16[lev - 1][k])
            assert np.all(np.abs(p16[lev][k] - exact) <= 0.5 * spacing(p16[lev][k]) + 1e-12)
        dx, dy = pyramid.derivatives(p16[lev][1])
        assert np.all(np.abs(p16[lev][2] - dx) <= 0.5 * spacing(p16[lev][2]) + 1e-12)
        assert np.all(np.abs(p16[lev][3] - dy) <= 0.5 * spacing(p16[lev][3]) + 1e-12)
    # the storage form stays close to the FP64 pyramid (a few binary16 spacings of 1/2)
    for a, b in zip(p16, p32):
        assert np.abs((a[0] + 0.5) - b[0]).max() < 4 * 2.0 ** -12
        assert np.abs(a[2] - b[2]).max() < 4 * 2.0 ** -12


def test_f16_storage_form_rejects_unknown_storage():
    with pytest.raises(ValueError):
        pyramid.build_pyramid(np.zeros((4, 4)), np.zeros((4, 4)), 1, storage="bf16")


def test_f16_storage_form_recovers_the_translation():
    """Solved on the 64 x 64 translation pair the storage form still recovers the motion, with
    a mean flow within 1e-2 px of the FP32 form's."""
    import synth
    from oracle import Params, solve_pair
    pair = synth.translation_pair(0)
    I0 = pair.I0.astype(np.float32).astype(np.float64)
    I1 = pair.I1.astype(np.float32).astype(np.float64)
    r32 = solve_pair(I0, I1, Params(levels=1, warps=1, iters=200))
    r16 = solve_pair(I0, I1, Params(levels=1, warps=1, iters=200, storage="f16"))
    assert abs(r16["u"].mean() - r32["u"].mean()) < 1e-2 and abs(r16["v"].mean() - r32["v"].mean()) < 1e-2
    assert abs(r16["u"].mean() - 0.3) < 0.03 and abs(r16["v"].mean() + 0.2) < 0.03
