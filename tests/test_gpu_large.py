"""Largest planes: a solve whose planes exceed 2 GiB, so that byte offsets pass 2^31.

The frames are an analytic texture translated by (0.3, -0.2) px, generated on the GPU; at these
sizes no oracle finishes, so the check is the property that holds at any size: the recovered flow
is that translation (mean over the interior within 0.03 px, which the FP64 oracle meets on the
same texture and settings at 128 x 128, checked below on the CPU) and the energy and gap are
finite.  Both the one-pass iteration kernel (built-in plan) and the K-iteration tiles (mode 4)
run; a 2048 x 2048 case first checks the same code path at a size where nothing is large.
"""
import math

import pytest

import numpy as np

torch = pytest.importorskip("torch")

import paper_2011_10979_amd as fm  # noqa: E402

SHIFT = (0.3, -0.2)
KW = dict(levels=2, warps=2, iters=40)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fm.Context(0)
    yield c
    c.close()
    torch.cuda.empty_cache()


def texture(n, dy, dx):
    """0.5 + 0.18 sin(0.21 x + 0.13 y) + 0.14 cos(0.17 x - 0.23 y) at (y - dy, x - dx), in FP64
    row blocks, stored FP32."""
    out = torch.empty((n, n), device="cuda", dtype=torch.float32)
    x = torch.arange(n, device="cuda", dtype=torch.float64) - dx
    for r0 in range(0, n, 2048):
        y = (torch.arange(r0, min(n, r0 + 2048), device="cuda", dtype=torch.float64) - dy)[:, None]
        t = 0.5 + 0.18 * torch.sin(0.21 * x + 0.13 * y) + 0.14 * torch.cos(0.17 * x - 0.23 * y)
        out[r0:r0 + y.shape[0]] = t.float()
        del t
    return out


def test_criterion_holds_for_the_oracle():
    """The pass criterion on the same texture, shift and settings, for the FP64 oracle at 128 x 128."""
    from oracle import Params, solve_pair
    n = 128
    y = np.arange(n, dtype=float)[:, None]
    x = np.arange(n, dtype=float)[None, :]

    def tex(dy, dx):
        t = 0.5 + 0.18 * np.sin(0.21 * (x - dx) + 0.13 * (y - dy)) + 0.14 * np.cos(0.17 * (x - dx) - 0.23 * (y - dy))
        return t.astype(np.float32).astype(np.float64)

    r = solve_pair(tex(0.0, 0.0), tex(SHIFT[1], SHIFT[0]), Params(**KW))
    m = 16
    mu, mv = r["u"][m:-m, m:-m].mean(), r["v"][m:-m, m:-m].mean()
    assert abs(mu - SHIFT[0]) < 0.03 and abs(mv - SHIFT[1]) < 0.03, (mu, mv)


@pytest.mark.gpu
@pytest.mark.parametrize("n", [2048, 24576])
@pytest.mark.parametrize("mode", [0, 4])
def test_largest_planes_solve_a_translation(ctx, n, mode):
    print(f"[case] {n}x{n} tb_mode {mode}: plane {n * n * 4 / 2**30:.2f} GiB", flush=True)
    I0 = texture(n, 0.0, 0.0)
    I1 = texture(n, SHIFT[1], SHIFT[0])
    fm.set_tuning("tb_mode", mode)
    try:
        u, v, res = ctx.solve(I0, I1, fm.Params(**KW))
        torch.cuda.synchronize()
    finally:
        fm.set_tuning("tb_mode", 0)
    m = 16
    mu = u[m:-m, m:-m].double().mean().item()
    mv = v[m:-m, m:-m].double().mean().item()
    print(f"[parity] {n}x{n} tb_mode {mode}: mean flow ({mu:.4f}, {mv:.4f}), energy {res['energy']:.4e} "
          f"gap {res['gap']:.4e}", flush=True)
    assert abs(mu - SHIFT[0]) < 0.03 and abs(mv - SHIFT[1]) < 0.03, (mu, mv)
    assert math.isfinite(res["energy"]) and math.isfinite(res["gap"])
    del I0, I1, u, v
