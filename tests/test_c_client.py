"""A plain C program uses the library through include/flow.h alone.

tests/c_client/solve_pair.c allocates device buffers with hipMalloc, builds a pair whose second
frame is the first translated by (0.3, -0.2) px, solves it with flow_solve (2 levels, 3 warps, 100
iterations) and checks that the mean interior flow is that translation within 0.02 px.  With these
settings the FP64 oracle's mean interior flow is (0.3006, -0.2005), checked on the CPU below, so the
threshold leaves room for the float path while a wrong sign, a swapped component or a lost level
still fails.
"""
import os
import subprocess

import numpy as np
import pytest

from paper_2011_10979_amd import build as b

SHIFT = (0.3, -0.2)


def _texture(y, x):
    t = 0.5 + 0.18 * np.sin(0.21 * x + 0.13 * y) + 0.14 * np.cos(0.17 * x - 0.23 * y)
    t += 0.12 * np.exp(-((x - 40.0) ** 2 + (y - 30.0) ** 2) / 180.0)
    t -= 0.10 * np.exp(-((x - 90.0) ** 2 + (y - 60.0) ** 2) / 260.0)
    return t


def test_c_client_scenario_is_recovered_by_the_oracle():
    """The program's pass criterion holds for the FP64 oracle on the same pair and settings."""
    from oracle import Params, solve_pair
    H, W = 48, 64    # a smaller cut of the same texture keeps the CPU run short
    ii, jj = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    I0 = _texture(ii, jj).astype(np.float32).astype(np.float64)
    I1 = _texture(ii - SHIFT[1], jj - SHIFT[0]).astype(np.float32).astype(np.float64)
    r = solve_pair(I0, I1, Params(levels=2, warps=3, iters=100))
    mu, mv = r["u"][8:-8, 8:-8].mean(), r["v"][8:-8, 8:-8].mean()
    assert abs(mu - SHIFT[0]) < 0.02 and abs(mv - SHIFT[1]) < 0.02, (mu, mv)


def test_c_client_builds_as_c11():
    """flow.h and the HIP runtime header compile as C11 and the program links against the library."""
    if not os.path.exists(b.LIB):
        pytest.skip("libflowmi.so not built")
    assert os.access(b.build_c_client(), os.X_OK)


@pytest.mark.gpu
def test_c_client_solves_a_translation():
    exe = b.C_CLIENT if os.path.exists(b.C_CLIENT) else b.build_c_client()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "mean flow" in r.stdout
