"""flow_solve_static (the allocation-free entry point) against flow_solve on the same inputs: two
calls in a row, the second on a smaller pair, each bitwise equal to the context solve with the
built-in plan (the same kernels on the same layout)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2011_10979_amd as fm  # noqa: E402
import synth  # noqa: E402
from helpers import to_dev, f32  # noqa: E402


@pytest.mark.parametrize("scheme,beta,storage", [("padmm", 0.0, "f32"), ("rpadmm2", 0.05, "f32"), ("pdr", 0.0, "f32"),
                                                 ("padmm", 0.0, "f16")])
def test_static_solve_equals_flow_solve_twice_in_a_row(scheme, beta, storage):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    relax = 1.9 if scheme == "rpadmm2" else 1.0
    ctx = fm.Context(0)
    try:
        for k, (H, W, levels) in enumerate(((240, 320, 4), (75, 101, 3))):
            print(f"[case] static solve {scheme} beta {beta} {storage} {H}x{W} call {k + 1}", flush=True)
            pair = synth.vga_pair(seed=40 + k, H=H, W=W)
            I0, I1 = to_dev(f32(pair.I0), pad=3), to_dev(f32(pair.I1), pad=3)
            p = fm.Params(scheme=scheme, relax=relax, beta=beta, storage=storage, levels=levels, warps=2, iters=20)
            u, v, res = fm.solve_static(I0, I1, p)
            ru, rv, rres = ctx.solve(I0, I1, fm.Params(**{**p.__dict__, "use_graph": 0}))
            assert torch.equal(u, ru) and torch.equal(v, rv), (scheme, H, W)
            assert res["energy"] == rres["energy"] and res["gap"] == rres["gap"]
            assert np.isfinite(res["energy"])
    finally:
        ctx.close()


def test_static_solve_limits():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    need, limit = fm.static_bytes(1080, 1920, fm.Params(levels=6))
    assert need <= limit == 256 << 20
    I = torch.zeros((2000, 2000), dtype=torch.float32, device="cuda")
    with pytest.raises(fm.FlowError) as e:
        fm.solve_static(I, I.clone(), fm.Params(levels=6))
    assert e.value.status == fm.FLOW_E_NOMEM
    J = torch.zeros((64, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(fm.FlowError) as e:
        fm.solve_static(J, J.clone(), fm.Params(levels=1, tol=1e-3))
    assert e.value.status == fm.FLOW_E_INVAL
