"""FP64 CPU oracle for the preconditioned dual TV-L1 optical-flow solvers (test infrastructure).

This package is a plain, slow, deliberately unoptimised NumPy restatement of what the method
computes, written from the paper (Sun, Tai, Yuan, "Variational Image Motion Estimation by
Accelerated Dual Optimization", arXiv 2011.10979).  It exists only to check the GPU library:
tests, the smoke check and the CPU-baseline leg of the benchmark may use it; the product path
never imports it and shares no code with it (the seeded input generators in `synth` are the only
common dependency, and they hold none of the method's arithmetic).

Modules
  ops       discrete gradient / divergence / Laplacian, projections, bilinear sampling, resolvent
  pyramid   coarse-to-fine pyramid, derivative filter, warping + linearisation, flow upsampling
  schemes   one iteration of rpADMMI (pADMM for r = 1), rpADMMII, Zach-pADMM and pDR (+ SRBGS)
  energy    primal energy, dual objective, dual gap, feasibility residual
  solve     the coarse-to-fine driver

Parity status: every function has at least one pin in tests/test_oracle_*.py except the
coarse-to-fine choices that the paper leaves open (pyramid filter, derivative filter, upsampling,
warp clamping, intensity scale): "parity unpinned" by the paper for those, pinned only by exactness
properties of the chosen definitions.
"""
from . import ops, pyramid, schemes, energy, solve  # noqa: F401
from .solve import Params, solve_pair  # noqa: F401
