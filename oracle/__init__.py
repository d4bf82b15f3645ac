"""FP64 CPU oracle for the priorconditioned lagged-diffusivity solver.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct
restatement of what the method computes (Arridge, Betcke and Harhanen,
"A priorconditioned LSQR algorithm for linear ill-posed problems with
edge-preserving regularization"). It is imported by the test-suite, by the
smoke check and by the benchmark's CPU-baseline leg, and by nothing else: the
product path (the HIP library and its Python binding) never imports, calls or
falls back to it, and it shares no code with that path.

Modules, in the order the method uses them:
  regularizers  r(t) of eq. (1.3)-(1.5) and the diffusivity r'(t)/t of (1.12)-(1.13)
  grid          forward-difference gradient, |grad f|, R(f), and M = G^T diag(kappa) G + eps I
  operators     the forward map A and its adjoint (separable blur, dense matrix)
  multigrid     Galerkin geometric multigrid V-cycle, a fixed SPD approximation of M^{-1}
                (Section 4.2)
  mlsqr         Algorithm 2 (MLSQR) with the damping of Section 3.3 / eq. (3.6)
  lagged        Algorithm 3, the lagged-diffusivity outer loop, with fixed iteration counts

Everything is float64. Inputs given as float32 (data, blur taps, dense
matrices) are widened exactly to float64 first.
"""

from . import regularizers, grid, operators, multigrid, mlsqr, lagged  # noqa: F401
from .lagged import solve  # noqa: F401
