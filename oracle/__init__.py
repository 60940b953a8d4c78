"""CPU oracle for the restarted Krylov evolution v(t) = exp(-iHt) v0 with the a-posteriori bound.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy/SciPy
implementation written from the paper (TimeEvolver, Michel & Zell, CPC 2022).
It exists to check the HIP path: only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  The product path never calls it,
and it shares no code, tables or constants with the HIP library.

Modules
  quadrature  adaptive tanh-sinh rule for the error integral (Sec. "Improvement of
              Error Bound", eq. errorIntegral; Alg. 1 step 2) and the fast non-adaptive
              Gauss-Legendre option (Sec. "Description of Program")
  krylov      Alg. 1: Arnoldi step on A = -iH (eq. arnoldi), diagonalisation of the
              Hessenberg matrix, step-size search (eqs. errorRate, stepSize) and the
              restart loop, plus the roundoff estimate of eq. numericalError.

Readings of points where the paper is silent or garbled are listed in the
module docstrings; every function there names the passage it follows.
Parity status: every function is pinned by a `-m "not gpu"` test (dense exact
solutions, closed forms, invariants, an arbitrary-precision quadrature, the
paper's forward-backward example).  The step search's substep loop (reading R4)
is pinned on its own: the error it attaches to each accepted step must equal the
integral over [0, tau] computed without the oracle's quadrature (closed forms,
an integrand whose only feature lies in the first substep interval, QUADPACK on
integrands captured from evolutions), and the literal bounds of the printed loop,
planted, fail those pins.  None is "parity unpinned".
"""

from .quadrature import gauss_legendre, tanh_sinh, QuadratureResult
from .krylov import (Options, ArnoldiResult, EvolveResult, StepUnderflow, WARN_NUMERICAL,
                     WARN_QUADRATURE, spmv, arnoldi, hessenberg_eig, bound_integrand,
                     step_size, krylov_coefficients, evolve, hessenberg_from_lanczos)

__all__ = [
    "tanh_sinh", "gauss_legendre", "QuadratureResult", "Options", "ArnoldiResult", "EvolveResult", "StepUnderflow",
    "WARN_NUMERICAL", "WARN_QUADRATURE", "spmv", "arnoldi", "hessenberg_eig", "bound_integrand",
    "step_size", "krylov_coefficients", "evolve", "hessenberg_from_lanczos",
]
