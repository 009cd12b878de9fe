"""FP64 CPU oracle for the rid-preconditioned Davidson solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
imports, links or calls it, and it shares no code with the GPU library: it
takes its inputs from the seeded generator in ``synth`` and implements every
step of the method itself, in plain NumPy float64, in the order and notation of
the paper (Zhou & Parker, "Converging TDDFT calculations in 5 iterations with
minimal auxiliary preconditioning"):

* ``operators``  -- the response operators A, A+B, A-B (Eq. hessian with the
  XC kernel dropped and RI-factored ERIs, Eq. pqrs_approx) and the ris model
  T (Eqs. pqrs_approx, TDDFT-ris_approx; exchange cutoff of Sec. 3.1; the
  (d, s) angular-momentum split of Sec. 3.2), plus dense builders for tiny
  sizes;
* ``linalg``     -- Gram-Schmidt with a drop rule (Sec. 2.1);
* ``precond``    -- the diagonal preconditioner and the inner Krylov solve of
  Eq. precondition with the ris model, and the ris initial guesses;
* ``davidson``   -- Davidson for TDA (Eq. TDA) and full TDDFT (Eq. Casida);
* ``response``   -- the polarizability of Eq. TDDFT_polar.

Every function's parity status is pinned by tests under ``tests/`` (tests
whose names start with ``test_oracle``).
"""

from .operators import OracleProblem  # noqa: F401
from .davidson import eigen_tda, eigen_rpa, SolveResult  # noqa: F401
from .response import polarizability, ResponseResult  # noqa: F401
