"""Plain CPU FP64 oracle for the Gamma-point Tamm-Dancoff Liouville operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package:
only the tests, the ``smoke()`` check of the build entry point and the
``cpu_baseline`` leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, tables, helpers or pre/post-processing); the only common
code is the seeded input generator in ``gen/``.

What it computes follows Sec. 2.1 of the paper (Eqs. dterm, k1eterm, k1d and
TDDFT_VEXX_TDA; Eqs. k2eterm and k2dterm for the operator of the Z-vector
equation, Eq. z-v-eq, solved by conjugate gradients as in Sec. 3.3), with the
readings listed in ``liouville.py`` and ``zvector.py``.  It is slow and
obviously correct: whole-box FFTs (a library primitive) for transforms and
Poisson solves, and plain numpy sums everywhere else.

Pins (tests/test_oracle_*.py) tie every function here to something other than
itself: brute-force direct DFTs, a real-space Coulomb sum, closed forms for
plane-wave orbitals, an FFT-free Casida assembly, Hermiticity, unitary
invariance of the exchange term, the alpha = 0 and c_K = 0 reductions, the
G = 0 eigenvalue shift and dense diagonalisation.
"""
from .planewave import (  # noqa: F401
    gvectors, gamma_inner, gamma_overlap, real_space, coefficients, coulomb_kernel, poisson,
)
from .liouville import (  # noqa: F401
    TERM_D, TERM_K1E, TERM_K1D, TERM_ALL, TERM_K2E, TERM_K2D, TERM_FULL, apply_liouville,
    apply_transition, transition_diagonal,
)
from .davidson import davidson, davidson_transition  # noqa: F401
from .adjoint import energy, grad_a, grad_occ  # noqa: F401
from .zvector import cg_inexact, solve_zvector_transition  # noqa: F401
