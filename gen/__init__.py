"""Seeded synthetic inputs for the Liouville-apply path.

This package is the only code shared by the GPU path's tests/benchmarks and the
CPU oracle.  It draws random numbers and prepares *inputs* (plane-wave sphere,
orthonormal orbital coefficients, eigenvalues, the f_xc field and trial blocks);
it contains none of the operator's arithmetic (no transforms of the method, no
Poisson kernel, no Liouville terms).
"""
from .systems import (  # noqa: F401
    Config, CONFIGS, System, half_sphere, make_system, trials_in_span,
    trials_random, plane_wave_pair_system, batch_configs,
)
