"""Seeded synthetic inputs for the wave-equation solves (source samples f^(0..nt-1)
and initial data psi_0, psi_1 on the interior grid).

This module is shared by the tests, the benchmark, the oracle side and the HIP side
as a pure input generator: it holds none of the solver's arithmetic (no operator,
no right-hand-side assembly, no transform of the method).
"""
from .workloads import (  # noqa: F401
    grid_points, manufactured_1d, manufactured_2d, random_source, gaussian_field_source,
    jacobi_smoothed_source, serving_trace, WORKLOADS,
)
