"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *generates inputs* (geometries, sparsity patterns, random
angular factors, shift grids, quadrature weights and right-hand-side picks).
It holds none of the method's arithmetic, so the CPU oracle and the HIP path
can both consume it without sharing any computation.
"""
from .system import ASEDParams, TBSystem  # noqa: F401
from .grids import rhs_atoms, shift_grid, trapezoid_weights  # noqa: F401
from .silicon import si_bulk, si_crack_111, si_slab_001  # noqa: F401
from .water import water_box  # noqa: F401
from . import configs  # noqa: F401
