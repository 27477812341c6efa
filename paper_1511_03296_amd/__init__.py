"""MI355X-native bilateral solver (Barron & Poole, "The Fast Bilateral Solver").

The solver runs as HIP kernels for gfx950 in ``libbsolve.so`` (C ABI in
``include/bsolve.h``); this package is its Python binding.  Importing it loads
the library and raises ImportError if it has not been built.
"""
from .solver import BilateralGrid, SolveOptions, bilateral_solve, read_stats  # noqa: F401

__all__ = ["BilateralGrid", "SolveOptions", "bilateral_solve", "read_stats"]
