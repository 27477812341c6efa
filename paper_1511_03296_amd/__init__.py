"""MI355X-native bilateral solver (Barron & Poole, "The Fast Bilateral Solver").

The solver runs as HIP kernels for gfx950 in ``libbsolve.so`` (C ABI in
``include/bsolve.h``); this package is its Python binding.  The first use of
the API loads the library and raises ImportError if it has not been built
(``python -m paper_1511_03296_amd.build``).
"""
__all__ = ["BilateralGrid", "SolveOptions", "bilateral_solve", "read_stats", "BatchState",
           "BatchPlan", "bilateral_solve_batch", "domain_transform", "dt_confidence",
           "NotConverged", "require_converged"]


def __getattr__(name):
    if name in __all__:
        from . import solver
        return getattr(solver, name)
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
