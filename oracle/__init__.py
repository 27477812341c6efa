"""FP64 CPU oracle of the fast bilateral solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the test-suite, the smoke check and the benchmark's CPU-baseline leg do.
It shares no code with the HIP library.  ``bilateral`` is the matrix-free
solver in the paper's steps; ``dense`` builds the paper's matrices explicitly
for tiny images, to pin ``bilateral`` against the paper's equations.
"""
