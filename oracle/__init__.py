"""FP64 CPU oracle of the differentiable simulation step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP path.
"""
from .oracle import Oracle, build, library_path  # noqa: F401
