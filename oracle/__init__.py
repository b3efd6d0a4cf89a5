"""Plain FP64 CPU oracle of the DG shallow-water step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The product path (the HIP library and its binding) never does.
"""
from .oracle import Oracle, build_oracle, load_oracle  # noqa: F401
