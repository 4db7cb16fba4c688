"""FP64 CPU oracle for the multi-mode difference-map iteration.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the package smoke check
and the benchmark's CPU-baseline leg, never by the GPU library.
"""
from . import dm_oracle  # noqa: F401
