"""CPU oracle of the LES residual, RK5 step and pressure functional (plain
FP64 NumPy).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the package smoke check
and the benchmark's CPU-baseline leg, never by the GPU library, with which it
shares no code.
"""
from . import brute, functional, les  # noqa: F401
