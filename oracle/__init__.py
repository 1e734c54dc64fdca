"""CPU reference (oracle) for the short-range MD hot path.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the library.  Shares no code with the
GPU implementation.
"""
from .oracle import *  # noqa: F401,F403
