"""CPU oracle for the global-best PSO step (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library neither imports nor links it.
"""
from .oracle import *  # noqa: F401,F403
