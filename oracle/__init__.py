"""FP64 CPU oracle for the SBV log-likelihood (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never links or calls it.
"""
from .oracle import *  # noqa: F401,F403
