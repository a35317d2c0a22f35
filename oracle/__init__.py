"""CPU oracle of the DG S_N sweep and VEF-moment reduction (test infrastructure only).

Only the test-suite, the smoke entry point and the CPU-baseline leg of the
benchmark may import this package.  The HIP library never does.
"""
from .oracle import *  # noqa: F401,F403
