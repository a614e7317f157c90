"""FP64 CPU oracle for FCC / GCC-PHAT TDoA (test infrastructure only).

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg import this package.  The GPU library never calls it, and it shares no
code with the GPU path.
"""
from .fcc_oracle import *  # noqa: F401,F403
from .fcc_oracle import __all__  # noqa: F401
