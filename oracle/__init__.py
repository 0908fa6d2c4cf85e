"""FP64 CPU oracle of the RI qsGW iteration.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package.  It shares no code with the HIP path.
"""
from .qsgw_oracle import *  # noqa: F401,F403
