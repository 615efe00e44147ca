"""FP64 CPU oracle (test infrastructure only; never called by the product path).

Only the test-suite, the GPU smoke check and the benchmark's CPU-baseline leg
may import this package.
"""
from .mf_oracle import *  # noqa: F401,F403
