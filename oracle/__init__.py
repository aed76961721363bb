"""CPU oracle for the HOP hot path -- test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``hop_oracle.c`` (plain C, FP64, no
contraction) through ctypes and adds an FP64 NumPy reference for the
learned-radius network.  Nothing here is shared with the GPU path.
"""
from .oracle import *  # noqa: F401,F403
from .oracle import __all__  # noqa: F401
