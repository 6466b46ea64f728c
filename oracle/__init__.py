"""FP64 CPU oracle for the low-rank MEG method (test infrastructure only).

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
import this package.  It shares no code with the HIP path.
"""
from .meg_oracle import *  # noqa: F401,F403
from .meg_oracle import __all__  # noqa: F401
