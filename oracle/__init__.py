"""Force2Vec CPU oracle (test infrastructure only).

Plain FP64 implementation of the paper's method in C (f2v_oracle.c), loaded
through ctypes.  Only tests, the smoke check and the benchmark's CPU-baseline
leg use it; the HIP product path never imports it.
"""
from .oracle import *  # noqa: F401,F403
from .oracle import __all__  # noqa: F401
