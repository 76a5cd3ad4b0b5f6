"""CPU FP64 oracle for the reduced-basis warm-start solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  It is a plain, slow
restatement of what the method computes (see ``rbws_oracle.c`` for the C part
and ``mlp.py`` for the learned warm start) and shares no code with the HIP
library.
"""
from .core import *  # noqa: F401,F403
from . import mlp  # noqa: F401
