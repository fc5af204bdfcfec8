"""Plain, slow FP64 CPU oracle for the algebraic multilevel overlapping Schwarz
preconditioner (Al Daas & Jolivet, "A robust algebraic multilevel domain
decomposition preconditioner for sparse SPD matrices").

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU product path
never calls it and shares no code with it.
"""
from .dd_oracle import *  # noqa: F401,F403
