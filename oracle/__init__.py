"""CPU FP64 oracle for HBMC-ordered IC(0)-CG.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  See ``oracle.core``.
"""
from .core import *  # noqa: F401,F403
