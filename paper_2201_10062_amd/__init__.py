"""MI355X (gfx950) sine-transform-preconditioned MINRES for all-at-once heat-equation
systems (Hon, Fung, Dong, Serra-Capizzano, arXiv 2201.10062).

The solver lives in libsmr.so (HIP kernels + C ABI, include/smr.h); ``smr`` is its
ctypes binding.
"""
from . import smr  # noqa: F401
from .smr import Batch, Plan, SmrError, load, solve_batched  # noqa: F401

__all__ = ["smr", "Batch", "Plan", "SmrError", "load", "solve_batched"]
