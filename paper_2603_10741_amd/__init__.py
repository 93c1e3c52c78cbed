"""MI355X-native principal-cell operators for nonlinear hyperelastic lattices.

The compute path is the HIP library liblat.so (C ABI in include/lat.h); this package holds
its ctypes binding (`binding`), autograd wrappers (`autograd`) and the build step (`build`).
"""
from .binding import (BF16, F32, F64, RULE_FULL, RULE_REDUCED, LatError, Plan)  # noqa: F401

__all__ = ["Plan", "LatError", "RULE_FULL", "RULE_REDUCED", "F64", "F32", "BF16"]
