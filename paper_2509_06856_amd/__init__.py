"""libslse: SLSE-FRS (Sequential Least-Squares Estimators with Fast Randomized
Sketching) on AMD Instinct MI355X.  The compute path is the HIP library
libslse.so (C ABI in include/slse.h); `slse` holds the PyTorch-facing wrappers
and `_lib` the ctypes binding.
"""
from . import _lib  # noqa: F401

__all__ = ["_lib", "slse"]
