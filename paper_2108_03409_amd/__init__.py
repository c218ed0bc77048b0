"""MI355X-native hot path of neural-quantum-state variational Monte Carlo.

The compute lives in libnqsvmc.so (HIP kernels for gfx950, C ABI in
include/nqsvmc.h); ``nqsvmc`` is its ctypes binding.
"""
from . import nqsvmc  # noqa: F401

__all__ = ["nqsvmc"]
