"""MI355X-native canonical k-mer counting (the counting step of Gerbil, arXiv 1607.06618).

The work runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/gerbil.h`` (``libgerbil.so``); ``gerbil`` is its ctypes binding.
"""
from . import gerbil  # noqa: F401

__all__ = ["gerbil"]
