"""MI355X-native arrested Newton flow for 3D Skyrmions (arXiv:2604.25876).

The compute path is the HIP library libskyr.so (C ABI in include/skyr.h);
`skyr` is its thin ctypes binding.  Importing the package loads nothing; the
library is loaded on first use and a missing build is an error.
"""
from . import skyr  # noqa: F401

__all__ = ["skyr"]
