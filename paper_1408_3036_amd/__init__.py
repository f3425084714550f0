"""MI355X-native Sternheimer chi0 / Lanczos dielectric matrix (HIP for gfx950).

The compute runs in liblgw.so (hand-written HIP kernels behind a C ABI, see
include/lgw.h); this package only marshals torch tensors into that ABI.
"""
from .lgw import (Lgw, LgwError, chi0_apply_many, load_library, library_path, STATUS, FLAG_CONV,
                  FLAG_BREAK, FLAG_MAXIT)

__all__ = ["Lgw", "LgwError", "chi0_apply_many", "load_library", "library_path", "STATUS", "FLAG_CONV",
           "FLAG_BREAK", "FLAG_MAXIT"]
