"""MI355X Blind-Match: encrypted 1:N biometric matching (CKKS) on gfx950.

The computation lives in libblindmatch.so (hand-written HIP kernels behind the
C ABI declared in include/blindmatch.h).  This package is its thin Python
binding: `binding` exposes every C entry point under its own name.
"""
from .binding import *  # noqa: F401,F403
from .binding import lib, declared_symbols, BMError, LIB_PATH  # noqa: F401
