"""MI355X (gfx950) Anderson acceleration with low-synchronization QR updates.

The compute path is the HIP library ``libaa.so`` (C ABI in ``include/aa.h``);
this package is its binding (``aa``) plus a convenience context class.  There
is no CPU fallback: if the library is not built the import of ``aa`` still
works but every call raises.
"""
from . import aa  # noqa: F401
from .aa import (AAContext, MGS, CGS2, DCGS2, ICWY, VARIANTS, AAError,  # noqa: F401
                 lib)

__all__ = ["aa", "AAContext", "MGS", "CGS2", "DCGS2", "ICWY", "VARIANTS", "AAError", "lib"]
