"""Incoherent harmonic sum on MI355X (gfx950): HIP kernels behind a C ABI.

``hs`` is the ctypes binding of ``libhs.so`` (see ``include/hs.h``);
``ops`` allocates torch outputs around it.  Nothing here computes on the CPU:
without the built library every call raises.
"""
from . import hs  # noqa: F401
from .hs import HsError, Plan  # noqa: F401
