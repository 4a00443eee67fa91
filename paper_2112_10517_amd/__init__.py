"""MI355X (gfx950) flux-differencing LGL-DGSEM for the compressible Euler equations.

The method of Ranocha et al. (arXiv:2112.10517) behind a C ABI
(``include/esdg.h``) implemented in hand-written HIP (``csrc/``); this package
holds the ctypes binding (``esdg``), the in-tree build (``build``) and the
seeded synthetic inputs (``inputs``).  The library is loaded lazily.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "esdg", "build"]
