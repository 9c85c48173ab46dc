"""MI355X-native progressive spatio-temporal filtering (PSTF) hash path.

The product is ``libpsf.so`` (C ABI declared in ``include/psf.h``), built from
the HIP sources in ``csrc/`` for gfx950; ``psf`` is its ctypes binding.
"""
from . import psf  # noqa: F401
from .psf import Batch, Table, load  # noqa: F401
