"""MI355X (gfx950) Green's-function pixel-by-pixel greedy optimiser.

The product is the C-ABI library libgfo.so (include/gfo.h) built from the HIP
sources in csrc/; this package holds its ctypes binding (``_lib``), a job
wrapper that owns the device buffers (``job``), the autotuner and the
serving loop.  Importing the package does not need a GPU; calling into the
library does, and fails loudly if the library is not built.
"""
from . import _lib  # noqa: F401
from ._lib import GfoError  # noqa: F401

__all__ = ["_lib", "GfoError"]
