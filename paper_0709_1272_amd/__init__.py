"""tileqr: tiled Householder QR for AMD Instinct MI355X (gfx950).

The factorisation, its application to right-hand sides and the least-squares
solver run in hand-written HIP kernels behind the C-ABI library
``libtileqr.so`` (declared in ``include/tileqr.h``); ``tileqr`` is its thin
ctypes binding (imported on demand, so CPU-only users of ``synth`` never load
the HIP runtime).  ``synth`` draws the seeded synthetic inputs.
"""
import importlib

__all__ = ["tileqr", "synth"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
