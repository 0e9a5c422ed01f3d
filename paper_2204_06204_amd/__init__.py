"""MI355X-native matrix-free SIMP hot path (arXiv 2204.06204, first-order
bilevel topology optimization): hand-written HIP kernels for gfx950 behind
the C ABI of include/fbto.h, with a thin ctypes binding (grid.Grid) and a
torch.autograd adjoint (autograd)."""
from ._lib import FbtoError, load as load_library, LIB_PATH

__all__ = ["FbtoError", "load_library", "LIB_PATH", "Grid"]


def __getattr__(name):
    if name == "Grid":
        from .grid import Grid
        return Grid
    raise AttributeError(name)
