"""ctypes declarations of the C ABI in include/fbto.h (marshalling only).

The shared library is built in-tree (``paper_2204_06204_amd/libfbto.so``)
by ``paper_2204_06204_amd.build.build()``.  Loading fails loudly when it is
missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfbto.so")

FBTO_OK, FBTO_ERR_ARG, FBTO_ERR_ALLOC, FBTO_ERR_HIP = 0, 1, 2, 3
FBTO_ERR_INFEASIBLE, FBTO_ERR_BREAKDOWN, FBTO_ERR_NONFINITE, FBTO_ERR_UNSUPPORTED = 4, 5, 6, 7
FBTO_INEXACT = 8
FBTO_OPT_PROJ_PASSES, FBTO_OPT_APPLY_TILE, FBTO_OPT_CGF_TILE = 0, 1, 2
FBTO_F64, FBTO_F32 = 0, 1
FBTO_PCG_JACOBI, FBTO_RICHARDSON, FBTO_DAMPED_JACOBI, FBTO_KRYLOV = 0, 1, 2, 3
FBTO_SOLVE_INFO = 8
FBTO_NOALLOC_MAX_ELEMS = 2147483647
FBTO_OUTER_INFO = 8
SI = dict(rnorm2=0, rnormi=1, fnorm2=2, steps=3, status=4)
OI = dict(compliance=0, dx_inf=1, r_inf=2, lam=3, volume=4, rrel=5, status=6, grad_mean=7)


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("max_rhs", C.c_int32),
                ("young", C.c_double), ("poisson", C.c_double), ("penal", C.c_double),
                ("rho_min", C.c_double), ("filter_radius", C.c_double)]


class Grid2DDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("max_rhs", C.c_int32), ("filter_half", C.c_int32),
                ("young", C.c_double), ("poisson", C.c_double), ("penal", C.c_double),
                ("rho_min", C.c_double), ("filter_sigma", C.c_double)]


_VP = C.c_void_p
_SIGS = {
    "fbto_setup_grid": (C.c_int, [C.POINTER(GridDesc), _VP, C.c_int32, _VP, _VP, C.POINTER(_VP)]),
    "fbto_setup_grid_2d": (C.c_int, [C.POINTER(Grid2DDesc), _VP, C.POINTER(_VP)]),
    "fbto_destroy_grid": (C.c_int, [_VP]),
    "fbto_grid_sizes": (C.c_int, [_VP, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "fbto_apply_K": (C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_int32, _VP]),
    "fbto_inner_solve": (C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_int32, C.c_int, C.c_int32,
                                   C.c_double, C.c_double, _VP, _VP]),
    "fbto_solve_refined": (C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_int32, C.c_double, C.c_int32,
                                     C.c_int32, C.c_double, _VP, C.POINTER(C.c_int32), _VP]),
    "fbto_sensitivity": (C.c_int, [_VP, C.c_int, _VP, _VP, _VP, _VP, C.c_int32, _VP, _VP, _VP]),
    "fbto_filter": (C.c_int, [_VP, C.c_int, C.c_int32, _VP, _VP, _VP]),
    "fbto_project_volume": (C.c_int, [_VP, C.c_int, _VP, _VP, C.c_double, C.c_double, C.c_double,
                                      C.c_int32, _VP, _VP, _VP]),
    "fbto_project_volume_sorted": (C.c_int, [_VP, C.c_int, _VP, _VP, C.c_double, C.c_double, C.c_double,
                                             _VP, _VP]),
    "fbto_outer_step": (C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_int32, C.c_int32, C.c_double,
                                  C.c_int32, C.c_int32, C.c_double, C.c_double, _VP, _VP]),
    "fbto_outer_steps": (C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                   C.c_int32, C.c_int32, C.c_double, C.c_double, _VP, _VP]),
    "fbto_outer_step_exact": (C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_int32, C.c_int32, C.c_double,
                                        C.c_double, C.c_int32, C.c_int32, C.c_double, C.c_double, _VP, _VP]),
    "fbto_outer_step_krylov": (C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_int32, C.c_int32, C.c_double,
                                         C.c_int32, C.c_double, C.c_int32, C.c_double, C.c_double, _VP, _VP]),
    "fbto_project_volume_noalloc": (C.c_int, [C.c_int, C.c_int64, _VP, _VP, C.c_double, C.c_double,
                                              C.c_double, C.c_int32, _VP, _VP, _VP]),
    "fbto_optimality": (C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_int32, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_int32, _VP, _VP]),
    "fbto_set_option": (C.c_int, [_VP, C.c_int, C.c_int64]),
    "fbto_last_error": (C.c_char_p, []),
    "fbto_version": (C.c_char_p, []),
}

EXPORTED = tuple(_SIGS)

_lib = None


class FbtoError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"fbto status {status}: {message}")
        self.status = status


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libfbto.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with paper_2204_06204_amd.build.build() "
                          "(there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


def check(status: int, lib=None):
    if status != FBTO_OK:
        lib = lib or load()
        raise FbtoError(status, lib.fbto_last_error().decode())
