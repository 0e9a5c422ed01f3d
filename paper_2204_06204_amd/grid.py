"""Python binding of the C ABI (include/fbto.h): one method per entry point,
same names, argument marshalling only.  Tensors are torch tensors on the HIP
device; torch supplies device memory and the current stream, every step of
the computation runs in libfbto.so.

Precision follows the tensors' dtype: float64 -> FBTO_F64, float32 -> FBTO_F32.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import FbtoError, check


def _prec(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return _lib.FBTO_F64
    if t.dtype == torch.float32:
        return _lib.FBTO_F32
    raise TypeError(f"unsupported dtype {t.dtype} (float32 or float64)")


def _ptr(t: Optional[torch.Tensor], dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} entries, expected {numel}")
    return C.c_void_p(t.data_ptr())


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Grid:
    """A structured hex8 voxel grid with supports and springs (fbto_setup_grid)."""

    def __init__(self, nx: int, ny: int, nz: int, *, fixed_mask: Optional[np.ndarray] = None,
                 springs: Sequence[Tuple[int, float]] = (), young: float = 1.0,
                 poisson: float = 0.3, penal: float = 3.0, rho_min: float = 1e-3,
                 filter_radius: float = 1.5, max_rhs: int = 1):
        self.lib = _lib.load()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.E = self.nx * self.ny * self.nz
        self.N = (self.nx + 1) * (self.ny + 1) * (self.nz + 1)
        self.ndof = 3 * self.N
        self.max_rhs = int(max_rhs)
        desc = _lib.GridDesc(self.nx, self.ny, self.nz, self.max_rhs, young, poisson, penal,
                             rho_min, filter_radius)
        mask_p = None
        if fixed_mask is not None:
            m = np.ascontiguousarray(np.asarray(fixed_mask, dtype=np.uint8))
            if m.size != self.ndof:
                raise ValueError("fixed_mask must have 3N entries")
            self._mask = m
            mask_p = m.ctypes.data_as(C.c_void_p)
        dof = np.ascontiguousarray([s[0] for s in springs], dtype=np.int64)
        kk = np.ascontiguousarray([s[1] for s in springs], dtype=np.float64)
        self._springs = (dof, kk)
        h = C.c_void_p()
        check(self.lib.fbto_setup_grid(C.byref(desc), mask_p, len(dof),
                                       dof.ctypes.data_as(C.c_void_p) if len(dof) else None,
                                       kk.ctypes.data_as(C.c_void_p) if len(dof) else None,
                                       C.byref(h)), self.lib)
        self.handle = h

    @classmethod
    def from_problem(cls, p, max_rhs: Optional[int] = None) -> "Grid":
        return cls(p.nx, p.ny, p.nz, fixed_mask=p.fixed_mask, springs=p.springs, young=p.young,
                   poisson=p.poisson, penal=p.penal, rho_min=p.rho_min,
                   filter_radius=p.filter_radius, max_rhs=max_rhs or p.nrhs)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fbto_destroy_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def grid_sizes(self):
        e, n, d = C.c_int64(), C.c_int64(), C.c_int64()
        check(self.lib.fbto_grid_sizes(self.handle, C.byref(e), C.byref(n), C.byref(d)), self.lib)
        return e.value, n.value, d.value

    # ------------------------------------------------------------------
    def _nrhs(self, v: torch.Tensor) -> int:
        if v.numel() % self.ndof:
            raise ValueError(f"vector length must be a multiple of {self.ndof} (the DOF count)")
        return v.numel() // self.ndof

    def apply_K(self, rho: torch.Tensor, u: torch.Tensor, y: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
        if y is None:
            y = torch.empty_like(u)
        nr = self._nrhs(u)
        check(self.lib.fbto_apply_K(self.handle, _prec(u), _ptr(rho, u.dtype, self.E, "rho"),
                                    _ptr(u, name="u"), _ptr(y, u.dtype, u.numel(), "y"), nr,
                                    _stream(stream)), self.lib)
        return y

    def inner_solve(self, rho, f, u, steps: int, method: str = "pcg", omega: float = 0.0,
                    rtol: float = 0.0, info: Optional[torch.Tensor] = None, stream=None):
        meth = {"pcg": _lib.FBTO_PCG_JACOBI, "richardson": _lib.FBTO_RICHARDSON,
                "jacobi": _lib.FBTO_DAMPED_JACOBI, "krylov": _lib.FBTO_KRYLOV}[method]
        nr = self._nrhs(u)
        check(self.lib.fbto_inner_solve(self.handle, _prec(u), _ptr(rho, u.dtype, self.E, "rho"),
                                        _ptr(f, u.dtype, u.numel(), "f"), _ptr(u, name="u"), nr,
                                        meth, int(steps), float(omega), float(rtol),
                                        _ptr(info, torch.float64, None, "info"), _stream(stream)),
              self.lib)
        return u

    def solve_refined(self, rho64, f64, u64, rtol: float, max_refine: int, inner_steps: int,
                      inner_dtype=torch.float32, inner_rtol: float = 0.0,
                      info: Optional[torch.Tensor] = None, stream=None):
        prec = _lib.FBTO_F32 if inner_dtype == torch.float32 else _lib.FBTO_F64
        nr = self._nrhs(u64)
        nref = C.c_int32(0)
        check(self.lib.fbto_solve_refined(self.handle, prec, _ptr(rho64, torch.float64, self.E, "rho"),
                                          _ptr(f64, torch.float64, u64.numel(), "f"),
                                          _ptr(u64, torch.float64, None, "u"), nr, float(rtol),
                                          int(max_refine), int(inner_steps), float(inner_rtol),
                                          _ptr(info, torch.float64, None, "info"), C.byref(nref),
                                          _stream(stream)), self.lib)
        return nref.value

    def sensitivity(self, rho, u, lam=None, f=None, dobj=None, obj=None, stream=None):
        if dobj is None:
            dobj = torch.empty(self.E, dtype=u.dtype, device=u.device)
        nr = self._nrhs(u)
        check(self.lib.fbto_sensitivity(self.handle, _prec(u), _ptr(rho, u.dtype, self.E, "rho"),
                                        _ptr(u, name="u"), _ptr(lam, u.dtype, u.numel(), "lam"),
                                        _ptr(f, u.dtype, u.numel(), "f"), nr,
                                        _ptr(dobj, u.dtype, self.E, "dobj"),
                                        _ptr(obj, torch.float64, None, "obj"), _stream(stream)),
              self.lib)
        return dobj

    def filter(self, x, out=None, transpose: bool = False, stream=None):
        if out is None:
            out = torch.empty_like(x)
        check(self.lib.fbto_filter(self.handle, _prec(x), 1 if transpose else 0,
                                   _ptr(x, None, self.E, "in"), _ptr(out, x.dtype, self.E, "out"),
                                   _stream(stream)), self.lib)
        return out

    def project_volume(self, y, x=None, lo: float = 0.0, hi: float = 1.0, vmax: float = None,
                       lam: Optional[torch.Tensor] = None, stream=None, method: str = "newton",
                       max_passes: int = 0, status: Optional[torch.Tensor] = None):
        """method "newton": fbto_project_volume (passes of a safeguarded
        Newton search on the multiplier, at most `max_passes`, 0 = the
        library's default; `status` receives 0, FBTO_INEXACT or
        FBTO_ERR_NONFINITE); "sort": fbto_project_volume_sorted (Alg. 4 by
        radix sort and scans; exact, no status)."""
        if x is None:
            x = torch.empty_like(y)
        if method == "newton":
            check(self.lib.fbto_project_volume(
                self.handle, _prec(y), _ptr(y, None, self.E, "y"), _ptr(x, y.dtype, self.E, "x"),
                float(lo), float(hi), float(vmax), int(max_passes),
                _ptr(lam, torch.float64, None, "lambda"), _ptr(status, torch.float64, None, "status"),
                _stream(stream)), self.lib)
        elif method == "sort":
            if max_passes or status is not None:
                raise ValueError("max_passes and status belong to the Newton projection")
            check(self.lib.fbto_project_volume_sorted(
                self.handle, _prec(y), _ptr(y, None, self.E, "y"), _ptr(x, y.dtype, self.E, "x"),
                float(lo), float(hi), float(vmax), _ptr(lam, torch.float64, None, "lambda"),
                _stream(stream)), self.lib)
        else:
            raise ValueError(f"unknown method {method!r}")
        return x

    def optimality(self, x, u, f, alpha: float, lo: float, vmax: float, rtol: float = 1e-8,
                   max_steps: int = 100000, out: Optional[torch.Tensor] = None, stream=None):
        """fbto_optimality: FP64 [5] = l(x), Delta^v, Delta, relative residual
        of the exact solve, status."""
        if out is None:
            out = torch.zeros(5, dtype=torch.float64, device=x.device)
        nr = self._nrhs(u)
        check(self.lib.fbto_optimality(self.handle, _prec(x), _ptr(x, None, self.E, "x"),
                                       _ptr(u, x.dtype, None, "u"), _ptr(f, x.dtype, u.numel(), "f"), nr,
                                       float(alpha), float(lo), float(vmax), float(rtol), int(max_steps),
                                       _ptr(out, torch.float64, None, "out"), _stream(stream)), self.lib)
        return out

    def set_option(self, option: str, value: int):
        """fbto_set_option: "proj_passes", "apply_tile" or "cgf_tile"."""
        opt = {"proj_passes": _lib.FBTO_OPT_PROJ_PASSES, "apply_tile": _lib.FBTO_OPT_APPLY_TILE,
               "cgf_tile": _lib.FBTO_OPT_CGF_TILE}[option]
        check(self.lib.fbto_set_option(self.handle, opt, int(value)), self.lib)

    def outer_step(self, x, u, f, k: int, alpha0: float, inner_steps: int, lo: float, vmax: float,
                   mean_project: bool = True, info: Optional[torch.Tensor] = None, stream=None,
                   method: str = "pcg", beta: float = 1.0, rtol: float = 1e-8):
        """method "pcg": Alg. 1 with `inner_steps` Jacobi-PCG steps
        (fbto_outer_step); "krylov": Alg. 3 with one Krylov-preconditioned
        step of degree `inner_steps` and step `beta` (fbto_outer_step_krylov);
        "exact": projected gradient descent with the low-level problem solved
        to `rtol` in at most `inner_steps` PCG steps (fbto_outer_step_exact)."""
        nr = self._nrhs(u)
        common = (self.handle, _prec(x), _ptr(x, None, self.E, "x"), _ptr(u, x.dtype, None, "u"),
                  _ptr(f, x.dtype, u.numel(), "f"), nr, int(k), float(alpha0))
        tail = (1 if mean_project else 0, float(lo), float(vmax), _ptr(info, torch.float64, None, "info"),
                _stream(stream))
        if method == "pcg":
            check(self.lib.fbto_outer_step(*common, int(inner_steps), *tail), self.lib)
        elif method == "krylov":
            check(self.lib.fbto_outer_step_krylov(*common, int(inner_steps), float(beta), *tail), self.lib)
        elif method == "exact":
            check(self.lib.fbto_outer_step_exact(*common, float(rtol), int(inner_steps), *tail), self.lib)
        else:
            raise ValueError(f"unknown method {method!r}")
        return x


    def outer_steps(self, x, u, f, k: int, n_steps: int, alpha0: float, inner_steps: int, lo: float, vmax: float,
                    mean_project: bool = True, info: Optional[torch.Tensor] = None, stream=None):
        """Outer iterations k .. k + n_steps - 1 of Alg. 1 in one call
        (fbto_outer_steps): the results of n_steps outer_step calls.  info:
        float64 [n_steps * 8], one record per iteration."""
        nr = self._nrhs(u)
        if info is not None and info.numel() < 8 * int(n_steps):
            raise ValueError("info needs 8 values per iteration")
        check(self.lib.fbto_outer_steps(self.handle, _prec(x), _ptr(x, None, self.E, "x"), _ptr(u, x.dtype, None, "u"),
                                        _ptr(f, x.dtype, u.numel(), "f"), nr, int(k), int(n_steps), float(alpha0),
                                        int(inner_steps), 1 if mean_project else 0, float(lo), float(vmax),
                                        _ptr(info, torch.float64, None, "info"), _stream(stream)), self.lib)
        return x


class PlaneGrid(Grid):
    """A plane grid of nx x ny Q4 elements with the separable Gaussian filter
    (fbto_setup_grid_2d); vectors are [nrhs][2N].  Every method of Grid
    applies to it."""

    def __init__(self, nx: int, ny: int, *, fixed_mask: Optional[np.ndarray] = None, young: float = 1.0,
                 poisson: float = 0.3, penal: float = 3.0, rho_min: float = 0.0, filter_half: int = 3,
                 filter_sigma: float = 1.4, max_rhs: int = 1):
        self.lib = _lib.load()
        self.nx, self.ny, self.nz = int(nx), int(ny), 1
        self.E = self.nx * self.ny
        self.N = (self.nx + 1) * (self.ny + 1)
        self.ndof = 2 * self.N
        self.max_rhs = int(max_rhs)
        desc = _lib.Grid2DDesc(self.nx, self.ny, self.max_rhs, int(filter_half), young, poisson, penal,
                               rho_min, filter_sigma)
        mask_p = None
        if fixed_mask is not None:
            m = np.ascontiguousarray(np.asarray(fixed_mask, dtype=np.uint8))
            if m.size != self.ndof:
                raise ValueError("fixed_mask must have 2N entries")
            self._mask = m
            mask_p = m.ctypes.data_as(C.c_void_p)
        h = C.c_void_p()
        check(self.lib.fbto_setup_grid_2d(C.byref(desc), mask_p, C.byref(h)), self.lib)
        self.handle = h

    @classmethod
    def from_problem(cls, p, max_rhs: Optional[int] = None) -> "PlaneGrid":
        return cls(p.nx, p.ny, fixed_mask=p.fixed_mask, young=p.young, poisson=p.poisson, penal=p.penal,
                   rho_min=p.rho_min, filter_half=p.filter_half, filter_sigma=p.filter_sigma,
                   max_rhs=max_rhs or p.nrhs)


__all__ = ["Grid", "PlaneGrid", "FbtoError"]


def project_volume_noalloc(y: torch.Tensor, x: Optional[torch.Tensor] = None, lo: float = 0.0,
                           hi: float = 1.0, vmax: float = None, max_passes: int = 0,
                           lam: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None,
                           stream=None) -> torch.Tensor:
    """fbto_project_volume_noalloc: the projection of Grid.project_volume
    (method "newton") without a grid handle and without device allocation
    in the library; its workspace is a static device array shared by every
    call on the GPU (calls that overlap on one GPU race)."""
    lib = _lib.load()
    if x is None:
        x = torch.empty_like(y)
    n = y.numel()
    check(lib.fbto_project_volume_noalloc(
        _prec(y), n, _ptr(y, None, n, "y"), _ptr(x, y.dtype, n, "x"), float(lo), float(hi), float(vmax),
        int(max_passes), _ptr(lam, torch.float64, None, "lambda"), _ptr(status, torch.float64, None, "status"),
        _stream(stream)), lib)
    return x
