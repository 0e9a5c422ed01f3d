"""CPU-side checks of the C ABI: the library loads without a GPU, exports
every function include/fbto.h declares, and rejects invalid arguments on
the host before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fbto.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fbto_[A-Za-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2204_06204_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2204_06204_amd.build import build
        build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("fbto_setup_grid", "fbto_apply_K", "fbto_inner_solve", "fbto_sensitivity",
              "fbto_filter", "fbto_project_volume", "fbto_outer_step", "fbto_solve_refined",
              "fbto_outer_step_krylov", "fbto_outer_step_exact", "fbto_destroy_grid", "fbto_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2204_06204_amd import _lib
    names = declared_functions()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(_lib.EXPORTED)


def test_host_side_argument_errors(lib):
    from paper_2204_06204_amd import _lib
    h = C.c_void_p()
    bad = [
        _lib.GridDesc(0, 4, 4, 1, 1.0, 0.3, 3.0, 1e-3, 1.5),      # empty axis
        _lib.GridDesc(4, 4, 4, 5, 1.0, 0.3, 3.0, 1e-3, 1.5),      # max_rhs
        _lib.GridDesc(4, 4, 4, 1, -1.0, 0.3, 3.0, 1e-3, 1.5),     # young
        _lib.GridDesc(4, 4, 4, 1, 1.0, 0.5, 3.0, 1e-3, 1.5),      # poisson
        _lib.GridDesc(4, 4, 4, 1, 1.0, 0.3, 0.5, 1e-3, 1.5),      # penal
        _lib.GridDesc(4, 4, 4, 1, 1.0, 0.3, 3.0, 1.0, 1.5),       # rho_min
        _lib.GridDesc(4, 4, 4, 1, 1.0, 0.3, 3.0, 1e-3, -2.0),     # radius
    ]
    for d in bad:
        assert lib.fbto_setup_grid(C.byref(d), None, 0, None, None, C.byref(h)) == _lib.FBTO_ERR_ARG
        assert lib.fbto_last_error().decode() != ""
        assert not h.value
    d = _lib.GridDesc(4, 4, 4, 1, 1.0, 0.3, 3.0, 1e-3, 1.5)
    assert lib.fbto_setup_grid(C.byref(d), None, 2, None, None, C.byref(h)) == _lib.FBTO_ERR_ARG
    assert lib.fbto_setup_grid(None, None, 0, None, None, C.byref(h)) == _lib.FBTO_ERR_ARG
    # spring DOF out of range
    dof = (C.c_int64 * 1)(10 ** 9)
    kk = (C.c_double * 1)(0.1)
    assert lib.fbto_setup_grid(C.byref(d), None, 1, dof, kk, C.byref(h)) == _lib.FBTO_ERR_ARG
    # calls on a NULL handle
    assert lib.fbto_apply_K(None, 0, None, None, None, 1, None) == _lib.FBTO_ERR_ARG
    assert lib.fbto_outer_step(None, 0, None, None, None, 1, 1, 0.1, 1, 1, 0.0, 1.0, None, None) == _lib.FBTO_ERR_ARG
    assert lib.fbto_outer_step_krylov(None, 0, None, None, None, 1, 1, 0.1, 20, 1.0, 1, 0.0, 1.0, None,
                                      None) == _lib.FBTO_ERR_ARG
    assert lib.fbto_outer_step_exact(None, 0, None, None, None, 1, 1, 0.1, 1e-8, 100, 1, 0.0, 1.0, None,
                                     None) == _lib.FBTO_ERR_ARG
    assert lib.fbto_project_volume(None, 0, None, None, 0.0, 1.0, 1.0, 0, None, None, None) == _lib.FBTO_ERR_ARG
    assert lib.fbto_set_option(None, _lib.FBTO_OPT_PROJ_PASSES, 4) == _lib.FBTO_ERR_ARG
    assert lib.fbto_version().decode().startswith("fbto")


def test_noalloc_projection_rejects_on_the_host(lib):
    """The allocation-free projection checks its arguments before any HIP
    call: sizes beyond its scratch's limit, empty inputs, bad budgets."""
    from paper_2204_06204_amd import _lib
    fake = C.c_void_p(0x1000)  # never dereferenced: every call below fails on the host
    big = _lib.FBTO_NOALLOC_MAX_ELEMS + 1
    assert lib.fbto_project_volume_noalloc(0, big, fake, fake, 0.0, 1.0, 1.0, 0, None, None,
                                           None) == _lib.FBTO_ERR_ARG
    assert "at most" in lib.fbto_last_error().decode()
    assert lib.fbto_project_volume_noalloc(0, 0, fake, fake, 0.0, 1.0, 1.0, 0, None, None,
                                           None) == _lib.FBTO_ERR_ARG
    assert lib.fbto_project_volume_noalloc(0, 10, None, fake, 0.0, 1.0, 1.0, 0, None, None,
                                           None) == _lib.FBTO_ERR_ARG
    assert lib.fbto_project_volume_noalloc(0, 10, fake, fake, 0.0, 1.0, 1.0, 65, None, None,
                                           None) == _lib.FBTO_ERR_ARG
    assert lib.fbto_project_volume_noalloc(7, 10, fake, fake, 0.0, 1.0, 1.0, 0, None, None,
                                           None) == _lib.FBTO_ERR_ARG
    assert lib.fbto_project_volume_noalloc(1, 10, fake, fake, 0.5, 1.0, 4.0, 0, None, None,
                                           None) == _lib.FBTO_ERR_INFEASIBLE


def test_plane_grid_host_errors(lib):
    from paper_2204_06204_amd import _lib
    h = C.c_void_p()
    bad = [
        _lib.Grid2DDesc(0, 4, 1, 3, 1.0, 0.3, 3.0, 0.0, 1.4),      # empty axis
        _lib.Grid2DDesc(4, 4, 5, 3, 1.0, 0.3, 3.0, 0.0, 1.4),      # max_rhs
        _lib.Grid2DDesc(4, 4, 1, 9, 1.0, 0.3, 3.0, 0.0, 1.4),      # window half-width
        _lib.Grid2DDesc(4, 4, 1, 3, 1.0, 0.3, 3.0, 0.0, 0.0),      # sigma
        _lib.Grid2DDesc(4, 4, 1, 3, 1.0, 0.5, 3.0, 0.0, 1.4),      # poisson
    ]
    for d in bad:
        assert lib.fbto_setup_grid_2d(C.byref(d), None, C.byref(h)) == _lib.FBTO_ERR_ARG
        assert lib.fbto_last_error().decode() != ""
        assert not h.value
    assert lib.fbto_setup_grid_2d(None, None, C.byref(h)) == _lib.FBTO_ERR_ARG
