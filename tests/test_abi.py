"""The C-ABI library loads and exports every function include/idp.h declares;
host-side argument checks answer without a GPU (no device calls here)."""
import ctypes as C
import os
import re

import pytest

from paper_2007_00094_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "idp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(idp_\w+)\s*\(",
                                 text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("idp_create", "idp_step", "idp_max_dt", "idp_destroy",
                     "idp_export_matrices", "idp_debug_export"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = capi.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert name in capi.SIGNATURES, name


def test_strerror_and_defaults_on_host():
    L = capi.lib()
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert L.idp_strerror(code)
    p = capi.idp_params()
    assert L.idp_default_params(C.byref(p), 3) == 0
    assert (p.dim, p.gamma, p.cfl, p.limiter_passes, p.newton_max_iter) == (3, 1.4, 0.5, 2, 2)
    assert p.newton_tol == 1e-10 and p.relax_bounds == 0 and p.flags == 0
    assert L.idp_default_params(C.byref(p), 4) == capi.IDP_EINVAL


@pytest.mark.parametrize("field,value,code", [
    ("dim", 4, capi.IDP_EINVAL), ("cfl", 1.5, capi.IDP_EINVAL),
    ("gamma", 1.0, capi.IDP_EINVAL), ("limiter_passes", 3, capi.IDP_EINVAL),
    ("relax_bounds", 2, capi.IDP_EINVAL)])
def test_create_rejects_bad_params_before_any_device_call(field, value, code):
    L = capi.lib()
    p = capi.idp_params()
    L.idp_default_params(C.byref(p), 2)
    setattr(p, field, value)
    h = C.c_void_p()
    xy = (C.c_double * 8)()
    cells = (C.c_int64 * 4)(0, 1, 2, 3)
    assert L.idp_create(C.byref(h), C.byref(p), 4, xy, 1, cells, None, None) == code
    assert L.idp_create(None, C.byref(p), 4, xy, 1, cells, None, None) == capi.IDP_EINVAL
    assert L.idp_step(None, None, 0.0, None) == capi.IDP_EINVAL
    assert L.idp_max_dt(None, None, None) == capi.IDP_EINVAL


def test_create_rejects_an_empty_mesh_before_any_device_call():
    L = capi.lib()
    p = capi.idp_params()
    L.idp_default_params(C.byref(p), 2)
    h = C.c_void_p()
    xy = (C.c_double * 8)()
    cells = (C.c_int64 * 4)(0, 1, 2, 3)
    assert L.idp_create(C.byref(h), C.byref(p), 0, xy, 1, cells, None, None) == capi.IDP_EINVAL
    assert L.idp_create(C.byref(h), C.byref(p), 4, xy, 0, cells, None, None) == capi.IDP_EINVAL
    assert not h.value


def test_create_batch_rejects_bad_arguments_before_any_device_call():
    L = capi.lib()
    p = capi.idp_params()
    L.idp_default_params(C.byref(p), 2)
    h = C.c_void_p()
    xy = (C.c_double * 8)()
    cells = (C.c_int64 * 4)(0, 1, 2, 3)
    co = (capi._dp * 1)(C.cast(xy, capi._dp))
    ce = (capi._i64p * 1)(C.cast(cells, capi._i64p))
    nn = (C.c_int64 * 1)(4)
    nc = (C.c_int64 * 1)(1)
    assert L.idp_create_batch(C.byref(h), C.byref(p), 0, nn, co, nc, ce, None, None) == capi.IDP_EINVAL
    p.flags = capi.IDP_FLAG_RENUMBER   # single meshes only
    assert L.idp_create_batch(C.byref(h), C.byref(p), 1, nn, co, nc, ce, None, None) == capi.IDP_ENOTSUP
    p.flags = 0
    assert L.idp_create_batch(None, C.byref(p), 1, nn, co, nc, ce, None, None) == capi.IDP_EINVAL
    assert L.idp_create_batch(C.byref(h), C.byref(p), 1, None, co, nc, ce, None, None) == capi.IDP_EINVAL
    bad = (C.c_int64 * 1)(0)
    assert L.idp_create_batch(C.byref(h), C.byref(p), 1, bad, co, nc, ce, None, None) == capi.IDP_EINVAL
    p.cfl = 2.0
    assert L.idp_create_batch(C.byref(h), C.byref(p), 1, nn, co, nc, ce, None, None) == capi.IDP_EINVAL
    assert L.idp_batch_steps(None, None, 1, None, None, None) == capi.IDP_EINVAL
    assert L.idp_batch_tune(None, None, 1, None, None, None) == capi.IDP_EINVAL
    assert L.idp_batch_max_dt(None, None, None) == capi.IDP_EINVAL
    assert L.idp_batch_info(None, None, None) == capi.IDP_EINVAL


def test_batch_create_refuses_relaxed_bounds_before_any_device_call():
    """The relaxation of the bounds is for single meshes only."""
    L = capi.lib()
    p = capi.idp_params()
    L.idp_default_params(C.byref(p), 2)
    p.relax_bounds = 1
    h = C.c_void_p()
    xy = (C.c_double * 8)(0, 0, 1, 0, 0, 1, 1, 1)
    cells = (C.c_int64 * 4)(0, 1, 2, 3)
    nn = (C.c_int64 * 1)(4)
    nc = (C.c_int64 * 1)(1)
    co = (C.POINTER(C.c_double) * 1)(C.cast(xy, C.POINTER(C.c_double)))
    ce = (C.POINTER(C.c_int64) * 1)(C.cast(cells, C.POINTER(C.c_int64)))
    assert L.idp_create_batch(C.byref(h), C.byref(p), 1, nn, co, nc, ce, None, None) == \
        capi.IDP_ENOTSUP
