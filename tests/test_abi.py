"""The C-ABI library: it loads, exports every entry point include/cbct.h declares, and
rejects invalid arguments on the host before touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1001_0599_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "cbct.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cbct_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_functions()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.exported_names()) == names


def test_status_strings():
    L = _lib.lib()
    for k, v in _lib.STATUS_NAMES.items():
        assert L.cbct_status_string(k).decode() == v


def _desc(**kw):
    d = dict(nx=32, ny=32, nz=32, hx=2.0, hy=2.0, hz=2.0, nu=64, nv=64, pu=1.5, pv=1.5, sad=1000.0, sdd=1500.0,
             n_views=16, angles=None, sample_ratio=1.0)
    d.update(kw)
    return _lib.GeometryDesc(**d)


@pytest.mark.parametrize("bad", [dict(nx=0), dict(pu=-1.0), dict(sdd=900.0), dict(sad=10.0), dict(n_views=0),
                                 dict(nv=4096)])
def test_plan_rejects_bad_geometry(bad):
    L = _lib.lib()
    h = C.c_void_p()
    st = L.cbct_plan_create(None, C.byref(_desc(**bad)), 1, 1, C.byref(h))
    assert st == 1 and not h.value
    assert L.cbct_last_error()


def test_plan_rejects_indivisible_levels():
    L = _lib.lib()
    h = C.c_void_p()
    assert L.cbct_plan_create(None, C.byref(_desc(nx=30)), 3, 1, C.byref(h)) == 1
    assert b"divisible" in L.cbct_last_error()
    assert L.cbct_plan_create(None, None, 1, 1, C.byref(h)) == 1


def test_plan_and_server_need_a_context():
    # a valid geometry without a context is rejected before any device is touched
    L = _lib.lib()
    h = C.c_void_p()
    assert L.cbct_plan_create(None, C.byref(_desc()), 1, 1, C.byref(h)) == 1
    assert b"context" in L.cbct_last_error() and not h.value
    assert L.cbct_server_create(None, C.c_size_t(1 << 30), 2, C.byref(h)) == 1
    assert not h.value


def test_context_rejects_bad_device():
    L = _lib.lib()
    h = C.c_void_p()
    assert L.cbct_context_create(-1, C.byref(h)) == 1 and not h.value
    assert L.cbct_context_create(1 << 20, C.byref(h)) == 1 and not h.value
    assert L.cbct_context_create(0, None) == 1
    d = C.c_int()
    assert L.cbct_context_device(None, C.byref(d)) == 1
    L.cbct_context_destroy(None)  # a no-op


def test_calls_reject_null_plan():
    L = _lib.lib()
    assert L.cbct_forward(None, 0, None, None, None, 0, None) == 1
    assert L.cbct_adjoint(None, 0, None, None, None, 0, None) == 1
    assert L.cbct_backproject_eq6(None, 0, None, None, None) == 1
    assert L.cbct_forward_siddon(None, 0, None, None, None, 0, None) == 1
    assert L.cbct_adjoint_siddon(None, 0, None, None, None, 0, None) == 1
    n = C.c_size_t()
    assert L.cbct_forward_workspace_size(None, 0, C.byref(n)) == 1
