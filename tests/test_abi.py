"""CPU checks of the C ABI library: it loads, exports every entry point the
public header declares, and rejects bad arguments on the host before any GPU
work (these calls never reach the device)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "debyefit.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(debye_\w+)\s*\(", src, flags=re.M)))


def test_header_and_binding_agree():
    import paper_2109_01928_amd as D
    assert _declared() == sorted(D.EXPORTED)


def test_library_exports_every_declared_symbol():
    import paper_2109_01928_amd as D
    L = D.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert L.debye_version().decode().startswith("debyefit")


def test_host_side_validation():
    import paper_2109_01928_amd as D
    L = D.lib()
    b = D._CBatch(0, 1, 10, 10, 1, 1, 1, 1, 1, 1)
    out = C.c_void_p()
    z = C.c_void_p(0)
    # n_mat < 1
    assert L.debye_plan_create(C.byref(b), z, z, z, 0, C.byref(out)) == D.ERANGE
    assert b"n_mat" in L.debye_last_error()
    # NULL plan
    b.n_mat = 1
    assert L.debye_fit_eval(None, C.byref(b), z, 1, 1e-8, 0, z, z, z, z, z) == D.EINVAL
    # too many poles
    b.max_poles = 25
    assert L.debye_plan_create(C.byref(b), z, z, z, 0, C.byref(out)) == D.ERANGE
    # basis: bad sizes and NULLs
    one = C.c_void_p(8)
    assert L.debye_basis(one, 0, one, 1, 1, 1, one, one, z) == D.ERANGE
    assert L.debye_basis(None, 5, one, 1, 1, 1, one, one, z) == D.EINVAL
    assert L.debye_basis(one, 5, one, 1, 1, 30, one, one, z) == D.ERANGE
    # material eval with no materials
    assert L.debye_material_eval(0, one, one, one, 5, one, 0, one, one, None, z) == D.ERANGE
    # host shape arrays inconsistent with the batch
    import numpy as np
    b = D._CBatch(2, 3, 10, 4, 8, 8, 8, 8, 8, 8)
    f = np.array([0, 5, 10], np.int64)
    c = np.array([0, 2, 4], np.int64)
    n = np.array([3, 4], np.int32)
    assert L.debye_plan_create(C.byref(b), f.ctypes.data_as(C.c_void_p), c.ctypes.data_as(C.c_void_p),
                               n.ctypes.data_as(C.c_void_p), 0, C.byref(out)) == D.EINVAL
    assert b"max_poles" in L.debye_last_error()
    f2 = np.array([0, 0, 10], np.int64)
    b.max_poles = 4
    assert L.debye_plan_create(C.byref(b), f2.ctypes.data_as(C.c_void_p), c.ctypes.data_as(C.c_void_p),
                               n.ctypes.data_as(C.c_void_p), 0, C.byref(out)) == D.ERANGE
    # plan flags: only DEBYE_PLAN_TARGET_GRAD is defined
    b = D._CBatch(2, 4, 10, 4, 8, 8, 8, 8, 8, 8)
    f = np.array([0, 5, 10], np.int64)
    assert L.debye_plan_create(C.byref(b), f.ctypes.data_as(C.c_void_p), c.ctypes.data_as(C.c_void_p),
                               n.ctypes.data_as(C.c_void_p), 2, C.byref(out)) == D.EINVAL
    assert b"flag" in L.debye_last_error()
    # L-BFGS polish context: parameter ranges and shape, checked before any allocation
    b1 = D._CBatch(2, 4, 10, 2, 8, 8, 8, 8, 8, 8)
    n4 = np.array([4, 4], np.int32)
    pp = C.c_void_p()
    fp, np4 = f.ctypes.data_as(C.c_void_p), n4.ctypes.data_as(C.c_void_p)
    assert L.debye_polish_create(C.byref(b1), fp, np4, 4, D._CLbfgs(5, 0, 30, 1e-4), C.byref(pp)) == D.ERANGE
    assert L.debye_polish_create(C.byref(b1), fp, np4, 4, D._CLbfgs(5, 5, 65, 1e-4), C.byref(pp)) == D.ERANGE
    assert L.debye_polish_create(C.byref(b1), fp, np4, 4, D._CLbfgs(5, 5, 5, 1.5), C.byref(pp)) == D.ERANGE
    assert L.debye_polish_create(C.byref(b1), fp, np4, 3, D._CLbfgs(5, 5, 5, 1e-4), C.byref(pp)) == D.ERANGE
    b2 = D._CBatch(2, 4, 10, 4, 8, 8, 8, 8, 8, 8)
    assert L.debye_polish_create(C.byref(b2), fp, np4, 4, D._CLbfgs(5, 5, 5, 1e-4), C.byref(pp)) == D.EINVAL
    assert b"one candidate per material" in L.debye_last_error()
    # the enqueueing calls need a context
    assert L.debye_lbfgs_polish(None, C.byref(b1), one, one, one, 1e-8, 0, None, z) == D.EINVAL
    assert L.debye_polish_begin(None, C.byref(b1), one, 1e-8, 0, z) == D.EINVAL
    assert L.debye_polish_step(None, C.byref(b1), one, one, one, 1e-8, 0, 0, None, z) == D.EINVAL
