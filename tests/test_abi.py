"""The C-ABI library loads and exports what include/mmot.h declares; argument
checks that run before any device call behave as documented (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mmot.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(mmot_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def _lib():
    from paper_2405_19246_amd import mmot
    if not os.path.exists(mmot.LIB_PATH):
        pytest.fail("libmmot.so is not built; run __graft_entry__.build()")
    return mmot


def test_every_declared_symbol_is_exported():
    mmot = _lib()
    L = mmot.lib()
    declared = _declared()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(mmot.EXPORTS)


def test_struct_layouts_match_header_sizes():
    mmot = _lib()
    assert ctypes.sizeof(mmot.Problem) == 48
    assert ctypes.sizeof(mmot.Opts) == 24
    assert ctypes.sizeof(mmot.Result) == 40
    assert ctypes.sizeof(mmot.Instance) == 56
    assert ctypes.sizeof(mmot.BatchTiming) == 48


@pytest.mark.parametrize("l,N,h,eps,code", [
    (1, 10, 0.1, 0.1, -1), (11, 10, 0.1, 0.1, -1), (3, 0, 0.1, 0.1, -1), (3, 10, 0.1, 0.0, -1),
    (3, 10, 0.1, -1.0, -1), (3, 10, 0.0, 0.1, -1), (3, 10, float("nan"), 0.1, -1), (10, 0, 0.1, 0.1, -1),
])
def test_plan_rejects_bad_shapes(l, N, h, eps, code):
    mmot = _lib()
    p = mmot.Problem(l, N, h, eps, 0)
    out = ctypes.c_void_p()
    rc = mmot.lib().mmot_plan(ctypes.byref(p), None, None, ctypes.byref(out))
    assert rc == code
    assert out.value is None
    assert mmot.last_error() != ""


def test_plan_rejects_bad_precision_and_opts():
    mmot = _lib()
    out = ctypes.c_void_p()
    p = mmot.Problem(3, 10, 0.1, 0.1, 7)
    assert mmot.lib().mmot_plan(ctypes.byref(p), None, None, ctypes.byref(out)) == -1
    p = mmot.Problem(3, 10, 0.1, 0.1, 0)
    o = mmot.Opts(1e-6, -1, 10, 0)
    assert mmot.lib().mmot_plan(ctypes.byref(p), ctypes.byref(o), None, ctypes.byref(out)) == -1
    o = mmot.Opts(float("nan"), 10, 10, 0)
    assert mmot.lib().mmot_plan(ctypes.byref(p), ctypes.byref(o), None, ctypes.byref(out)) == -1


def test_batch_rejects_bad_instance_before_device_work():
    mmot = _lib()
    arr = (mmot.Instance * 1)()
    arr[0] = mmot.Instance(3, 0, 0.1, 0.1, None, None)
    o = mmot.Opts(1e-6, 10, 10, 0)
    res = (mmot.Result * 1)()
    assert mmot.lib().mmot_solve_batch(arr, 1, 1, ctypes.byref(o), None, res) == -1
    assert "instance 0" in mmot.last_error()


def test_null_plan_calls_are_invalid():
    mmot = _lib()
    L = mmot.lib()
    assert L.mmot_marginal_product(None, 0, None, None) == -1
    assert L.mmot_solve(None, None, None, None) == -1
    assert L.mmot_dense_marginal_product(None, 0, None, None) == -1
    assert L.mmot_dense_sinkhorn_iter(None, None, None, 1) == -1
    assert L.mmot_plan_destroy(None) == 0
    assert L.mmot_serve_stop(None) == 0


def test_noalloc_product_checks_before_device_work():
    # size and argument checks of the no-allocation entry point need no GPU
    mmot = _lib()
    L = mmot.lib()
    p = mmot.Problem(10, 1000000, 1e-6, 0.01, 0)
    dummy = ctypes.c_void_p(16)
    assert L.mmot_marginal_product_noalloc(ctypes.byref(p), 0, dummy, dummy, None) == -1
    assert "workspace" in mmot.last_error()
    p = mmot.Problem(4, 100, 0.01, 0.01, 0)
    assert L.mmot_marginal_product_noalloc(ctypes.byref(p), 4, dummy, dummy, None) == -1
    assert L.mmot_marginal_product_noalloc(ctypes.byref(p), 0, None, dummy, None) == -1
    assert L.mmot_marginal_product_noalloc(None, 0, dummy, dummy, None) == -1


def test_plan_rejects_a_bad_grid_before_device_work():
    # non-uniform grid coordinates are checked on the host before any allocation
    import numpy as np
    mmot = _lib()
    out = ctypes.c_void_p()
    for bad in (np.array([0.0, 0.2, 0.1, 0.5]), np.array([0.0, np.nan, 0.3, 0.5]), np.array([0.0, 0.1, 0.2, np.inf])):
        x = np.ascontiguousarray(bad)
        p = mmot.Problem(3, 4, 0.0, 0.1, 0, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        assert mmot.lib().mmot_plan(ctypes.byref(p), None, None, ctypes.byref(out)) == -1
        assert "grid" in mmot.last_error()
        assert out.value is None


def test_noalloc_product_rejects_a_grid():
    import numpy as np
    mmot = _lib()
    x = np.linspace(0.0, 1.0, 10)
    p = mmot.Problem(3, 10, 0.0, 0.1, 0, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    dummy = ctypes.c_void_p(16)
    assert mmot.lib().mmot_marginal_product_noalloc(ctypes.byref(p), 0, dummy, dummy, None) == -5


def test_jacobi_flag_is_a_plan_option():
    mmot = _lib()
    arr = (mmot.Instance * 1)()
    dummy = ctypes.c_void_p(16)
    arr[0] = mmot.Instance(3, 10, 0.1, 0.1, dummy, dummy, None)
    o = mmot.Opts(1e-6, 10, 10, mmot.FLAG_JACOBI)
    res = (mmot.Result * 1)()
    assert mmot.lib().mmot_solve_batch(arr, 1, 1, ctypes.byref(o), None, res) == -5
    assert "JACOBI" in mmot.last_error()


def test_plan_2d_rejects_bad_shapes_before_device_work():
    mmot = _lib()
    out = ctypes.c_void_p()
    for args in [(0, 4, 0.1, 0.1, 0.1), (4, 0, 0.1, 0.1, 0.1), (4, 4, 0.0, 0.1, 0.1), (4, 4, 0.1, -1.0, 0.1),
                 (4, 4, 0.1, 0.1, 0.0), (1 << 20, 1 << 20, 0.1, 0.1, 0.1)]:
        p = mmot.Problem2D(*args)
        assert mmot.lib().mmot_plan_2d(ctypes.byref(p), None, None, ctypes.byref(out)) == -1
        assert out.value is None
    p = mmot.Problem2D(4, 4, 0.1, 0.1, 0.1)
    o = mmot.Opts(1e-6, 10, 10, mmot.FLAG_TILES)
    assert mmot.lib().mmot_plan_2d(ctypes.byref(p), ctypes.byref(o), None, ctypes.byref(out)) == -5
