"""Host logic: every C entry point rejects bad arguments with CBS_EINVAL before it touches a
device (NULL handles, unsupported grids, bad sizes), and leaves a message naming the call."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1709_09347_amd", "libcbs.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


@pytest.fixture(scope="module")
def cbs():
    import paper_1709_09347_amd as m
    return m


def _err(L):
    return L.cbs_last_error().decode()


@pytest.mark.parametrize("grid,why", [((8, 8, 12, 3, 0.4), "fd_order"), ((8, 8, 12, 10, 0.4), "fd_order"),
                                      ((0, 8, 12, 4, 0.4), "grid"), ((300, 8, 12, 4, 0.4), "grid"),
                                      ((8, 8, 1, 4, 0.4), "grid"), ((8, 8, 12, 4, 0.0), "grid"),
                                      ((240, 4, 12, 8, 0.3), "too wide")])
def test_system_create_rejects_unsupported_grids(cbs, grid, why):
    L = cbs.lib()
    v = np.zeros(max(1, grid[0] * grid[1] * grid[2]))
    h = ctypes.c_void_p()
    g = cbs.Grid(*grid)
    assert L.cbs_system_create(ctypes.byref(h), 0, ctypes.byref(g), v.ctypes.data, None) == cbs.CBS_EINVAL
    assert why in _err(L) and not h.value


def test_entry_points_reject_null_handles(cbs):
    L = cbs.lib()
    z = np.array([1.0, 0.0])
    p = cbs.default_params()
    dummy = ctypes.c_void_p(16)   # never dereferenced: every call returns on the NULL handle first
    checks = [
        ("cbs_system_create", lambda: L.cbs_system_create(None, 0, None, None, None)),
        ("cbs_system_set_vloc", lambda: L.cbs_system_set_vloc(None, z.ctypes.data)),
        ("cbs_apply", lambda: L.cbs_apply(None, 0.0, 1, z.ctypes.data, cbs.CBS_C128, dummy, dummy, None)),
        ("cbs_apply_parts", lambda: L.cbs_apply_parts(None, 0.0, 1, z.ctypes.data, z.ctypes.data, z.ctypes.data,
                                                      dummy, dummy, None)),
        ("cbs_bicg", lambda: L.cbs_bicg(None, 0.0, 1, z.ctypes.data, 1, dummy, ctypes.byref(p), dummy, dummy,
                                        None, None, None, None)),
        ("cbs_solve", lambda: L.cbs_solve(None, 0.0, ctypes.byref(p), dummy, 4, z.ctypes.data, None, None,
                                          ctypes.byref(ctypes.c_int32()), None, None)),
        ("cbs_grad_vloc", lambda: L.cbs_grad_vloc(None, 0, None, dummy, None, None, None)),
    ]
    for name, call in checks:
        assert call() == cbs.CBS_EINVAL, name
        assert name in _err(L), (name, _err(L))


def test_history_and_batch_sizes_are_checked(cbs):
    L = cbs.lib()
    z = np.array([1.0, 0.0])
    p = cbs.default_params()
    hist = np.zeros(8)
    dummy = ctypes.c_void_p(16)
    for stride, rows, h in ((0, 1, hist.ctypes.data), (1, 0, hist.ctypes.data), (1, 1, None)):
        rc = L.cbs_bicg_history(None, 0.0, 1, z.ctypes.data, 1, dummy, ctypes.byref(p), stride, rows, h,
                                dummy, dummy, None, None, None, None)
        assert rc == cbs.CBS_EINVAL and "cbs_bicg_history" in _err(L)
    # more than 2^31 history entries
    rc = L.cbs_bicg_history(None, 0.0, 1024, z.ctypes.data, 1024, dummy, ctypes.byref(p), 1, 1024,
                            hist.ctypes.data, dummy, dummy, None, None, None, None)
    assert rc == cbs.CBS_EINVAL
    n = ctypes.c_int32()
    E = np.array([0.1])
    assert L.cbs_solve_batched(0, None, 1, E.ctypes.data, ctypes.byref(p), None, 1, None, ctypes.byref(n),
                               None, None) == cbs.CBS_EINVAL
    assert "cbs_solve_batched" in _err(L)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_system_create_rejects_non_finite_potential(cbs, bad):
    L = cbs.lib()
    v = np.zeros(8 * 8 * 12)
    v[77] = bad
    h = ctypes.c_void_p()
    g = cbs.Grid(8, 8, 12, 4, 0.4)
    assert L.cbs_system_create(ctypes.byref(h), 0, ctypes.byref(g), v.ctypes.data, None) == cbs.CBS_EINVAL
    assert "v_loc[77]" in _err(L) and not h.value
