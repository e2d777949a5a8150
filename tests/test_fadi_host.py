"""Host logic of the library's fADI plan (no device work): the near-column
count, the shift count, gamma and the Zolotarev shifts of an HSS row block,
against the oracle (which evaluates the elliptic functions in 30-digit
arithmetic; the library uses the arithmetic-geometric mean)."""
import ctypes as C

import numpy as np
import pytest

from oracle import fadi

nd = pytest.importorskip("paper_2607_00928_amd")
from paper_2607_00928_amd import _lib  # noqa: E402

lib = _lib.lib
SMAX = 64


def lib_plan(n, level, a, tau):
    plan = np.zeros(2, np.int32)
    g = C.c_double()
    pq = np.zeros(4 * SMAX, np.float64)
    st = lib.nudft2_test_fadi_block(None, 0, n, level, a, tau,
                                    plan.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(g),
                                    pq.ctypes.data_as(C.POINTER(C.c_double)), SMAX, None, None)
    assert st == 0, lib.nudft2_last_error()
    b, s = int(plan[0]), int(plan[1])
    z = pq[0::2] + 1j * pq[1::2]
    return b, s, g.value, z[:s], z[SMAX:SMAX + s]


CASES = [(512, 5, 0, 1e-4), (512, 5, 17, 1e-4), (512, 1, 1, 1e-4), (512, 3, 6, 1e-9),
         (256, 4, 15, 1e-6), (96, 2, 1, 1e-5), (48, 3, 4, 1e-10), (1024, 6, 63, 1e-3),
         (20, 2, 3, 1e-6), (8, 2, 1, 1e-4)]


@pytest.mark.parametrize("n,level,a,tau", CASES)
def test_plan_matches_oracle(n, level, a, tau):
    b, s, g, p, q = lib_plan(n, level, a, tau)
    ob, os_, og, arcs, lo, hi = fadi.block_plan(n, level, a, tau)
    assert (b, s) == (ob, os_)
    if b == 0:
        return
    assert abs(g - og) <= 1e-10 * og
    op, oq = fadi.zolotarev_shifts(*arcs, s)
    assert np.abs(p - op).max() < 1e-10
    assert np.abs(q - oq).max() < 1e-10
    assert np.allclose(np.abs(p), 1.0, atol=1e-13) and np.allclose(np.abs(q), 1.0, atol=1e-13)


def test_plan_rejects_bad_block():
    plan = np.zeros(2, np.int32)
    g = C.c_double()
    pq = np.zeros(4, np.float64)
    i32 = plan.ctypes.data_as(C.POINTER(C.c_int32))
    dp = pq.ctypes.data_as(C.POINTER(C.c_double))
    assert lib.nudft2_test_fadi_block(None, 0, 64, 0, 0, 1e-4, i32, C.byref(g), dp, 1, None, None) == 1
    assert lib.nudft2_test_fadi_block(None, 0, 64, 2, 4, 1e-4, i32, C.byref(g), dp, 1, None, None) == 1
    assert lib.nudft2_test_fadi_block(None, 0, 64, 2, 1, 0.0, i32, C.byref(g), dp, 1, None, None) == 1
    # more shifts than room for them
    assert lib.nudft2_test_fadi_block(None, 0, 512, 3, 1, 1e-9, i32, C.byref(g), dp, 1, None, None) == 1
    assert plan[1] > 1
