"""GPU checks of the HSS stages against the oracle's kernel matrix G."""
import ctypes as C

import numpy as np
import pytest
import torch

from nudft_inputs import make_problem, complex_normal
from oracle import nudft as onu

pytestmark = pytest.mark.gpu

nd = pytest.importorskip("paper_2607_00928_amd")
from paper_2607_00928_amd import _lib  # noqa: E402

lib = _lib.lib
DEV = torch.device("cuda", 0)


@pytest.mark.parametrize("nx,ny,mx,my,delta,seed", [
    (32, 32, 64, 64, 0.25, 1),
    (128, 64, 256, 128, 0.3, 2),
    (48, 96, 96, 192, 0.4, 3),
])
@pytest.mark.parametrize("tol", [1e-5, 1e-9])
@pytest.mark.parametrize("fadi_1d", [True, False])
def test_hss1d_matvec(nx, ny, mx, my, delta, seed, tol, fadi_1d):
    pr = make_problem(nx, ny, mx, my, delta, seed)
    plan = nd.Plan(pr.points, nx, ny, fadi_1d=fadi_1d)
    rng = np.random.default_rng(seed)
    for dim, n in ((0, nx), (1, ny)):
        x = complex_normal(rng, (n,))
        xt = torch.from_numpy(x).to(DEV)
        yt = torch.empty(pr.M, dtype=torch.complex128, device=DEV)
        ranks = np.zeros(2 * 8, np.int32)
        st = lib.nudft2_test_hss1d_matvec(plan._handle, dim, tol, C.c_void_p(xt.data_ptr()),
                                          C.c_void_p(yt.data_ptr()),
                                          ranks.ctypes.data_as(C.POINTER(C.c_int32)), 0)
        assert st == 0, lib.nudft2_last_error()
        G = onu.kernel_1d(pr.points[:, dim], n)
        ref = G @ x
        err = np.linalg.norm(yt.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"1D dim{dim} n={n} tol={tol:.0e} fadi={fadi_1d}: rel err {err:.2e} "
              f"ranks {ranks.tolist()}")
        assert err < 5 * tol
    plan.close()


@pytest.mark.parametrize("nx,ny,mx,my,delta,seed", [
    (32, 32, 64, 64, 0.25, 1),
    (48, 32, 96, 64, 0.4, 5),
    (64, 64, 128, 128, 0.3, 6),
])
@pytest.mark.parametrize("prec,eps", [("fp64", 1e-2), ("fp64", 1e-4), ("fp64", 1e-7),
                                      ("fp32", 1e-2), ("fp32", 1e-4)])
@pytest.mark.parametrize("stages", [0, 1, 2])
def test_hss2d_matvec(nx, ny, mx, my, delta, seed, prec, eps, stages):
    pr = make_problem(nx, ny, mx, my, delta, seed)
    plan = nd.Plan(pr.points, nx, ny, precision=prec, eps=eps)
    rng = np.random.default_rng(seed)
    x = complex_normal(rng, (nx * ny,))
    xt = torch.from_numpy(x).to(DEV)
    yt = torch.empty(pr.M, dtype=torch.complex128, device=DEV)
    st = lib.nudft2_test_hss_matvec(plan._handle, C.c_void_p(xt.data_ptr()),
                                    C.c_void_p(yt.data_ptr()), stages, 0, 1)
    assert st == 0, lib.nudft2_last_error()
    G = onu.dense_G(pr.points, nx, ny)
    ref = G @ x
    err = np.linalg.norm(yt.cpu().numpy() - ref) / np.linalg.norm(ref)
    info = plan.info()
    print(f"2D {nx}x{ny} {prec} eps={eps:.0e} stages={stages}: rel err {err:.2e} ranks U {info['max_rank_u']} "
          f"V {info['max_rank_v']}")
    floor = 3e-6 if prec == "fp32" else 0.0
    assert err < 5 * eps + floor
    plan.close()
