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
def test_hss1d_matvec(nx, ny, mx, my, delta, seed, tol):
    pr = make_problem(nx, ny, mx, my, delta, seed)
    plan = nd.Plan(pr.points, nx, ny)
    rng = np.random.default_rng(seed)
    for dim, n in ((0, nx), (1, ny)):
        x = complex_normal(rng, (n,))
        xt = torch.from_numpy(x).to(DEV)
        yt = torch.empty(pr.M, dtype=torch.complex128, device=DEV)
        ranks = np.zeros(2 * 8, np.int32)
        st = lib.nudft2_test_hss1d_matvec(plan._handle, dim, tol, C.c_void_p(xt.data_ptr()),
                                          C.c_void_p(yt.data_ptr()),
                                          ranks.ctypes.data_as(C.POINTER(C.c_int32)))
        assert st == 0, lib.nudft2_last_error()
        G = onu.kernel_1d(pr.points[:, dim], n)
        ref = G @ x
        err = np.linalg.norm(yt.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"1D dim{dim} n={n} tol={tol:.0e}: rel err {err:.2e} ranks {ranks.tolist()}")
        assert err < 5 * tol
    plan.close()
