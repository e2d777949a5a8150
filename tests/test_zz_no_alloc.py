"""The no-allocation adjoint apply (nudft2_apply_adj_noalloc) against the
allocating one (nudft2_apply_adj) and the oracle, through the C-ABI: two
calls in a row on one GPU, the second with a smaller input, and the size
limit of its static scratch."""
import ctypes as C

import numpy as np
import pytest
import torch

from nudft_inputs import make_problem, complex_normal
from oracle import nudft as onu

pytestmark = pytest.mark.gpu

nd = pytest.importorskip("paper_2607_00928_amd")
from paper_2607_00928_amd import _lib  # noqa: E402

DEV = torch.device("cuda", 0)


def _adj(fn, plan, g, N):
    out = torch.empty((g.shape[0], N), dtype=torch.complex128, device=DEV)
    st = fn(plan._handle, C.c_void_p(g.data_ptr()), C.c_void_p(out.data_ptr()), g.shape[0])
    return st, out


def test_noalloc_adjoint_matches_allocating_one():
    lib = _lib.lib
    rng = np.random.default_rng(21)
    cases = [(96, 64, 2, 0.35, 61), (32, 32, 1, 0.25, 62)]   # second call: smaller input
    for nx, ny, nrhs, delta, seed in cases:
        pr = make_problem(nx, ny, 2 * nx, 2 * ny, delta, seed)
        plan = nd.Plan(pr.points, nx, ny)
        g = torch.from_numpy(complex_normal(rng, (nrhs, pr.M))).to(DEV)
        st1, c_alloc = _adj(lib.nudft2_apply_adj, plan, g, nx * ny)
        st2, c_free = _adj(lib.nudft2_apply_adj_noalloc, plan, g, nx * ny)
        assert st1 == 0 and st2 == 0, lib.nudft2_last_error()
        a, b = c_alloc.cpu().numpy(), c_free.cpu().numpy()
        ref = onu.apply_adj(pr.points, g.cpu().numpy(), nx, ny).reshape(nrhs, -1)
        scale = np.max(np.abs(ref))
        print(f"{nx}x{ny} nrhs {nrhs}: |noalloc - alloc| {np.max(np.abs(a - b)) / scale:.1e}, "
              f"|noalloc - oracle| {np.max(np.abs(b - ref)) / scale:.1e}")
        assert np.max(np.abs(b - a)) <= 1e-13 * scale
        assert np.max(np.abs(b - ref)) <= 1e-13 * scale
        plan.close()


def test_noalloc_adjoint_rejects_inputs_beyond_its_scratch():
    # nrhs * N * 16 bytes > 64 MiB: one 512 x 512 coefficient vector per
    # right-hand side is 4 MiB, so 17 right-hand sides cannot fit
    pr = make_problem(512, 512, 512, 512, 0.3, 63)
    plan = nd.Plan(pr.points, 512, 512)
    g = torch.zeros((17, pr.M), dtype=torch.complex128, device=DEV)
    st, _ = _adj(_lib.lib.nudft2_apply_adj_noalloc, plan, g, 512 * 512)
    assert st == 1
    assert b"64 MiB" in _lib.lib.nudft2_last_error()
    plan.close()
