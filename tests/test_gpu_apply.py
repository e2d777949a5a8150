"""GPU parity of the exact FP64 apply / adjoint against the oracle."""
import ctypes as C

import numpy as np
import pytest
import torch

from nudft_inputs import make_problem, complex_normal, config_problem
from oracle import nudft as onu

pytestmark = pytest.mark.gpu

nd = pytest.importorskip("paper_2607_00928_amd")
from paper_2607_00928_amd import _lib  # noqa: E402


def dev():
    return torch.device("cuda", 0)


def test_mfma_layout():
    rng = np.random.default_rng(0)
    a = np.ascontiguousarray(rng.integers(-8, 8, size=(16, 4)).astype(np.float64))
    b = np.ascontiguousarray(rng.integers(-8, 8, size=(4, 16)).astype(np.float64))
    d = np.zeros((16, 16))
    st = _lib.lib.nudft2_test_mfma_layout(_lib.dptr(a), _lib.dptr(b), _lib.dptr(d))
    assert st == 0
    assert np.array_equal(d, a @ b)
    a32, b32 = a.astype(np.float32), b.astype(np.float32)
    d32 = np.zeros((16, 16), np.float32)
    fp = lambda x: x.ctypes.data_as(__import__("ctypes").POINTER(__import__("ctypes").c_float))
    st = _lib.lib.nudft2_test_mfma_layout32(fp(a32), fp(b32), fp(d32))
    assert st == 0
    assert np.array_equal(d32, a32 @ b32)


@pytest.mark.parametrize("nx,ny,mx,my,delta,seed", [
    (32, 32, 64, 64, 0.25, 1),       # the small workload
    (48, 34, 70, 50, 0.4, 2),        # ragged: n not a multiple of 16 / 64, M % 64 != 0
    (2, 2, 3, 5, 0.3, 3),            # smallest sizes
    (96, 128, 192, 256, 0.3, 4),
])
def test_apply_and_adjoint_parity(nx, ny, mx, my, delta, seed):
    pr = make_problem(nx, ny, mx, my, delta, seed)
    rng = np.random.default_rng(seed)
    c2 = np.stack([pr.c_true, complex_normal(rng, (nx, ny))])
    plan = nd.Plan(pr.points, nx, ny)
    f_ref = onu.apply(pr.points, c2)
    f = plan.apply(torch.from_numpy(c2).to(dev())).cpu().numpy()
    err = np.max(np.abs(f - f_ref)) / np.max(np.abs(f_ref))
    print(f"apply {nx}x{ny} M={pr.M}: max rel err {err:.2e}")
    assert err < 1e-13
    g = complex_normal(rng, (2, pr.M))
    c_ref = onu.apply_adj(pr.points, g, nx, ny)
    c = plan.apply_adj(torch.from_numpy(g).to(dev())).cpu().numpy()
    err = np.max(np.abs(c - c_ref)) / np.max(np.abs(c_ref))
    print(f"adjoint {nx}x{ny}: max rel err {err:.2e}")
    assert err < 1e-13
    plan.close()


def test_apply_full_size_sampled():
    # n = 512, M = 1024^2: compare 2000 sampled rows of A c and 64 sampled
    # coefficients of A^* f with the oracle evaluated one by one.
    pr = config_problem("n512")
    plan = nd.Plan(pr.points, 512, 512)
    f = plan.apply(torch.from_numpy(pr.c_true).to(dev())).cpu().numpy()
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(pr.M, 2000, replace=False))
    f_ref = onu.apply(pr.points[rows], pr.c_true)
    err = np.max(np.abs(f[rows] - f_ref)) / np.max(np.abs(f_ref))
    print(f"apply n512 sampled: {err:.2e}")
    assert err < 1e-12
    g = complex_normal(rng, (pr.M,))
    c = plan.apply_adj(torch.from_numpy(g).to(dev())).cpu().numpy()
    kx = rng.integers(0, 512, 16)
    ky = rng.integers(0, 512, 16)
    k = onu.centred_freqs(512)
    ex = onu.expi_turns(onu.phase_turns(k[kx], pr.points[:, 0]))
    ey = onu.expi_turns(onu.phase_turns(k[ky], pr.points[:, 1]))
    ref = (ex * ey).conj().T @ g
    got = c[kx, ky]
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"adjoint n512 sampled: {err:.2e}")
    assert err < 1e-11
    plan.close()


def test_adjoint_is_deterministic_and_batched():
    """The adjoint adds its row chunks' partial sums in chunk order, so two
    calls give bit-identical results; in a batch plan every problem's block of
    the result matches its own oracle adjoint (several right-hand sides)."""
    shapes = [(32, 48, 0.3), (8, 8, 0.2), (64, 64, 0.4)]
    probs = [make_problem(nx, ny, 2 * nx + 3, 2 * ny + 1, d, 50 + i)
             for i, (nx, ny, d) in enumerate(shapes)]
    rng = np.random.default_rng(9)
    bp = nd.BatchPlan([p.points for p in probs], [s[0] for s in shapes], [s[1] for s in shapes])
    g = complex_normal(rng, (3, bp.M))
    gt = torch.from_numpy(g).to(dev())
    c1 = bp.apply_adj(gt).cpu().numpy()
    c2 = bp.apply_adj(gt).cpu().numpy()
    assert np.array_equal(c1, c2)
    for i, (p, (nx, ny, _)) in enumerate(zip(probs, shapes)):
        gi = g[:, bp.m_off[i]:bp.m_off[i + 1]]
        ref = onu.apply_adj(p.points, gi, nx, ny).reshape(3, -1)
        got = c1[:, bp.n_off[i]:bp.n_off[i + 1]]
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err < 1e-13, (i, err)
    bp.close()
