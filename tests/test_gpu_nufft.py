"""The NUFFT (spreading + FFT) that applies A and A^* inside the refinement
iterations when opts.nufft_tol > 0 (Section 4.1 applies A by a NUFFT), against
the oracle's exact direct sums: relative 2-norm error within the requested
tolerance on jittered, ragged, random and polar grids, batch plans and the
full n = 512 size (sampled rows); the two transforms are exact adjoints of
each other; refined solves with the NUFFT operator reach the oracle's
least-squares solution."""
import numpy as np
import pytest
import torch

from nudft_inputs import make_problem, make_grid_problem, complex_normal, config_problem
from oracle import nudft as onu

pytestmark = pytest.mark.gpu

nd = pytest.importorskip("paper_2607_00928_amd")

DEV = torch.device("cuda", 0)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _cases():
    return {
        "jittered32": make_problem(32, 32, 64, 64, 0.25, 1),
        "ragged48x34": make_problem(48, 34, 70, 50, 0.4, 2),
        "tiny6x4": make_problem(6, 4, 9, 7, 0.3, 3),
        "random64": make_grid_problem("random", 64, 4),
        "polar64": make_grid_problem("polar", 64, 5),
    }


@pytest.mark.parametrize("name", ["jittered32", "ragged48x34", "tiny6x4", "random64", "polar64"])
@pytest.mark.parametrize("tol", [1e-6, 1e-9, 1e-12])
def test_nufft_matches_direct_sums(name, tol):
    pr = _cases()[name]
    nx, ny = pr.nx, pr.ny
    rng = np.random.default_rng(7)
    C = np.stack([pr.c_true, complex_normal(rng, (nx, ny))])
    F = complex_normal(rng, (2, pr.M))
    plan = nd.Plan(pr.points, nx, ny)
    f = plan.nufft(torch.from_numpy(C).to(DEV), tol).cpu().numpy()
    c = plan.nufft_adj(torch.from_numpy(F).to(DEV), tol).cpu().numpy()
    plan.close()
    f_ref = onu.apply(pr.points, C)
    c_ref = onu.apply_adj(pr.points, F, nx, ny)
    e2 = max(rel(f[i], f_ref[i]) for i in range(2))
    e1 = max(rel(c[i], c_ref[i]) for i in range(2))
    print(f"{name} tol {tol:.0e}: type 2 {e2:.2e}, type 1 {e1:.2e}")
    assert e2 < 10 * tol and e1 < 10 * tol


def test_nufft_transforms_are_adjoint():
    pr = make_problem(48, 34, 70, 50, 0.4, 2)
    rng = np.random.default_rng(8)
    c = complex_normal(rng, (48, 34))
    f = complex_normal(rng, (pr.M,))
    plan = nd.Plan(pr.points, 48, 34)
    Ac = plan.nufft(torch.from_numpy(c).to(DEV), 1e-9).cpu().numpy()
    Af = plan.nufft_adj(torch.from_numpy(f).to(DEV), 1e-9).cpu().numpy()
    plan.close()
    lhs = np.vdot(f, Ac)
    rhs = np.vdot(Af.reshape(-1), c.reshape(-1))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_nufft_batch_plan():
    shapes = [(32, 48), (8, 8), (64, 32)]
    probs = [make_problem(nx, ny, 2 * nx + 1, 2 * ny + 3, 0.3, 60 + i) for i, (nx, ny) in enumerate(shapes)]
    bp = nd.BatchPlan([p.points for p in probs], [s[0] for s in shapes], [s[1] for s in shapes])
    cflat = np.concatenate([p.c_true.reshape(-1) for p in probs])
    f = bp.nufft(torch.from_numpy(cflat).to(DEV), 1e-11).cpu().numpy()
    rng = np.random.default_rng(9)
    g = complex_normal(rng, (bp.M,))
    c = bp.nufft_adj(torch.from_numpy(g).to(DEV), 1e-11).cpu().numpy()
    bp.close()
    for i, (p, (nx, ny)) in enumerate(zip(probs, shapes)):
        fi = f[bp.m_off[i]:bp.m_off[i + 1]]
        assert rel(fi, onu.apply(p.points, p.c_true)) < 1e-10
        ci = c[bp.n_off[i]:bp.n_off[i + 1]].reshape(nx, ny)
        assert rel(ci, onu.apply_adj(p.points, g[bp.m_off[i]:bp.m_off[i + 1]], nx, ny)) < 1e-10


def test_nufft_full_size_sampled():
    pr = config_problem("n512")
    plan = nd.Plan(pr.points, 512, 512)
    ct = torch.from_numpy(pr.c_true).to(DEV)
    f_exact = plan.apply(ct)
    f = plan.nufft(ct, 1e-12)
    e_all = ((f - f_exact).norm() / f_exact.norm()).item()   # against the exact GPU apply
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(pr.M, 2000, replace=False))
    f_ref = onu.apply(pr.points[rows], pr.c_true)
    e_rows = rel(f.cpu().numpy()[rows], f_ref)
    print(f"n512 type 2, tol 1e-12: sampled rows vs oracle {e_rows:.2e}, "
          f"all rows vs the exact apply {e_all:.2e}")
    plan.close()
    assert e_rows < 1e-11 and e_all < 1e-11


@pytest.mark.parametrize("refine", [0, 1, 2])
def test_refined_solve_with_nufft_operator(refine):
    pr = make_problem(48, 32, 96, 64, 0.4, 21)
    rng = np.random.default_rng(22)
    f = onu.apply(pr.points, pr.c_true) if refine != 1 else complex_normal(rng, (pr.M,))
    ref = onu.lstsq(pr.points, f, 48, 32)
    plan = nd.Plan(pr.points, 48, 32, precision="fp32", eps=1e-2, ir_maxit=100, ir_tol=1e-13,
                   refine=refine, nufft_tol=1e-13)
    plan.factor()
    c, si = plan.solve(torch.from_numpy(f).to(DEV), return_info=True)
    plan.close()
    e = rel(c.cpu().numpy(), ref)
    print(f"refine {refine} with the NUFFT operator: {e:.2e} ({si['iterations']} its)")
    assert e < 1e-10
