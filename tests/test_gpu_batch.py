"""Batched plans: many independent problems of uneven size factored and solved
together (one launch per tree level for all problems).  Every problem of a
batch is checked against the oracle on its own."""
import ctypes as C
import time

import numpy as np
import pytest
import torch

from nudft_inputs import batch_problems, complex_normal, make_problem
from oracle import nudft as onu

pytestmark = pytest.mark.gpu

nd = pytest.importorskip("paper_2607_00928_amd")

DEV = torch.device("cuda", 0)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _pack(problems):
    f = [onu.apply(p.points, p.c_true) for p in problems]
    return f, torch.from_numpy(np.concatenate(f)).to(DEV)


def _split_c(bp, c, problems):
    c = c.cpu().numpy()
    out = []
    for i, p in enumerate(problems):
        nx, ny = p.c_true.shape
        out.append(c[..., bp.n_off[i]:bp.n_off[i + 1]].reshape(c.shape[:-1] + (nx, ny)))
    return out


MIXED = [(32, 32, 0.25, 11), (48, 32, 0.3, 12), (32, 64, 0.3, 13), (16, 16, 0.2, 14),
         (64, 48, 0.4, 15), (8, 8, 0.3, 16)]


def _mixed():
    return [make_problem(nx, ny, 2 * nx, 2 * ny, d, s) for (nx, ny, d, s) in MIXED]


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 1, 0)])
def test_batch_hss_expansions_per_problem(order):
    """1D and recompressed 2D HSS expansions of every problem of a batch
    against the oracle's dense kernel matrices (the same bounds as for a
    single problem): problems of different leaf widths side by side."""
    spec = [(48, 48, 0.25, 22), (64, 32, 0.3, 23), (32, 32, 0.25, 21)]
    probs = [make_problem(nx, ny, 2 * nx, 2 * ny, d, s) for (nx, ny, d, s) in (spec[i] for i in order)]
    nxs = [p.c_true.shape[0] for p in probs]
    nys = [p.c_true.shape[1] for p in probs]
    lib = nd._lib.lib
    eps = 1e-2
    bp = nd.BatchPlan([p.points for p in probs], nxs, nys, precision="fp64", eps=eps)
    rng = np.random.default_rng(5)
    for i, p in enumerate(probs):
        for dim, n in ((0, nxs[i]), (1, nys[i])):
            x = complex_normal(rng, (n,))
            xt = torch.from_numpy(x).to(DEV)
            yt = torch.empty(p.M, dtype=torch.complex128, device=DEV)
            st = lib.nudft2_test_hss1d_matvec(bp._handle, dim, eps / 10, C.c_void_p(xt.data_ptr()),
                                              C.c_void_p(yt.data_ptr()), None, i)
            assert st == 0, lib.nudft2_last_error()
            e = rel(yt.cpu().numpy(), onu.kernel_1d(p.points[:, dim], n) @ x)
            print(f"problem {i} ({nxs[i]}x{nys[i]}) 1D dim {dim}: {e:.2e}")
            assert e < 5 * eps / 10
        G = onu.dense_G(p.points, nxs[i], nys[i])
        x = complex_normal(rng, (nxs[i] * nys[i],))
        for stages in (0, 1, 2):
            xt = torch.from_numpy(x).to(DEV)
            yt = torch.empty(p.M, dtype=torch.complex128, device=DEV)
            st = lib.nudft2_test_hss_matvec(bp._handle, C.c_void_p(xt.data_ptr()),
                                            C.c_void_p(yt.data_ptr()), stages, i, 1)
            assert st == 0, lib.nudft2_last_error()
            e = rel(yt.cpu().numpy(), G @ x)
            print(f"problem {i} ({nxs[i]}x{nys[i]}) 2D stages {stages}: {e:.2e}")
            assert e < 5 * eps
    bp.close()


def test_batch_two_equal_problems():
    probs = [make_problem(32, 32, 64, 64, 0.25, 21), make_problem(32, 32, 64, 64, 0.25, 22)]
    f, ft = _pack(probs)
    bp = nd.BatchPlan([p.points for p in probs], [32, 32], [32, 32], precision="fp32",
                      eps=1e-3, ir_maxit=40, ir_tol=1e-13)
    bp.factor()
    c, si = bp.solve(ft, return_info=True)
    cs = _split_c(bp, c, probs)
    for p, fi, ci in zip(probs, f, cs):
        ref = onu.lstsq(p.points, fi, 32, 32)
        e = rel(ci, ref)
        print(f"two-problem batch: err {e:.2e} ({si['iterations']} its)")
        assert e < 1e-10
    bp.close()


def test_batch_apply_adjoint_parity():
    probs = _mixed()
    f, ft = _pack(probs)
    bp = nd.BatchPlan([p.points for p in probs], [p.c_true.shape[0] for p in probs],
                      [p.c_true.shape[1] for p in probs])
    cflat = torch.from_numpy(np.concatenate([p.c_true.reshape(-1) for p in probs])).to(DEV)
    got_f = bp.apply(cflat).cpu().numpy()
    for i, (p, fi) in enumerate(zip(probs, f)):
        e = rel(got_f[bp.m_off[i]:bp.m_off[i + 1]], fi)
        assert e < 1e-13, (i, e)
    got_a = _split_c(bp, bp.apply_adj(ft), probs)
    for p, fi, ai in zip(probs, f, got_a):
        ref = onu.apply_adj(p.points, fi, *p.c_true.shape)
        assert rel(ai, ref) < 1e-13
    bp.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_mixed_direct_and_refined(prec):
    probs = _mixed()
    f, ft = _pack(probs)
    nxs = [p.c_true.shape[0] for p in probs]
    nys = [p.c_true.shape[1] for p in probs]
    refs = [onu.lstsq(p.points, fi, nx, ny) for p, fi, nx, ny in zip(probs, f, nxs, nys)]
    eps = 1e-3
    bp = nd.BatchPlan([p.points for p in probs], nxs, nys, precision=prec, eps=eps, ir_maxit=0)
    bp.factor()
    c0 = _split_c(bp, bp.solve(ft), probs)
    bp.close()
    bp = nd.BatchPlan([p.points for p in probs], nxs, nys, precision=prec, eps=eps,
                      ir_maxit=40, ir_tol=1e-13)
    bp.factor()
    c1, si = bp.solve(ft, return_info=True)
    c1 = _split_c(bp, c1, probs)
    for i, (a, b, r) in enumerate(zip(c0, c1, refs)):
        e0, e1 = rel(a, r), rel(b, r)
        print(f"{prec} problem {i} {nxs[i]}x{nys[i]}: direct {e0:.2e}, refined {e1:.2e}")
        assert e0 < eps + (2e-6 if prec == "fp32" else 1e-13)   # measured <= 0.29 eps
        assert e1 < 1e-10
    # several right-hand sides through the batch
    F2 = torch.stack([ft, 2j * ft]).contiguous()
    c2 = _split_c(bp, bp.solve(F2), probs)
    for i, r in enumerate(refs):
        assert rel(c2[i][0], r) < 1e-10 and rel(c2[i][1], 2j * r) < 1e-10
    bp.close()


def test_batch_64_uneven_problems():
    """64 problems, n^x, n^y uniform over {32, 48, 64, 96, 128}, M = 4N each,
    FP32 factors + FP64 refinement.  Consistent right-hand sides: every
    solution must match its c_true; the smallest problems are also checked
    against the oracle's dense least-squares solution."""
    probs = batch_problems()
    print("64-problem batch: shapes", [p.c_true.shape for p in probs], flush=True)
    f, ft = _pack(probs)
    nxs = [p.c_true.shape[0] for p in probs]
    nys = [p.c_true.shape[1] for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bp = nd.BatchPlan([p.points for p in probs], nxs, nys, precision="fp32", eps=1e-2,
                      ir_maxit=60, ir_tol=1e-12)
    bp.factor()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c, si = bp.solve(ft, return_info=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    cs = _split_c(bp, c, probs)
    print(f"64-problem batch: N total {sum(x * y for x, y in zip(nxs, nys))}, "
          f"M total {bp.M}, factor {t1 - t0:.2f} s, refined solve {t2 - t1:.2f} s "
          f"({si['iterations']} its)")
    worst = max(rel(ci, p.c_true) for ci, p in zip(cs, probs))
    print(f"worst error vs c_true {worst:.2e}")
    assert worst < 1e-10
    small = [i for i in range(len(probs)) if nxs[i] * nys[i] <= 1536][:4]
    for i in small:
        ref = onu.lstsq(probs[i].points, f[i], nxs[i], nys[i])
        assert rel(cs[i], ref) < 1e-10
    bp.close()


def test_batch_per_problem_stopping_test():
    """The refinement stops when every problem of the batch meets ir_tol on
    its own (norms per problem and right-hand side): a small problem beside
    two large ones reaches 1e-10 at ir_tol = 1e-10, which a stopping test on
    the concatenated vector would not guarantee."""
    shapes = [(128, 128), (8, 8), (96, 128)]
    probs = [make_problem(nx, ny, 2 * nx, 2 * ny, 0.3, 70 + i) for i, (nx, ny) in enumerate(shapes)]
    # the small problem's coefficients are scaled down, so that its share of
    # the concatenated norms is tiny
    probs[1].c_true *= 1e-3
    f, ft = _pack(probs)
    bp = nd.BatchPlan([p.points for p in probs], [s[0] for s in shapes], [s[1] for s in shapes],
                      precision="fp32", eps=1e-2, ir_maxit=60, ir_tol=1e-10)
    bp.factor()
    cs = _split_c(bp, bp.solve(ft), probs)
    bp.close()
    for i, (ci, p) in enumerate(zip(cs, probs)):
        e = rel(ci, p.c_true)
        print(f"problem {i} {shapes[i]}: err vs c_true {e:.2e}")
        assert e < 1e-10, (i, e)


def test_batch_64_graph_captured_solve():
    """The 64-problem batch with the refinement iteration captured into a HIP
    graph and replayed (opts.graph): the same iterations and solutions as the
    eager launches, every problem within 1e-10 of c_true."""
    probs = batch_problems()
    f, ft = _pack(probs)
    nxs = [p.c_true.shape[0] for p in probs]
    nys = [p.c_true.shape[1] for p in probs]
    out = {}
    for graph in (False, True):
        bp = nd.BatchPlan([p.points for p in probs], nxs, nys, precision="fp32", eps=1e-2,
                          ir_maxit=60, ir_tol=1e-12, graph=graph)
        bp.factor()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c, si = bp.solve(ft, return_info=True)
        torch.cuda.synchronize()
        out[graph] = (c.cpu().numpy(), si["iterations"], time.perf_counter() - t0)
        bp.close()
    print(f"64-problem batch solve: eager {out[False][2]:.3f} s ({out[False][1]} its), "
          f"graph {out[True][2]:.3f} s ({out[True][1]} its)")
    assert out[True][1] == out[False][1]
    assert rel(out[True][0], out[False][0]) < 1e-12
    cs = _split_c(bp, torch.from_numpy(out[True][0]), probs)
    worst = max(rel(ci, p.c_true) for ci, p in zip(cs, probs))
    assert worst < 1e-10
