"""Pins for the oracle's HSS machinery (trees, face-split generators,
recompression, URV) and its derivatives."""
import numpy as np
import pytest

from nudft_inputs import make_problem, complex_normal
from oracle import nudft, hss, grad


@pytest.fixture(scope="module")
def small():
    # n = 16 with 4-column leaves: depth 2, so transfer matrices and all
    # three sibling cases of the face-split interactions are exercised.
    pr = make_problem(16, 16, 32, 32, 0.25, 21)
    return pr


def test_tree_partitions(small):
    # Theorem 3.2: the product tree is an HSS tree (disjoint unions)
    pts = small.points
    t = hss.tree_2d(pts, 16, 16, 2)
    for k, nd in t.nodes.items():
        if nd.children:
            rows = np.concatenate([t.nodes[c].rows for c in nd.children])
            cols = np.concatenate([t.nodes[c].cols for c in nd.children])
            assert np.array_equal(np.sort(rows), nd.rows)
            assert np.array_equal(np.sort(cols), np.sort(nd.cols))
            assert rows.size == np.unique(rows).size
    assert t.nodes[t.root].rows.size == pts.shape[0]
    assert np.array_equal(np.sort(t.nodes[t.root].cols), np.arange(256))


def test_col_ranges_half_open():
    # columns l with l/n in [a/2^l, (a+1)/2^l); ragged for n = 48
    for n, L in [(48, 2), (64, 2), (12, 1)]:
        got = np.concatenate([hss.col_range(n, L, a) for a in range(1 << L)])
        assert np.array_equal(got, np.arange(n))
        for a in range(1 << L):
            for l in hss.col_range(n, L, a):
                assert a / (1 << L) <= l / n < (a + 1) / (1 << L)


def test_hss_1d_exact_and_truncated(small):
    x = small.points[:, 0]
    G = nudft.kernel_1d(x, 16)
    h0 = hss.hss_1d(x, 16, 2, 0.0)
    assert np.max(np.abs(hss.expand(h0, x.size, 16) - G)) < 1e-13
    for tol in (1e-3, 1e-5):
        h = hss.hss_1d(x, 16, 2, tol)
        err = np.linalg.norm(hss.expand(h, x.size, 16) - G) / np.linalg.norm(G)
        assert err < 3 * tol


def test_face_split_generators_exact(small):
    # Theorem 3.3: from exact 1D HSS matrices the assembled generators
    # reproduce H^x . H^y (the row-wise Kronecker product of the expansions).
    pts = small.points
    M = pts.shape[0]
    hx = hss.hss_1d(pts[:, 0], 16, 2, 0.0)
    hy = hss.hss_1d(pts[:, 1], 16, 2, 0.0)
    h = hss.face_split(pts, 16, 16, hx, hy)
    H = hss.expand(h, M, 256)
    ref = hss.face(hss.expand(hx, M, 16), hss.expand(hy, M, 16))
    assert np.max(np.abs(H - ref)) < 1e-13
    # and, with truncated 1D factors, still exactly the face-split product
    hx = hss.hss_1d(pts[:, 0], 16, 2, 1e-3)
    hy = hss.hss_1d(pts[:, 1], 16, 2, 1e-3)
    h = hss.face_split(pts, 16, 16, hx, hy)
    ref = hss.face(hss.expand(hx, M, 16), hss.expand(hy, M, 16))
    assert np.max(np.abs(hss.expand(h, M, 256) - ref)) < 1e-13


def test_face_split_widths(small):
    # rank bound of Theorem 3.3: r^x d^y + r^y d^x + r^x r^y
    pts = small.points
    hx = hss.hss_1d(pts[:, 0], 16, 2, 1e-3)
    hy = hss.hss_1d(pts[:, 1], 16, 2, 1e-3)
    h = hss.face_split(pts, 16, 16, hx, hy)
    for k in h.tree.leaves():
        _, a, b = k
        rx, ry = hx.U[(2, a)].shape[1], hy.U[(2, b)].shape[1]
        dx, dy = 4, 4
        assert h.U[k].shape[1] == rx * dy + ry * dx + rx * ry


def test_approximation_bound(small):
    # Theorem 3.5: ||H - G||_F <= (1 + C) eps ||G||_F with C = 1 + sqrt(M) eps
    pts = small.points
    M = pts.shape[0]
    G = nudft.dense_G(pts, 16, 16)
    for tol in (1e-2, 1e-4):
        hx = hss.hss_1d(pts[:, 0], 16, 2, tol)
        hy = hss.hss_1d(pts[:, 1], 16, 2, tol)
        Hx = hss.expand(hx, M, 16)
        Gx = nudft.kernel_1d(pts[:, 0], 16)
        ex = np.linalg.norm(Hx - Gx) / np.linalg.norm(Gx)
        Hy = hss.expand(hy, M, 16)
        Gy = nudft.kernel_1d(pts[:, 1], 16)
        ey = np.linalg.norm(Hy - Gy) / np.linalg.norm(Gy)
        e = max(ex, ey)
        H = hss.expand(hss.face_split(pts, 16, 16, hx, hy), M, 256)
        err = np.linalg.norm(H - G) / np.linalg.norm(G)
        C = np.max(np.linalg.norm(Hx, axis=1)) / np.max(np.linalg.norm(Gx, axis=1))
        assert err <= (1 + C) * e * (1 + 1e-9)
        assert err <= (2 + np.sqrt(M) * e) * e


def test_recompression_stage1_exact_stage2_bounded(small):
    pts = small.points
    M = pts.shape[0]
    hx = hss.hss_1d(pts[:, 0], 16, 2, 1e-4)
    hy = hss.hss_1d(pts[:, 1], 16, 2, 1e-4)
    h = hss.face_split(pts, 16, 16, hx, hy)
    H = hss.expand(h, M, 256)
    h1 = hss.recompress(h, 0.0)        # orthogonalisation only (Section 2.3)
    assert np.max(np.abs(hss.expand(h1, M, 256) - H)) < 1e-12
    for eps in (1e-2, 1e-3):
        h2 = hss.recompress(h, eps)
        err = np.linalg.norm(hss.expand(h2, M, 256) - H) / np.linalg.norm(H)
        assert err < 4 * eps
        # truncation never grows a basis
        for k in h2.U:
            assert h2.U[k].shape[1] <= h.U[k].shape[1]
        # leaf bases are orthonormal after recompression
        for k in h2.U:
            U = h2.U[k]
            assert np.allclose(U.conj().T @ U, np.eye(U.shape[1]), atol=1e-12)


def test_urv_equals_dense_least_squares(small):
    pts = small.points
    M = pts.shape[0]
    rng = np.random.default_rng(3)
    f = complex_normal(rng, (M,))
    for eps in (0.0, 1e-2):
        hx = hss.hss_1d(pts[:, 0], 16, 2, 1e-3)
        hy = hss.hss_1d(pts[:, 1], 16, 2, 1e-3)
        h = hss.recompress(hss.face_split(pts, 16, 16, hx, hy), eps)
        u = hss.urv_factor(h)
        c = hss.urv_solve(u, f, 256)
        H = hss.expand(h, M, 256)
        ref = np.linalg.lstsq(H, f, rcond=None)[0]
        assert np.linalg.norm(c - ref) < 1e-11 * np.linalg.norm(ref)


def test_urv_square_case_is_inverse():
    # M = N exact grid with jitter: square HSS, URV gives H^{-1} f
    pr = make_problem(8, 8, 8, 8, 0.2, 31)
    M = pr.M
    hx = hss.hss_1d(pr.points[:, 0], 8, 1, 1e-8)
    hy = hss.hss_1d(pr.points[:, 1], 8, 1, 1e-8)
    h = hss.face_split(pr.points, 8, 8, hx, hy)
    H = hss.expand(h, M, 64)
    f = complex_normal(np.random.default_rng(0), (M,))
    c = hss.urv_solve(hss.urv_factor(h), f, 64)
    assert np.linalg.norm(H @ c - f) < 1e-9 * np.linalg.norm(f)


def test_direct_solver_accuracy_tracks_eps():
    # Algorithm 4.1 on the small jittered workload: error of the order of eps
    # (the paper reports e_s within about one order of eps).
    pr = make_problem(32, 32, 64, 64, 0.25, 1)
    f = nudft.apply(pr.points, pr.c_true)
    for eps in (1e-2, 1e-4):
        c = hss.direct_solve(pr.points, f, 32, 32, eps)
        e = nudft.rel_err(c, pr.c_true)
        assert e < 10 * eps


def test_gradient_formula_vs_finite_differences():
    # App. derivation in oracle.grad: central differences in f, x_j, y_j
    pr = make_problem(4, 4, 8, 8, 0.25, 41, with_target=True)
    pts = pr.points.copy()
    rng = np.random.default_rng(5)
    f = nudft.apply(pts, pr.c_true) + 0.1 * complex_normal(rng, (pr.M,))
    L0, g = grad.loss_target(pts, f, 4, 4, pr.c_target)
    c, gf, gx, gy = grad.lsq_grads(pts, f, 4, 4, g)
    h = 1e-6
    for j in (0, 17, 40):
        for coord, gg in ((0, gx), (1, gy)):
            p1, p2 = pts.copy(), pts.copy()
            p1[j, coord] += h
            p2[j, coord] -= h
            Lp, _ = grad.loss_target(p1, f, 4, 4, pr.c_target)
            Lm, _ = grad.loss_target(p2, f, 4, 4, pr.c_target)
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - gg[j]) < 1e-6 * max(1.0, abs(gg[j]))
        # f: dL = Re(conj(gf) df) -> real and imaginary directions
        for d in (1.0, 1j):
            f1, f2 = f.copy(), f.copy()
            f1[j] += h * d
            f2[j] -= h * d
            Lp, _ = grad.loss_target(pts, f1, 4, 4, pr.c_target)
            Lm, _ = grad.loss_target(pts, f2, 4, 4, pr.c_target)
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - np.real(np.conj(gf[j]) * d)) < 1e-6 * max(1.0, abs(gf[j]))
