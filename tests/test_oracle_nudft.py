"""Pins for the oracle's transform, adjoint, least squares and kernel.

Each test fixes an oracle function against something other than itself: an
FFT, a pure-Python brute force, a closed form or an identity the paper states.
"""
import cmath
import math

import numpy as np
import pytest

from nudft_inputs import jittered_points, complex_normal, make_problem
from oracle import nudft


def grid_points(mx, my):
    p = np.repeat(np.arange(mx), my) / mx
    q = np.tile(np.arange(my), mx) / my
    return np.stack([p, q], axis=1).astype(np.float64)


def test_apply_exact_grid_is_fft2():
    # Section 1.1 (related work): on the uniform grid x = p/n the transform is a
    # 2D DFT.  With centred k the sum picks up the sign (-1)^(p+q).
    nx, ny = 8, 6
    rng = np.random.default_rng(0)
    c = complex_normal(rng, (nx, ny))
    pts = grid_points(nx, ny)
    f = nudft.apply(pts, c).reshape(nx, ny)
    sign = (-1.0) ** (np.arange(nx)[:, None] + np.arange(ny)[None, :])
    ref = sign * np.fft.fft2(c)
    assert np.max(np.abs(f - ref)) < 1e-12 * np.max(np.abs(ref))


def test_apply_brute_force_tiny():
    # pure-Python double sum with cmath.exp, n = 2..4
    rng = np.random.default_rng(1)
    for nx, ny in [(2, 2), (2, 4), (4, 2), (4, 4)]:
        pts = rng.uniform(0, 1, size=(7, 2))
        c = complex_normal(rng, (nx, ny))
        f = nudft.apply(pts, c)
        A = nudft.dense_matrix(pts, nx, ny)
        for j in range(7):
            s = 0j
            for i in range(nx):
                for i2 in range(ny):
                    kx, ky = i - nx // 2, i2 - ny // 2
                    s += c[i, i2] * cmath.exp(-2j * math.pi * (kx * pts[j, 0] + ky * pts[j, 1]))
                    col = i2 + i * ny
                    assert abs(A[j, col] - cmath.exp(-2j * math.pi * (kx * pts[j, 0] + ky * pts[j, 1]))) < 1e-14
            assert abs(f[j] - s) < 1e-13


def test_face_splitting_rows():
    # Section 3.1: A = A^x face-split A^y, row j = kron(A^x(j,:), A^y(j,:)),
    # checked against the definition with explicit loops.
    rng = np.random.default_rng(2)
    pts = rng.uniform(0, 1, size=(5, 2))
    nx, ny = 4, 6
    A = nudft.dense_matrix(pts, nx, ny)
    Ax = nudft.nudft_1d(pts[:, 0], nx)
    Ay = nudft.nudft_1d(pts[:, 1], ny)
    for j in range(5):
        row = np.array([Ax[j, a] * Ay[j, b] for a in range(nx) for b in range(ny)])
        assert np.allclose(A[j], row, atol=1e-15, rtol=0)


def test_adjoint_identity():
    rng = np.random.default_rng(3)
    pts = jittered_points(rng, 12, 10, 0.3)
    c = complex_normal(rng, (6, 4))
    f = complex_normal(rng, (pts.shape[0],))
    lhs = np.vdot(f, nudft.apply(pts, c))
    rhs = np.vdot(nudft.apply_adj(pts, f, 6, 4), c)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_adjoint_matches_dense():
    rng = np.random.default_rng(4)
    pts = jittered_points(rng, 8, 8, 0.25)
    f = complex_normal(rng, (2, 64))
    A = nudft.dense_matrix(pts, 4, 4)
    got = nudft.apply_adj(pts, f, 4, 4)
    for r in range(2):
        assert np.allclose(got[r].reshape(-1), A.conj().T @ f[r], atol=1e-12)


def test_phase_reduction_exact():
    # (k x mod 1) with k up to 256 and x with a full mantissa: compare with
    # exact rational arithmetic.
    from fractions import Fraction
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, 20)
    k = np.array([-256, -7, 0, 3, 255])
    t = nudft.phase_turns(k, x)
    for i in range(20):
        for jj, kk in enumerate(k):
            ex = Fraction(float(x[i])) * int(kk)
            ex = ex - round(ex)
            assert abs(float(ex) - t[i, jj]) <= 2e-16


def test_lstsq_exact_grid_inverse_fft():
    # exact grid, M = N: c* = ifft2 of the sign-corrected samples
    nx, ny = 8, 8
    rng = np.random.default_rng(6)
    pts = grid_points(nx, ny)
    f = complex_normal(rng, (nx * ny,))
    c = nudft.lstsq(pts, f, nx, ny)
    sign = (-1.0) ** (np.arange(nx)[:, None] + np.arange(ny)[None, :])
    ref = np.fft.ifft2(sign * f.reshape(nx, ny))
    assert np.max(np.abs(c - ref)) < 1e-12


def test_lstsq_oversampled_grid_is_scaled_adjoint():
    # oversampled grid m = 2n, no jitter: A^*A = M I so c* = A^* f / M
    nx, ny = 4, 6
    rng = np.random.default_rng(7)
    pts = grid_points(2 * nx, 2 * ny)
    f = complex_normal(rng, (pts.shape[0],))
    c = nudft.lstsq(pts, f, nx, ny)
    A = nudft.dense_matrix(pts, nx, ny)
    assert np.allclose(A.conj().T @ A, pts.shape[0] * np.eye(nx * ny), atol=1e-10)
    ref = (A.conj().T @ f).reshape(nx, ny) / pts.shape[0]
    assert np.max(np.abs(c - ref)) < 1e-13


def test_lstsq_consistent_rhs_recovers_truth():
    pr = make_problem(8, 8, 16, 16, 0.3, 11)
    f = nudft.apply(pr.points, pr.c_true)
    c = nudft.lstsq(pr.points, f, 8, 8)
    assert nudft.rel_err(c, pr.c_true) < 1e-12


def test_lstsq_matches_pinv_and_normal_equations():
    rng = np.random.default_rng(8)
    pts = rng.uniform(0, 1, size=(40, 2))
    f = complex_normal(rng, (40,))
    c = nudft.lstsq(pts, f, 4, 4).reshape(-1)
    A = nudft.dense_matrix(pts, 4, 4)
    c_pinv = np.linalg.pinv(A) @ f
    c_ne = np.linalg.solve(A.conj().T @ A, A.conj().T @ f)
    assert np.allclose(c, c_pinv, atol=1e-11)
    assert np.allclose(c, c_ne, atol=1e-9)


@pytest.mark.parametrize("n", [8, 16, 32])
def test_kernel_is_rowwise_inverse_dft(n):
    # G^x = A^x F^{-1} (Section 2.5): row-wise inverse FFT of the 0-based
    # NUDFT matrix equals the closed-form kernel.
    rng = np.random.default_rng(n)
    x = rng.uniform(0, 1, 50)
    x[:5] = np.arange(5) / n            # include exact coincidences gamma = xi
    A0 = nudft.nudft_1d(x, n, centred=False)
    G_fft = np.fft.ifft(A0, axis=1)     # A F^{-1}: F^{-1} = conj(F)/n acts as ifft on rows
    G = nudft.kernel_1d(x, n)
    assert np.max(np.abs(G - G_fft)) < 1e-13
    assert np.allclose(G[np.arange(5), np.arange(5)], 1.0, atol=1e-15)


def test_kernel_sylvester_displacement():
    # Gamma G - G D = u v^T with u_j = gamma_j^n - 1, v_l = xi_l / n
    n = 16
    rng = np.random.default_rng(9)
    x = rng.uniform(0, 1, 30)
    G = nudft.kernel_1d(x, n)
    gam = np.exp(-2j * np.pi * x)
    xi = np.exp(-2j * np.pi * np.arange(n) / n)
    lhs = gam[:, None] * G - G * xi[None, :]
    u = gam ** n - 1.0
    v = xi / n
    assert np.max(np.abs(lhs - np.outer(u, v))) < 1e-13
    s = np.linalg.svd(lhs, compute_uv=False)
    assert s[1] < 1e-12 * s[0]


def test_kernel_equal_row_norms():
    # Lemma 3.4: every row of G^x, G^y and G has norm 1 (rows of A have norm
    # sqrt(n) and F/sqrt(n) is unitary); ||G||_F = sqrt(M).
    pr = make_problem(8, 16, 16, 32, 0.4, 12)
    G = nudft.dense_G(pr.points, 8, 16)
    norms = np.linalg.norm(G, axis=1)
    assert np.allclose(norms, 1.0, atol=1e-13)
    assert abs(np.linalg.norm(G) - np.sqrt(pr.M)) < 1e-10


def test_centring_phase_relation():
    pr = make_problem(8, 4, 16, 8, 0.3, 13)
    A_c = nudft.dense_matrix(pr.points, 8, 4, centred=True)
    A_0 = nudft.dense_matrix(pr.points, 8, 4, centred=False)
    phi = nudft.centring_phase(pr.points, 8, 4)
    assert np.max(np.abs(A_c - phi[:, None] * A_0)) < 1e-13


def test_G_times_F_is_A():
    # A = G F with F = F^x (x) F^y (Section 3.1)
    pr = make_problem(4, 8, 8, 16, 0.3, 14)
    G = nudft.dense_G(pr.points, 4, 8)
    F = np.kron(nudft.dft_matrix(4), nudft.dft_matrix(8))
    A0 = nudft.dense_matrix(pr.points, 4, 8, centred=False)
    assert np.max(np.abs(G @ F - A0)) < 1e-12
    # F c <-> fft2 of the C-order array
    c = complex_normal(np.random.default_rng(0), (4, 8))
    assert np.allclose(F @ c.reshape(-1), np.fft.fft2(c).reshape(-1), atol=1e-12)


def test_face_product_norm_lemma():
    # Lemma 2.1 on random matrices
    rng = np.random.default_rng(15)
    for _ in range(5):
        A1 = complex_normal(rng, (9, 4))
        A2 = complex_normal(rng, (9, 3))
        F = (A1[:, :, None] * A2[:, None, :]).reshape(9, 12)
        b1 = np.max(np.linalg.norm(A1, axis=1)) * np.linalg.norm(A2)
        b2 = np.max(np.linalg.norm(A2, axis=1)) * np.linalg.norm(A1)
        assert np.linalg.norm(F) <= min(b1, b2) * (1 + 1e-12)


def test_face_product_rank_lemma():
    # Lemma 3.1: rank(A1 . A2) <= rank A1 rank A2, via (U1 . U2)(V1 (x) V2)^*
    rng = np.random.default_rng(16)
    U1, V1 = complex_normal(rng, (30, 2)), complex_normal(rng, (7, 2))
    U2, V2 = complex_normal(rng, (30, 3)), complex_normal(rng, (5, 3))
    A1, A2 = U1 @ V1.conj().T, U2 @ V2.conj().T
    F = (A1[:, :, None] * A2[:, None, :]).reshape(30, 35)
    s = np.linalg.svd(F, compute_uv=False)
    assert np.sum(s > 1e-10 * s[0]) <= 6
    UU = (U1[:, :, None] * U2[:, None, :]).reshape(30, 6)
    assert np.allclose(F, UU @ np.kron(V1, V2).conj().T, atol=1e-12)
