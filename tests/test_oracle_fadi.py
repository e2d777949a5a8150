"""Pins of the oracle's fADI pieces (CPU only).

Each check is fixed by mathematics other than the code under test:
* the ADI error identity X - X_s = r(A) X r(B)^{-1} (closed form, any shifts);
* one shift at the exact eigenvalues reproduces a 1 x 1 Cauchy matrix;
* the Moebius map sends the four arc ends to (-gamma, -1, 1, gamma) and the
  arcs into the real intervals;
* the single optimal shift on [1, gamma] is the geometric mean sqrt(gamma)
  (dn(K/2) = sqrt(k')), and all shifts lie in [1, gamma];
* the shifted rational function stays within the Zolotarev bound on the arcs;
* the block factor reproduces the kernel matrix G(J_a, K_a^c) of Section 2.5
  entrywise within the Zolotarev bound;
* the 1D HSS built on it approximates G to the truncation tolerance.
"""
import math

import numpy as np
import pytest

from oracle import fadi, hss, nudft


def _rand_c(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_adi_error_identity_random_shifts():
    rng = np.random.default_rng(11)
    a = fadi.arc_point(rng.uniform(0.0, 0.2, 37))
    b = fadi.arc_point(rng.uniform(0.3, 0.9, 23))
    c, d = _rand_c(rng, 37), _rand_c(rng, 23)
    X = np.outer(c, d) / (a[:, None] - b[None, :])
    for s in (1, 3, 7):
        p = fadi.arc_point(rng.uniform(0.0, 0.2, s))
        q = fadi.arc_point(rng.uniform(0.3, 0.9, s))
        Z, Y, w = fadi.fadi(a, b, c, d, p, q)
        Xs = (Z * w[None, :]) @ Y.T
        # closed form of the error, built from r alone
        r_a = np.prod([(a - pj) / (a - qj) for pj, qj in zip(p, q)], axis=0)
        r_b = np.prod([(b - pj) / (b - qj) for pj, qj in zip(p, q)], axis=0)
        E = r_a[:, None] * X / r_b[None, :]
        assert np.abs(X - Xs - E).max() <= 1e-13 * np.abs(X).max()


def test_fadi_single_exact_shift_is_exact():
    a, b, c, d = 0.3 + 0.4j, -1.0 + 0.5j, 2.0 - 1.0j, 0.5 + 0.25j
    Z, Y, w = fadi.fadi([a], [b], np.array([c]), np.array([d]), np.array([a]), np.array([b]))
    assert abs(Z[0, 0] * w[0] * Y[0, 0] - c * d / (a - b)) < 1e-15


@pytest.mark.parametrize("arcs", [(0.0, 1 / 32, 1 / 32 + 2 / 512, 1 - 2 / 512),
                                  (0.25, 0.5, 0.5 + 1 / 64, 1.25 - 1 / 64),
                                  (0.875, 1.0, 1.0 + 3 / 128, 1.875 - 3 / 128)])
def test_symmetric_map(arcs):
    e0, e1, f0, f1 = arcs
    g, T, T_inv = fadi.symmetric_map(e0, e1, f0, f1)
    assert g > 1.0
    assert abs(T(fadi.arc_point(e0)) + g) < 1e-9 * g
    assert abs(T(fadi.arc_point(e1)) + 1.0) < 1e-12
    assert abs(T(fadi.arc_point(f1)) - g) < 1e-9 * g
    assert abs(T_inv(-g + 0j) - fadi.arc_point(e0)) < 1e-9
    assert abs(T_inv(g + 0j) - fadi.arc_point(f1)) < 1e-9
    wE = np.array([T(fadi.arc_point(t)) for t in np.linspace(e0, e1, 41)[1:-1]])
    wF = np.array([T(fadi.arc_point(t)) for t in np.linspace(f0, f1, 41)[1:-1]])
    assert np.abs(wE.imag).max() < 1e-8 * g and np.abs(wF.imag).max() < 1e-8 * g
    assert np.all((wE.real < -1.0) & (wE.real > -g))
    assert np.all((wF.real > 1.0) & (wF.real < g))


@pytest.mark.parametrize("gamma", [3.0, 320.7, 1.06e5])
def test_symmetric_shifts(gamma):
    w1 = fadi.symmetric_shifts(gamma, 1)
    assert abs(w1[0] - math.sqrt(gamma)) < 1e-12 * math.sqrt(gamma)
    for s in (2, 5, 12):
        w = fadi.symmetric_shifts(gamma, s)
        assert np.all(np.diff(w) < 0) and w[0] < gamma and w[-1] > 1.0
        # symmetric in the sense w_j w_{s+1-j} = gamma (the map x -> gamma/x
        # swaps the ends of [1, gamma])
        assert np.allclose(w * w[::-1], gamma, rtol=1e-12)
        xs = np.geomspace(1.0, gamma, 20001)
        err = np.max(np.abs(np.prod([(xs - wj) / (xs + wj) for wj in w], axis=0))) ** 2
        assert err <= fadi.zolotarev_bound(gamma, s)


@pytest.mark.parametrize("arcs,s", [((0.0, 1 / 32, 1 / 32 + 2 / 512, 1 - 2 / 512), 9),
                                    ((0.5, 0.75, 0.75 + 1 / 256, 1.5 - 1 / 256), 13)])
def test_zolotarev_shifts_on_arcs(arcs, s):
    e0, e1, f0, f1 = arcs
    p, q = fadi.zolotarev_shifts(e0, e1, f0, f1, s)
    assert np.allclose(np.abs(p), 1.0, atol=1e-12) and np.allclose(np.abs(q), 1.0, atol=1e-12)
    tp = np.mod(-np.angle(p) / (2 * np.pi) - e0, 1.0)
    tq = np.mod(-np.angle(q) / (2 * np.pi) - e0, 1.0)
    assert np.all(tp <= e1 - e0 + 1e-12) and np.all((tq >= f0 - e0 - 1e-12) & (tq <= f1 - e0 + 1e-12))
    g = fadi.gamma_of(e0, e1, f0, f1)
    rE = np.abs(fadi.adi_rational(fadi.arc_point(np.linspace(e0, e1, 4001)), p, q)).max()
    rF = np.abs(fadi.adi_rational(fadi.arc_point(np.linspace(f0, f1, 40001)), p, q)).min()
    assert rE / rF <= fadi.zolotarev_bound(g, s) * (1 + 1e-9)


def test_shift_count():
    g = 320.7
    for tau in (1e-3, 1e-6, 1e-11):
        s = fadi.shift_count(g, tau)
        assert fadi.zolotarev_bound(g, s) <= tau < fadi.zolotarev_bound(g, s - 1) or s == 1


@pytest.mark.parametrize("n,level,a,tau", [(128, 3, 0, 1e-6), (128, 3, 7, 1e-6), (128, 1, 1, 1e-9),
                                           (96, 2, 2, 1e-4), (64, 2, 1, 1e-11), (20, 2, 3, 1e-6)])
def test_row_block_factor_matches_kernel(n, level, a, tau):
    rng = np.random.default_rng(5 + n + level + a)
    x = rng.uniform(0.0, 1.0, 3000)
    rows = np.nonzero(hss.row_bins(x, level) == a)[0]
    f = fadi.row_block_factor(x[rows], n, level, a, tau)
    cols = hss.col_range(n, level, a)
    kc = np.setdiff1d(np.arange(n), cols)
    # near and far columns partition K^c; far ones lie >= b/n off the interval
    assert sorted(np.concatenate([f.near, f.far]).tolist()) == kc.tolist()
    if f.b:
        lo, hi = a / (1 << level), (a + 1) / (1 << level)
        dist = np.minimum(np.mod(f.far / n - hi, 1.0), np.mod(lo - f.far / n, 1.0))
        assert dist.min() >= f.b / n - 1e-15
    G = nudft.kernel_1d(x[rows], n, kc)
    app = f.Z @ f.Mt[kc].T
    assert np.all(f.Mt[cols] == 0)
    bound = fadi.zolotarev_bound(f.gamma, f.s) if f.b else 0.0
    assert np.all(np.abs(G - app) <= bound * np.abs(G) + 1e-13)
    assert np.abs(G - app).max() <= tau * np.abs(G).max()


@pytest.mark.parametrize("n,L,tol", [(64, 2, 1e-6), (128, 3, 1e-4), (48, 2, 1e-9)])
def test_hss_1d_fadi_accuracy(n, L, tol):
    rng = np.random.default_rng(n + L)
    x = rng.uniform(0.0, 1.0, 4 * n)
    h = fadi.hss_1d_fadi(x, n, L, tol)
    G = nudft.kernel_1d(x, n)
    H = hss.expand(h, x.size, n)
    assert np.linalg.norm(H - G) <= 4 * tol * np.linalg.norm(G)
    for k in h.tree.level(L):
        U = h.U[k]
        assert np.allclose(U.conj().T @ U, np.eye(U.shape[1]), atol=1e-12)
