"""fADI factors of the HSS row blocks of the 1D transformed NUDFT matrix
(oracle, test infrastructure: only the tests, the smoke check and the
benchmark's CPU leg may import it).

Section 2.5: with g_j = exp(-2 pi i x_j) and xi_l = exp(-2 pi i l/n), the
matrix G = A F^{-1} satisfies the displacement (Sylvester) equation

    diag(g) G - G diag(xi) = u v^T,   u_j = g_j^n - 1,   v_l = xi_l / n,

so G(j, l) = u_j v_l / (g_j - xi_l).  The paper builds its 1D HSS
approximations from this equation with the factored ADI method (fADI, of
Benner, Li and Truhar) followed by an interpolative decomposition, and only
cites the construction.  This module writes out the pieces from their
published definitions:

* ``symmetric_map``: the Moebius transformation taking two disjoint arcs E, F of
  the unit circle onto [-gamma, -1] and [1, gamma] (a Moebius map is fixed by
  three points; the fourth lands on gamma because the cross-ratio is
  invariant).
* ``zolotarev_shifts``: the optimal ADI shifts for [-gamma, -1] x [1, gamma],
  +-gamma dn((2j - 1) K / (2s), k), k = sqrt(1 - gamma^-2) (the elliptic-
  function parameters of Wachspress), carried back to the arcs, and the shift
  count from Beckermann and Townsend's bound on the Zolotarev number,
  Z_s <= 4 exp(-pi^2 s / log(16 gamma)).
* ``fadi``: the fADI recurrences for A X - X B = c d^T with diagonal A, B:
      z_1 = (A - q_1)^{-1} c,  z_{j+1} = z_j + (q_{j+1} - p_j)(A - q_{j+1})^{-1} z_j,
      y_1 = (B - p_1)^{-1} d,  y_{j+1} = y_j + (p_{j+1} - q_j)(B - p_{j+1})^{-1} y_j,
      X_s = sum_j (q_j - p_j) z_j y_j^T,
  whose error is X - X_s = r(A) X r(B)^{-1}, r(z) = prod_j (z - p_j)/(z - q_j).
* ``row_block_factor``: the HSS row block G(J_a, K_a^c) of node (level, a) of
  the 1D tree (Theorem 2.2's index sets).  Its arc E (the node's interval)
  touches the frequencies just outside the interval, so the b columns next to
  each end of the interval are kept exactly and fADI runs on the remaining
  ("far") columns, which lie at least b/n away.  Result: G(J_a, l) ~= sum_j
  Z(., j) Mt(l, j) for every l in K_a^c (Mt(l, .) = 0 for l in K_a).  The
  number of near columns and of shifts is the cheapest pair that reaches the
  requested accuracy.
* ``hss_1d_fadi``: a 1D HSS approximation whose leaf row bases come from these
  factors (thin QR of Z, truncated SVD of the small core); everything else is
  ``hss.hss_1d``'s.

Readings: the paper gives neither the shift strategy for the adjacent arcs nor
the accuracy split between fADI and the truncation; here fADI is run to a
tenth of the truncation tolerance (its error is entrywise, |err| <= Z_s |G|),
and near columns are tried in the counts 1, 2, 3, 4, 6, 8.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np

from . import hss, nudft

NEAR_COUNTS = (1, 2, 3, 4, 6, 8)
FADI_TOL_FRACTION = 0.1


def arc_point(theta):
    """exp(-2 pi i theta): the point of the unit circle for turn theta."""
    return np.exp(-2j * np.pi * np.asarray(theta, dtype=np.float64))


def cross_ratio(z1, z2, z3, z4):
    return ((z1 - z3) * (z2 - z4)) / ((z1 - z4) * (z2 - z3))


def gamma_of(e0, e1, f0, f1) -> float:
    """gamma > 1 of [-gamma, -1] u [1, gamma], the image of the arcs
    E = c([e0, e1]), F = c([f0, f1]) (turns, e0 < e1 < f0 < f1 < e0 + 1):
    the cross-ratio of (-gamma, -1, 1, gamma) is (1 + gamma)^2 / (4 gamma)."""
    rho = cross_ratio(arc_point(e0), arc_point(e1), arc_point(f0), arc_point(f1)).real
    return 2.0 * rho - 1.0 + 2.0 * math.sqrt(rho * rho - rho)


def symmetric_map(e0, e1, f0, f1):
    """(gamma, T, T_inv): T Moebius with T(c(e0)) = -gamma, T(c(e1)) = -1,
    T(c(f0)) = 1, hence T(c(f1)) = gamma."""
    g = gamma_of(e0, e1, f0, f1)
    z1, z2, z3 = arc_point(e0), arc_point(e1), arc_point(f0)
    w1, w2, w3 = -g, -1.0, 1.0

    def S(z, a, b, c):          # a -> 0, b -> 1, c -> infinity
        return ((z - a) * (b - c)) / ((z - c) * (b - a))

    def S_inv(s, a, b, c):
        k = s * (b - a) / (b - c)
        return (a - k * c) / (1.0 - k)

    def T(z):
        return S_inv(S(z, z1, z2, z3), w1, w2, w3)

    def T_inv(w):
        return S_inv(S(w, w1, w2, w3), z1, z2, z3)

    return g, T, T_inv


def shift_count(gamma: float, tau: float) -> int:
    """Smallest s with 4 exp(-pi^2 s / log(16 gamma)) <= tau."""
    return max(1, int(math.ceil(math.log(4.0 / tau) * math.log(16.0 * gamma) / math.pi ** 2)))


def zolotarev_bound(gamma: float, s: int) -> float:
    return 4.0 * math.exp(-math.pi ** 2 * s / math.log(16.0 * gamma))


def symmetric_shifts(gamma: float, s: int) -> np.ndarray:
    """w_j = gamma dn((2j - 1) K(k) / (2s), k), k^2 = 1 - gamma^-2, j = 1..s:
    the zeros of the optimal rational function on [-gamma, -1] are -w_j and
    its poles on [1, gamma] are +w_j.  Evaluated in 30-digit arithmetic."""
    with mpmath.workdps(30):
        m = 1 - mpmath.mpf(1) / mpmath.mpf(gamma) ** 2
        K = mpmath.ellipk(m)
        w = [gamma * float(mpmath.ellipfun('dn', (2 * j - 1) * K / (2 * s), m=m))
             for j in range(1, s + 1)]
    return np.array(w, dtype=np.float64)


def zolotarev_shifts(e0, e1, f0, f1, s: int):
    """ADI shifts p (on E) and q (on F) for the arcs E = c([e0, e1]),
    F = c([f0, f1]): the symmetric shifts mapped back through T^{-1}."""
    g, _, T_inv = symmetric_map(e0, e1, f0, f1)
    w = symmetric_shifts(g, s)
    return T_inv(-w.astype(np.complex128)), T_inv(w.astype(np.complex128))


def fadi(a, b, c, d, p, q):
    """fADI for diag(a) X - X diag(b) = c d^T with shifts p, q: returns Z, Y
    and the weights q - p with X_s = Z diag(q - p) Y^T."""
    a, b = np.asarray(a, complex), np.asarray(b, complex)
    s = len(p)
    Z = np.empty((a.size, s), complex)
    Y = np.empty((b.size, s), complex)
    Z[:, 0] = c / (a - q[0])
    Y[:, 0] = d / (b - p[0])
    for j in range(1, s):
        Z[:, j] = Z[:, j - 1] + (q[j] - p[j - 1]) * Z[:, j - 1] / (a - q[j])
        Y[:, j] = Y[:, j - 1] + (p[j] - q[j - 1]) * Y[:, j - 1] / (b - p[j])
    return Z, Y, np.asarray(q) - np.asarray(p)


def adi_rational(z, p, q):
    """r(z) = prod_j (z - p_j) / (z - q_j)."""
    z = np.asarray(z, complex)
    r = np.ones(z.shape, complex)
    for pj, qj in zip(p, q):
        r = r * (z - pj) / (z - qj)
    return r


def displacement_terms(x, n: int):
    """g, u of the rows and xi, v of the columns (Section 2.5), u_j =
    g_j^n - 1 with n x_j reduced mod 1 in extended precision first (f), then
    written as exp(-2 pi i f) - 1 = -2i sin(pi f) exp(-i pi f), which keeps
    its relative accuracy when f is near 0."""
    xl = np.asarray(x, dtype=np.longdouble)
    t = xl * n
    frac = (t - np.rint(t)).astype(np.float64)
    g = arc_point(x)
    u = -2j * np.sin(np.pi * frac) * np.exp(-1j * np.pi * frac)
    xi = arc_point(np.arange(n) / n)
    v = xi / n
    return g, u, xi, v


class BlockFactor:
    """G(J, l) ~= sum_j Z(:, j) Mt(l, j) for l in K^c (Mt(l, :) = 0 on K)."""

    def __init__(self, near, far, b, s, p, q, gamma, Z, Mt):
        self.near, self.far, self.b, self.s = near, far, b, s
        self.p, self.q, self.gamma = p, q, gamma
        self.Z, self.Mt = Z, Mt


def block_plan(n: int, level: int, a: int, tau: float):
    """(b, s, gamma, arcs): b = 0 means every column of K^c is kept exactly."""
    cols = hss.col_range(n, level, a)
    lo, hi = -(-a * n // (1 << level)), -(-(a + 1) * n // (1 << level))
    nc = n - cols.size
    best = (nc, 0, 0, 0.0, None)            # cost, b, s, gamma, arcs
    e0, e1 = a / (1 << level), (a + 1) / (1 << level)
    for b in NEAR_COUNTS:
        nf = nc - 2 * b
        if nf <= 0:
            break
        f0, f1 = (hi + b) / n, (lo - b - 1 + n) / n
        g = gamma_of(e0, e1, f0, f1)
        s = shift_count(g, tau)
        if 2 * b + s < best[0]:
            best = (2 * b + s, b, s, g, (e0, e1, f0, f1))
    return best[1], best[2], best[3], best[4], lo, hi


def row_block_factor(x_rows, n: int, level: int, a: int, tau: float,
                     shifts=None) -> BlockFactor:
    """fADI factor of G(J_a, K_a^c) for the rows x_rows of node (level, a).
    shifts: optional (p, q) used in place of the computed Zolotarev shifts
    (the same count), so that the recurrences can be compared on given
    inputs."""
    b, s, g, arcs, lo, hi = block_plan(n, level, a, tau)
    x_rows = np.asarray(x_rows, dtype=np.float64)
    cols = hss.col_range(n, level, a)
    kc = np.setdiff1d(np.arange(n), cols)
    if b == 0:
        Z = nudft.kernel_1d(x_rows, n, kc)
        Mt = np.zeros((n, kc.size), complex)
        Mt[kc, np.arange(kc.size)] = 1.0
        return BlockFactor(kc, np.zeros(0, np.int64), 0, 0, None, None, 0.0, Z, Mt)
    near = np.array([(hi + i) % n for i in range(b)] + [(lo - b + i) % n for i in range(b)],
                    dtype=np.int64)
    far = np.array([l % n for l in range(hi + b, lo - b + n)], dtype=np.int64)
    p, q = zolotarev_shifts(*arcs, s) if shifts is None else shifts
    assert len(p) == s and len(q) == s
    gr, u, xi, v = displacement_terms(x_rows, n)
    Zf, Yf, w = fadi(gr, xi[far], u, v[far], p, q)
    Z = np.hstack([nudft.kernel_1d(x_rows, n, near), Zf])
    Mt = np.zeros((n, 2 * b + s), complex)
    Mt[near, np.arange(2 * b)] = 1.0
    Mt[far, 2 * b:] = Yf * w[None, :]
    return BlockFactor(near, far, b, s, p, q, g, Z, Mt)


def hss_1d_fadi(x: np.ndarray, n: int, L: int, tol: float) -> hss.HSS:
    """hss.hss_1d with the leaf row bases from the fADI factors: U_a spans
    Z R^{-1} of the truncated SVD of the core R Mt(K^c)^T (Z = Q R)."""
    h = hss.hss_1d(x, n, L, 0.0) if L == 0 else None
    if h is not None:
        return h
    t = hss.tree_1d(x, n, L)
    leafU = {}
    for k in t.level(L):
        nd = t.nodes[k]
        f = row_block_factor(x[nd.rows], n, L, k[1], FADI_TOL_FRACTION * tol)
        kc = np.setdiff1d(np.arange(n), nd.cols)
        Q, R = hss.thin_qr(f.Z)
        Uc, _ = hss.trunc_left(R @ f.Mt[kc].T, tol)
        leafU[k] = Q @ Uc
    return hss.hss_1d(x, n, L, tol, leaf_row_bases=leafU)
