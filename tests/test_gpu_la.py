"""GPU checks of the batched dense building blocks (GEMM, Householder QR,
Q application, pivoted Cholesky, triangular solve) against NumPy/LAPACK."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

nd = pytest.importorskip("paper_2607_00928_amd")
from paper_2607_00928_amd import _lib  # noqa: E402

lib = _lib.lib
DEV = torch.device("cuda", 0)
CT = {0: (np.complex128, torch.complex128), 1: (np.complex64, torch.complex64)}
CT[2] = CT[1]   # complex64 with the products on the bf16 split
TOL = {0: 1e-12, 1: 2e-5, 2: 2e-5}
QB = 256   # reflectors per compact-WY block of the QR factors (T layout)


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def to_dev(Mat, prec, cols=None):
    """column-major device copy (ld = rows)"""
    npt, tt = CT[prec]
    return torch.from_numpy(np.ascontiguousarray(Mat.T.astype(npt))).to(DEV)


def from_dev(t, m, n):
    return t.cpu().numpy().reshape(n, m).T


def i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(C.POINTER(C.c_int64))


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("opa,opb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_batched_ragged(prec, opa, opb):
    rng = np.random.default_rng(10 * prec + 2 * opa + opb)
    shapes = [(1, 1, 1), (70, 33, 19), (64, 64, 64), (130, 5, 200), (3, 150, 17), (65, 129, 0)]
    if prec == 2:   # a k = 1 product keeps its launch on the FP32 instructions
        shapes[0] = (1, 1, 2)
    mats, keep = [], []
    mnk, ld, ptr = [], [], []
    alpha = 0.7 - 0.3j
    for (m, n, k) in shapes:
        A = crandn(rng, *((m, k) if opa == 0 else (k, m)))
        B = crandn(rng, *((k, n) if opb == 0 else (n, k)))
        Cm = crandn(rng, m, n)
        ta, tb, tc = to_dev(A, prec), to_dev(B, prec), to_dev(Cm, prec)
        keep += [ta, tb, tc]
        mats.append((A, B, Cm, tc))
        mnk += [m, n, k]
        ld += [max(A.shape[0], 1), max(B.shape[0], 1), max(m, 1)]
        ptr += [ta.data_ptr(), tb.data_ptr(), tc.data_ptr()]
    a1, p1 = i32(mnk)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    st = lib.nudft2_test_gemm(prec, opa, opb, len(shapes), p1, p2, p3, alpha.real, alpha.imag, 1.0)
    assert st == 0, lib.nudft2_last_error()
    for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
        oA = A if opa == 0 else A.conj().T
        oB = B if opb == 0 else B.conj().T
        ref = alpha * (oA @ oB) + Cm
        got = from_dev(tc, m, n)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() < TOL[prec] * scale * max(1, k) ** 0.5 * 10, (m, n, k)


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("opa,opb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_fp32_entrywise_error(prec, opa, opb):
    """Each entry of a complex64 product against the FP64 product of the same
    (rounded) operands, relative to (|op(A)| |op(B)|)_ij: FP32 rounding of k
    products and sums stays within a few times 2^-24 sqrt(k) of it.  The bf16
    split (prec 2) must meet the same bound as the FP32 instructions: a
    dropped split product (a0 b1, a1 b0: 2^-8; a0 b2, a1 b1, a2 b0: 2^-16)
    or a lost plane would exceed it by orders of magnitude.  Odd k (the split
    kernel reads k in pairs), k = 2, tiles past the matrix edge, long k with
    the library's split choice, alpha complex, beta = 0.5."""
    rng = np.random.default_rng(300 + 4 * prec + 2 * opa + opb)
    shapes = [(70, 33, 19), (2, 3, 2), (129, 65, 33), (64, 64, 64), (200, 150, 999),
              (17, 300, 3001), (1, 130, 77)]
    alpha, beta = 0.8 - 0.5j, 0.5
    mats, keep, mnk, ld, ptr = [], [], [], [], []
    for (m, n, k) in shapes:
        A = crandn(rng, *((m, k) if opa == 0 else (k, m))).astype(np.complex64)
        B = crandn(rng, *((k, n) if opb == 0 else (n, k))).astype(np.complex64)
        Cm = crandn(rng, m, n).astype(np.complex64)
        ts = [to_dev(X, prec) for X in (A, B, Cm)]
        keep += ts
        mats.append((A, B, Cm, ts[2]))
        mnk += [m, n, k]
        ld += [A.shape[0], B.shape[0], m]
        ptr += [t.data_ptr() for t in ts]
    a1, p1 = i32(mnk)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    st = lib.nudft2_test_gemm(prec, opa, opb, len(shapes), p1, p2, p3, alpha.real, alpha.imag, beta)
    assert st == 0, lib.nudft2_last_error()
    for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
        oA = (A if opa == 0 else A.conj().T).astype(np.complex128)
        oB = (B if opb == 0 else B.conj().T).astype(np.complex128)
        ref = alpha * (oA @ oB) + beta * Cm.astype(np.complex128)
        scale = abs(alpha) * (np.abs(oA) @ np.abs(oB)) + beta * np.abs(Cm)
        err = (np.abs(from_dev(tc, m, n) - ref) / scale).max()
        assert err < 8 * 2.0 ** -24 * np.sqrt(k), (m, n, k, err)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("opa", [0, 1])
@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_gemm_skinny(prec, opa, beta):
    """Products with at most 8 columns (the memory-bound path), including
    long k (split over workgroups) and a single row."""
    rng = np.random.default_rng(20 + 2 * prec + opa)
    shapes = [(1, 1, 1), (300, 1, 700), (5000, 3, 64), (17, 8, 3000), (64, 2, 40000), (1, 5, 9),
              (257, 7, 0)]
    mats, keep = [], []
    mnk, ld, ptr = [], [], []
    alpha = -0.4 + 1.1j
    for (m, n, k) in shapes:
        A = crandn(rng, *((m, k) if opa == 0 else (k, m)))
        B = crandn(rng, k, n)
        Cm = crandn(rng, m, n)
        ta, tb, tc = to_dev(A, prec), to_dev(B, prec), to_dev(Cm, prec)
        keep += [ta, tb, tc]
        mats.append((A, B, Cm, tc))
        mnk += [m, n, k]
        ld += [max(A.shape[0], 1), max(B.shape[0], 1), max(m, 1)]
        ptr += [ta.data_ptr(), tb.data_ptr(), tc.data_ptr()]
    a1, p1 = i32(mnk)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    st = lib.nudft2_test_gemm(prec, opa, 0, len(shapes), p1, p2, p3, alpha.real, alpha.imag, beta)
    assert st == 0, lib.nudft2_last_error()
    for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
        oA = A if opa == 0 else A.conj().T
        ref = alpha * (oA @ B) + beta * Cm
        got = from_dev(tc, m, n)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() < TOL[prec] * scale * max(1, k) ** 0.5 * 10, (m, n, k)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_gemm_skinny_ch_long_k_few_rows(prec, beta):
    """A^H B with at most 8 columns, a long k and few rows of C (the sweep's
    V^H c against a block of reflectors): a workgroup per row of C, no k
    split.  Ragged k (not a multiple of the 256-thread stride), one and eight
    columns, a row count that is not a multiple of anything."""
    rng = np.random.default_rng(400 + 2 * prec + int(beta > 0))
    shapes = [(256, 1, 11000), (200, 3, 9001), (5, 8, 4097), (77, 1, 2049)]
    alpha = 0.3 + 0.9j
    mats, keep, mnk, ld, ptr = [], [], [], [], []
    for (m, n, k) in shapes:
        A = crandn(rng, k, m)
        B = crandn(rng, k, n)
        Cm = crandn(rng, m, n)
        ts = [to_dev(X, prec) for X in (A, B, Cm)]
        keep += ts
        mats.append((A, B, Cm, ts[2]))
        mnk += [m, n, k]
        ld += [k, k, m]
        ptr += [t.data_ptr() for t in ts]
    a1, p1 = i32(mnk)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    st = lib.nudft2_test_gemm(prec, 1, 0, len(shapes), p1, p2, p3, alpha.real, alpha.imag, beta)
    assert st == 0, lib.nudft2_last_error()
    for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
        ref = alpha * (A.conj().T @ B) + beta * Cm
        got = from_dev(tc, m, n)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() < TOL[prec] * scale * k ** 0.5 * 10, (m, n, k)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_geqrf_ormqr(prec):
    rng = np.random.default_rng(3 + prec)
    # around the 256-column blocks and their 128-column halves: a block with
    # one reflector in its right half, exactly one block, a last block of one
    # half, several blocks with partial halves, wide problems
    shapes = [(100, 37), (37, 100), (64, 64), (5, 3), (1030, 546), (33, 1), (300, 97),
              (3000, 70), (257, 300), (700, 129), (400, 256), (130, 700), (2000, 600),
              (600, 384), (1000, 513)]
    keep = []
    mn, ld, ptr, data = [], [], [], []
    for (m, n) in shapes:
        A = crandn(rng, m, n)
        k = min(m, n)
        nob = (k + QB - 1) // QB
        tsize = QB * QB * (nob - 1) + (k - QB * (nob - 1)) ** 2
        tA = to_dev(A, prec)
        # R starts as garbage: the factorization must write all of it
        tR = torch.full((n, k), 7.0 - 3.0j, dtype=CT[prec][1], device=DEV)   # k x n col-major
        tT = torch.full((tsize,), 5.0 + 1.0j, dtype=CT[prec][1], device=DEV)
        keep += [tA, tR, tT]
        data.append((A, tA, tR, tT))
        mn += [m, n]
        ld += [m, k]
        ptr += [tA.data_ptr(), tR.data_ptr(), tT.data_ptr()]
    a1, p1 = i32(mn)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    st = lib.nudft2_test_geqrf(prec, len(shapes), p1, p2, p3)
    assert st == 0, lib.nudft2_last_error()
    # form Q (m x m) by applying Q to the identity, check Q R = A, Q unitary
    dims, ld2, ptr2, Qs = [], [], [], []
    for (m, n), (A, tA, tR, tT) in zip(shapes, data):
        tQ = to_dev(np.eye(m), prec)
        keep.append(tQ)
        Qs.append(tQ)
        dims += [m, min(m, n), m]
        ld2 += [m, m]
        ptr2 += [tA.data_ptr(), tT.data_ptr(), tQ.data_ptr()]
    b1, q1 = i32(dims)
    b2, q2 = i32(ld2)
    b3, q3 = i64(ptr2)
    st = lib.nudft2_test_ormqr(prec, 0, len(shapes), q1, q2, q3)
    assert st == 0, lib.nudft2_last_error()
    # explicit Q formation from the identity (trans = 2 skips the columns each
    # block leaves unchanged) must give the same Q
    ptr2i, Qi = [], []
    for (m, n), (A, tA, tR, tT) in zip(shapes, data):
        tQi = to_dev(np.eye(m), prec)
        keep.append(tQi)
        Qi.append(tQi)
        ptr2i += [tA.data_ptr(), tT.data_ptr(), tQi.data_ptr()]
    b4, q4 = i64(ptr2i)
    assert lib.nudft2_test_ormqr(prec, 2, len(shapes), q1, q2, q4) == 0, lib.nudft2_last_error()
    for (m, n), tQ, tQi in zip(shapes, Qs, Qi):
        d = np.abs(from_dev(tQi, m, m) - from_dev(tQ, m, m)).max()
        assert d < 10 * TOL[prec] * np.sqrt(m), (m, n, d)
    for (m, n), (A, tA, tR, tT), tQ in zip(shapes, data, Qs):
        k = min(m, n)
        Q = from_dev(tQ, m, m)
        R = from_dev(tR, k, n)
        assert np.abs(np.tril(R, -1)).max() == 0
        # A returns the explicit unit lower-trapezoidal reflectors
        V = from_dev(tA, m, n)[:, :k]
        assert np.abs(np.triu(V, 1)).max() == 0 and np.all(np.diag(V) == 1), (m, n)
        err = np.abs(Q[:, :k] @ R - A).max() / np.abs(A).max()
        orth = np.abs(Q.conj().T @ Q - np.eye(m)).max()
        print(f"qr {m}x{n} prec{prec}: recon {err:.1e} orth {orth:.1e}")
        assert err < 50 * TOL[prec] * np.sqrt(m)
        assert orth < 50 * TOL[prec] * np.sqrt(m)
        # |R| diagonal equals LAPACK's up to phases
        Rl = np.linalg.qr(A.astype(np.complex128), mode="r")
        assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rl)), rtol=1e-3 if prec else 1e-9)
    # Q^H (Q C) = C via the trans path
    dims3, ld3, ptr3, Cs = [], [], [], []
    for (m, n), (A, tA, tR, tT) in zip(shapes, data):
        Cm = crandn(rng, m, 7)
        tC = to_dev(Cm, prec)
        keep.append(tC)
        Cs.append((Cm, tC))
        dims3 += [m, min(m, n), 7]
        ld3 += [m, m]
        ptr3 += [tA.data_ptr(), tT.data_ptr(), tC.data_ptr()]
    c1, r1 = i32(dims3)
    c2, r2 = i32(ld3)
    c3, r3 = i64(ptr3)
    assert lib.nudft2_test_ormqr(prec, 0, len(shapes), r1, r2, r3) == 0
    assert lib.nudft2_test_ormqr(prec, 1, len(shapes), r1, r2, r3) == 0
    for (m, n), (Cm, tC) in zip(shapes, Cs):
        got = from_dev(tC, m, 7)
        assert np.abs(got - Cm).max() < 100 * TOL[prec] * np.sqrt(m)


def test_pchol_trace_rule():
    rng = np.random.default_rng(7)
    # up to 1100 rows: five cooperating workgroups per Gram, several panels
    sizes = [(40, 40), (300, 120), (473, 473), (17, 5), (1100, 70)]
    keep, data = [], []
    w, rmax, ptr = [], [], []
    tol2 = 1e-8
    for (n, rm) in sizes:
        # Hermitian PSD with geometrically decaying spectrum
        Qm, _ = np.linalg.qr(crandn(rng, n, n))
        lam = 10.0 ** (-12 * np.arange(n) / n)
        K = (Qm * lam) @ Qm.conj().T
        K = (K + K.conj().T) / 2
        tK = to_dev(K, 0)
        tL = torch.zeros((rm, n), dtype=torch.complex128, device=DEV)
        keep += [tK, tL]
        data.append((K, tK, tL, n, rm))
        w.append(n)
        rmax.append(rm)
        ptr += [tK.data_ptr(), tL.data_ptr()]
    a1, p1 = i32(w)
    a2, p2 = i32(rmax)
    a3, p3 = i64(ptr)
    ranks = np.zeros(len(sizes), np.int32)
    piv = np.zeros(sum(rmax), np.int32)
    st = lib.nudft2_test_pchol(len(sizes), p1, p2, p3, tol2,
                               ranks.ctypes.data_as(C.POINTER(C.c_int32)),
                               piv.ctypes.data_as(C.POINTER(C.c_int32)))
    assert st == 0, lib.nudft2_last_error()
    off = 0
    for (K, tK, tL, n, rm), r in zip(data, ranks):
        L = from_dev(tL, n, rm)[:, :r]
        p = piv[off:off + r]
        off += rm
        S = K - L @ L.conj().T
        tr = np.trace(K).real
        print(f"pchol n={n}: rank {r}, residual trace {np.trace(S).real / tr:.2e}")
        assert len(set(p.tolist())) == r
        if r < rm:
            assert np.trace(S).real <= tol2 * tr * (1 + 1e-6) + 1e-13 * tr
            assert np.trace(S).real >= -1e-10 * tr
        # L restricted to the pivot rows is lower triangular in pivot order
        Lp = L[p, :]
        assert np.abs(np.triu(Lp, 1)).max() < 1e-12 * np.abs(Lp).max()
        # the rank is not far from the trace-optimal rank of the spectrum
        lam = np.sort(np.linalg.eigvalsh(K))[::-1]
        tail = np.concatenate([np.cumsum(lam[::-1])[::-1], [0.0]])
        ropt = int(np.nonzero(tail <= tol2 * tr)[0][0])
        if r < rm:
            assert r <= 2 * ropt + 8


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("ct", [0, 1])
def test_trsv(prec, ct):
    rng = np.random.default_rng(11 + ct)
    # one block (<= 128) with the lane-slot boundaries 64 / 65 / 128, and blocked orders
    sizes = [(1, 1), (50, 3), (300, 2), (7, 1), (700, 2), (257, 1), (64, 1), (65, 2), (128, 1),
             (129, 3)]
    keep, data, dims, ld, ptr = [], [], [], [], []
    for (k, nr) in sizes:
        # well-conditioned triangle (a unit-scale random triangle is
        # exponentially ill-conditioned in k)
        R = np.triu(crandn(rng, k, k), 1) / np.sqrt(k) + (2 + np.abs(crandn(rng, k))) * np.eye(k)
        B = crandn(rng, k, nr)
        tR, tB = to_dev(R, prec), to_dev(B, prec)
        keep += [tR, tB]
        data.append((R, B, tB, k, nr))
        dims += [k, nr]
        ld += [k, k]
        ptr += [tR.data_ptr(), tB.data_ptr()]
    a1, p1 = i32(dims)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    assert lib.nudft2_test_trsv(prec, len(sizes), p1, p2, p3, ct) == 0
    for R, B, tB, k, nr in data:
        X = from_dev(tB, k, nr)
        ref = np.linalg.solve(R.conj().T if ct else R, B)
        assert np.abs(X - ref).max() < 100 * TOL[prec] * max(1, np.abs(ref).max())


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("opa,opb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_large_batch(prec, opa, opb):
    """A batch of 24 products of a few hundred rows and columns (many tiles,
    no k splitting): ragged m, n, k (not multiples of the tile or k stage), a
    tiny product and an empty one in the same batch, beta = 1."""
    rng = np.random.default_rng(40 + 10 * prec + 2 * opa + opb)
    shapes = [(600 - 7 * i, 520 + 5 * i, 200 + 13 * i) for i in range(24)]
    shapes += [(3, 2, 5), (0, 4, 4), (130, 129, 1 if prec != 2 else 3)]
    mats, keep = [], []
    mnk, ld, ptr = [], [], []
    alpha = 0.9 + 0.2j
    for (m, n, k) in shapes:
        A = crandn(rng, *((m, k) if opa == 0 else (k, m)))
        B = crandn(rng, *((k, n) if opb == 0 else (n, k)))
        Cm = crandn(rng, m, n)
        ta, tb, tc = to_dev(A, prec), to_dev(B, prec), to_dev(Cm, prec)
        keep += [ta, tb, tc]
        mats.append((A, B, Cm, tc))
        mnk += [m, n, k]
        ld += [max(A.shape[0], 1), max(B.shape[0], 1), max(m, 1)]
        ptr += [ta.data_ptr(), tb.data_ptr(), tc.data_ptr()]
    a1, p1 = i32(mnk)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    st = lib.nudft2_test_gemm(prec, opa, opb, len(shapes), p1, p2, p3, alpha.real, alpha.imag, 1.0)
    assert st == 0, lib.nudft2_last_error()
    for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
        if m == 0:
            continue
        oA = A if opa == 0 else A.conj().T
        oB = B if opb == 0 else B.conj().T
        ref = alpha * (oA @ oB) + Cm
        got = from_dev(tc, m, n)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() < TOL[prec] * scale * max(1, k) ** 0.5 * 10, (m, n, k)


@pytest.mark.parametrize("opa,opb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_forced_unsplit(opa, opb):
    """The tile kernel forced unsplit through the measurement hook: ragged m,
    n, k around the tile and k-stage sizes, a one-row and an empty product in
    the same batch, alpha complex, beta = 1."""
    rng = np.random.default_rng(60 + 2 * opa + opb)
    shapes = [(1100, 1030, 130), (129, 300, 17), (256, 128, 16), (1, 200, 33), (0, 5, 5),
              (385, 511, 1)]
    mats, keep = [], []
    mnk, ld, ptr = [], [], []
    alpha = 0.6 - 0.8j
    for (m, n, k) in shapes:
        A = crandn(rng, *((m, k) if opa == 0 else (k, m)))
        B = crandn(rng, *((k, n) if opb == 0 else (n, k)))
        Cm = crandn(rng, m, n)
        ta, tb, tc = to_dev(A, 1), to_dev(B, 1), to_dev(Cm, 1)
        keep += [ta, tb, tc]
        mats.append((A, B, Cm, tc))
        mnk += [m, n, k]
        ld += [max(A.shape[0], 1), max(B.shape[0], 1), max(m, 1)]
        ptr += [ta.data_ptr(), tb.data_ptr(), tc.data_ptr()]
    a1, p1 = i32(mnk)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    ms = C.c_float(0)
    st = lib.nudft2_test_gemm_cfg(1, opa, opb, len(shapes), p1, p2, p3, alpha.real, alpha.imag,
                                  1.0, -1, C.byref(ms))
    assert st == 0, lib.nudft2_last_error()
    for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
        if m == 0:
            continue
        oA = A if opa == 0 else A.conj().T
        oB = B if opb == 0 else B.conj().T
        ref = alpha * (oA @ oB) + Cm
        got = from_dev(tc, m, n)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() < TOL[1] * scale * max(1, k) ** 0.5 * 10, (m, n, k)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("beta", [0.0, 1.0, -0.5])
def test_gemm_small_output_long_k(prec, beta):
    """A^H B with at most 32 x 32 outputs and a long k (the small-output
    path): Grams whose two operands are one matrix (same pointer), cross
    products, outputs that are not multiples of 16, k not a multiple of the
    per-workgroup slice, and an empty k in the same batch.  Bound: a
    forward error of 8 u sqrt(k) |a_i| |b_j| per entry."""
    rng = np.random.default_rng(80 + 3 * prec + int(2 * beta))
    npt, _ = CT[prec]
    u = np.finfo(npt).eps / 2
    # (m, n, k, same operand)
    shapes = [(16, 16, 100003, True), (15, 15, 50000, True), (20, 31, 9000, False),
              (32, 32, 8193, False), (5, 12, 20000, False), (30, 9, 12000, False),
              (16, 16, 0, False), (27, 27, 16500, True)]
    mats, keep = [], []
    mnk, ld, ptr = [], [], []
    alpha = 0.8 - 0.45j
    for (m, n, k, same) in shapes:
        A = crandn(rng, k, m)
        B = A if same else crandn(rng, k, n)
        Cm = crandn(rng, m, n)
        ta, tc = to_dev(A, prec), to_dev(Cm, prec)
        tb = ta if same else to_dev(B, prec)
        keep += [ta, tb, tc]
        mats.append((A, B, Cm, tc))
        mnk += [m, n, k]
        ld += [max(k, 1), max(k, 1), m]
        ptr += [ta.data_ptr(), tb.data_ptr(), tc.data_ptr()]
    a1, p1 = i32(mnk)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    st = lib.nudft2_test_gemm(prec, 1, 0, len(shapes), p1, p2, p3, alpha.real, alpha.imag, beta)
    assert st == 0, lib.nudft2_last_error()
    for (m, n, k, same), (A, B, Cm, tc) in zip(shapes, mats):
        Ac, Bc = A.astype(npt).astype(np.complex128), B.astype(npt).astype(np.complex128)
        Cc = Cm.astype(npt).astype(np.complex128)
        ref = alpha * (Ac.conj().T @ Bc) + beta * Cc
        got = from_dev(tc, m, n)
        na = np.linalg.norm(Ac, axis=0)
        nb_ = np.linalg.norm(Bc, axis=0)
        bound = 8 * u * max(1, k) ** 0.5 * np.outer(na, nb_) + 8 * u * np.abs(beta * Cc) + 1e-300
        assert np.all(np.abs(got - ref) <= bound + 4 * u * np.abs(ref)), (m, n, k, same)


@pytest.mark.parametrize("prec,shapes", [
    (0, [(40000, 40), (20000, 70), (9000, 33), (600, 20)]),
    (1, [(40000, 40), (20000, 70), (9000, 33), (600, 20)]),
    (2, [(40000, 40), (20000, 70), (9000, 33), (600, 20)]),
    # taller than one row slab per CU holds (65536 FP64 / 131072 FP32 rows):
    # twice the rows per workgroup
    (0, [(90000, 36), (3000, 40)]),
    (1, [(140000, 36), (3000, 40)]),
])
def test_geqrf_tall_panels(prec, shapes):
    """Householder QR of tall panels that need many cooperating workgroups per
    panel (40000 rows: 79 FP32 / 157 FP64 workgroups exchanging column sums
    every column; up to 140000 rows with twice the rows per workgroup),
    batched with shorter ones.  Checks Q [R; 0] = A through the Q application,
    R upper triangular, and |diag R| against LAPACK."""
    rng = np.random.default_rng(90 + prec)
    keep, data = [], []
    mn, ld, ptr = [], [], []
    for (m, n) in shapes:
        A = crandn(rng, m, n)
        k = min(m, n)
        nob = (k + QB - 1) // QB
        tsize = QB * QB * (nob - 1) + (k - QB * (nob - 1)) ** 2
        tA = to_dev(A, prec)
        tR = torch.full((n, k), 7.0 - 3.0j, dtype=CT[prec][1], device=DEV)
        tT = torch.full((tsize,), 5.0 + 1.0j, dtype=CT[prec][1], device=DEV)
        keep += [tA, tR, tT]
        data.append((A, tA, tR, tT))
        mn += [m, n]
        ld += [m, k]
        ptr += [tA.data_ptr(), tR.data_ptr(), tT.data_ptr()]
    a1, p1 = i32(mn)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    st = lib.nudft2_test_geqrf(prec, len(shapes), p1, p2, p3)
    assert st == 0, lib.nudft2_last_error()
    # C = [R; 0], then C <- Q C must reproduce A
    dims, ld2, ptr2, Cs = [], [], [], []
    for (m, n), (A, tA, tR, tT) in zip(shapes, data):
        k = min(m, n)
        R = from_dev(tR, k, n)
        assert np.abs(np.tril(R, -1)).max() == 0
        Cm = np.zeros((m, n), dtype=np.complex128)
        Cm[:k] = R
        tC = to_dev(Cm, prec)
        keep.append(tC)
        Cs.append(tC)
        dims += [m, k, n]
        ld2 += [m, m]
        ptr2 += [tA.data_ptr(), tT.data_ptr(), tC.data_ptr()]
        Rl = np.linalg.qr(A, mode="r")
        assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rl)), rtol=1e-3 if prec else 1e-9)
    b1, q1 = i32(dims)
    b2, q2 = i32(ld2)
    b3, q3 = i64(ptr2)
    assert lib.nudft2_test_ormqr(prec, 0, len(shapes), q1, q2, q3) == 0
    for (m, n), (A, tA, tR, tT), tC in zip(shapes, data, Cs):
        err = np.abs(from_dev(tC, m, n) - A).max() / np.abs(A).max()
        print(f"tall qr {m}x{n} prec{prec}: recon {err:.1e}")
        assert err < 50 * TOL[prec] * np.sqrt(m)


@pytest.mark.parametrize("opa,opb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_gemm_split_k_few_tiles(opa, opb, beta):
    """FP32 products with a long k and few output tiles (the k loop split
    over workgroups, atomic accumulation into a pre-scaled C): ragged m, n,
    k around the tile, k stage and split sizes, beta 0 and 1."""
    rng = np.random.default_rng(100 + 4 * opa + 2 * opb + int(beta))
    shapes = [(300, 200, 5000), (129, 77, 3001), (128, 64, 700), (255, 130, 1029)]
    mats, keep = [], []
    mnk, ld, ptr = [], [], []
    alpha = -0.3 + 0.95j
    for (m, n, k) in shapes:
        A = crandn(rng, *((m, k) if opa == 0 else (k, m)))
        B = crandn(rng, *((k, n) if opb == 0 else (n, k)))
        Cm = crandn(rng, m, n)
        ta, tb, tc = to_dev(A, 1), to_dev(B, 1), to_dev(Cm, 1)
        keep += [ta, tb, tc]
        mats.append((A, B, Cm, tc))
        mnk += [m, n, k]
        ld += [A.shape[0], B.shape[0], m]
        ptr += [ta.data_ptr(), tb.data_ptr(), tc.data_ptr()]
    a1, p1 = i32(mnk)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    st = lib.nudft2_test_gemm(1, opa, opb, len(shapes), p1, p2, p3, alpha.real, alpha.imag, beta)
    assert st == 0, lib.nudft2_last_error()
    for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
        oA = A if opa == 0 else A.conj().T
        oB = B if opb == 0 else B.conj().T
        ref = alpha * (oA @ oB) + beta * Cm
        got = from_dev(tc, m, n)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() < TOL[1] * scale * k ** 0.5 * 10, (m, n, k)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("opa,opb", [(0, 0), (1, 0)])
def test_gemm_long_descriptor_list(prec, opa, opb):
    """100 ragged products in one launch: a descriptor list longer than fits in
    the kernel arguments (read from device memory), with a skinny and a
    small-output batch of the same length (beta = 1, alpha complex)."""
    rng = np.random.default_rng(120 + 10 * prec + 2 * opa + opb)
    batches = [[(int(rng.integers(1, 200)), int(rng.integers(9, 150)), int(rng.integers(0, 300)))
                for _ in range(100)],
               [(int(rng.integers(1, 400)), int(rng.integers(1, 9)), int(rng.integers(1, 500)))
                for _ in range(100)]]
    if opa == 1:
        batches.append([(int(rng.integers(9, 33)), int(rng.integers(9, 33)),
                         int(rng.integers(8200, 9000))) for _ in range(100)])
    alpha = 0.25 + 0.7j
    for shapes in batches:
        mats, keep = [], []
        mnk, ld, ptr = [], [], []
        for (m, n, k) in shapes:
            A = crandn(rng, *((m, k) if opa == 0 else (k, m)))
            B = crandn(rng, *((k, n) if opb == 0 else (n, k)))
            Cm = crandn(rng, m, n)
            ta, tb, tc = to_dev(A, prec), to_dev(B, prec), to_dev(Cm, prec)
            keep += [ta, tb, tc]
            mats.append((A, B, Cm, tc))
            mnk += [m, n, k]
            ld += [max(A.shape[0], 1), max(B.shape[0], 1), m]
            ptr += [ta.data_ptr(), tb.data_ptr(), tc.data_ptr()]
        a1, p1 = i32(mnk)
        a2, p2 = i32(ld)
        a3, p3 = i64(ptr)
        st = lib.nudft2_test_gemm(prec, opa, opb, len(shapes), p1, p2, p3, alpha.real, alpha.imag,
                                  1.0)
        assert st == 0, lib.nudft2_last_error()
        for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
            oA = A if opa == 0 else A.conj().T
            oB = B if opb == 0 else B.conj().T
            ref = alpha * (oA @ oB) + Cm
            got = from_dev(tc, m, n)
            scale = max(1.0, np.abs(ref).max())
            assert np.abs(got - ref).max() < TOL[prec] * scale * max(1, k) ** 0.5 * 10, (m, n, k)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_gemm_small_m_wide_long_k(prec, beta):
    """A^H B with m <= 32, 32 < n <= 128 and a long k (a panel's reflectors
    against the columns they update): each wave of the kernel owns 32 output
    columns.  Ragged m, n (one wave partly or not at all used), k not a
    multiple of the per-workgroup range, an empty k in the batch."""
    rng = np.random.default_rng(140 + 3 * prec + int(2 * beta))
    npt, _ = CT[prec]
    u = np.finfo(npt).eps / 2
    shapes = [(32, 96, 9000), (20, 128, 5000), (32, 33, 4100), (5, 100, 6000), (32, 64, 4096),
              (17, 40, 0), (1, 127, 4500)]
    mats, keep = [], []
    mnk, ld, ptr = [], [], []
    alpha = -0.6 + 0.55j
    for (m, n, k) in shapes:
        A = crandn(rng, k, m)
        B = crandn(rng, k, n)
        Cm = crandn(rng, m, n)
        ta, tb, tc = to_dev(A, prec), to_dev(B, prec), to_dev(Cm, prec)
        keep += [ta, tb, tc]
        mats.append((A, B, Cm, tc))
        mnk += [m, n, k]
        ld += [max(k, 1), max(k, 1), m]
        ptr += [ta.data_ptr(), tb.data_ptr(), tc.data_ptr()]
    a1, p1 = i32(mnk)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    st = lib.nudft2_test_gemm(prec, 1, 0, len(shapes), p1, p2, p3, alpha.real, alpha.imag, beta)
    assert st == 0, lib.nudft2_last_error()
    for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
        Ac, Bc = A.astype(npt).astype(np.complex128), B.astype(npt).astype(np.complex128)
        Cc = Cm.astype(npt).astype(np.complex128)
        ref = alpha * (Ac.conj().T @ Bc) + beta * Cc
        got = from_dev(tc, m, n)
        na = np.linalg.norm(Ac, axis=0)
        nb_ = np.linalg.norm(Bc, axis=0)
        bound = 8 * u * max(1, k) ** 0.5 * np.outer(na, nb_) + 8 * u * np.abs(beta * Cc) + 1e-300
        assert np.all(np.abs(got - ref) <= bound + 4 * u * np.abs(ref)), (m, n, k)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("opa,opb", [(0, 0), (1, 0), (0, 1)])
def test_gemm_few_row_tiles(prec, opa, opb):
    """Products with at most 256 rows and many column tiles (the shape of the
    V^H C products of the blocked QR): ragged m around the 64-row tiles, n not
    a multiple of 64, one launch with the k loop split and one without,
    beta = 1, alpha complex."""
    rng = np.random.default_rng(160 + 10 * prec + 2 * opa + opb)
    alpha = 0.45 - 0.85j
    for shapes in ([(256, 2000, 700), (200, 1500, 300), (129, 2100, 64), (64, 4096, 33)],
                   [(250, 3000, 150)] * 6):
        mats, keep = [], []
        mnk, ld, ptr = [], [], []
        for (m, n, k) in shapes:
            A = crandn(rng, *((m, k) if opa == 0 else (k, m)))
            B = crandn(rng, *((k, n) if opb == 0 else (n, k)))
            Cm = crandn(rng, m, n)
            ta, tb, tc = to_dev(A, prec), to_dev(B, prec), to_dev(Cm, prec)
            keep += [ta, tb, tc]
            mats.append((A, B, Cm, tc))
            mnk += [m, n, k]
            ld += [A.shape[0], B.shape[0], m]
            ptr += [ta.data_ptr(), tb.data_ptr(), tc.data_ptr()]
        a1, p1 = i32(mnk)
        a2, p2 = i32(ld)
        a3, p3 = i64(ptr)
        st = lib.nudft2_test_gemm(prec, opa, opb, len(shapes), p1, p2, p3, alpha.real, alpha.imag,
                                  1.0)
        assert st == 0, lib.nudft2_last_error()
        for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
            oA = A if opa == 0 else A.conj().T
            oB = B if opb == 0 else B.conj().T
            ref = alpha * (oA @ oB) + Cm
            got = from_dev(tc, m, n)
            scale = max(1.0, np.abs(ref).max())
            assert np.abs(got - ref).max() < TOL[prec] * scale * k ** 0.5 * 10, (m, n, k)


@pytest.mark.parametrize("pd,ps", [(0, 0), (1, 1), (1, 0), (0, 1)])
def test_copy_conj_transpose(pd, ps):
    """Batched copies with precision change, plain and conjugate-transposed in
    one batch: ragged shapes that span several 32 x 32 tiles, one-row and
    one-column blocks, an empty one, padded leading dimensions on both sides.
    Bit-exact (a copy, conjugation and round-to-nearest conversion); the
    padding rows of every destination keep their sentinel."""
    rng = np.random.default_rng(70 + 2 * pd + ps)
    npd, _ = CT[pd]
    nps, _ = CT[ps]
    shapes = [(1000, 700, 1), (700, 1000, 0), (33, 31, 1), (1, 257, 1), (257, 1, 1), (0, 5, 1),
              (64, 64, 0), (95, 130, 1), (5, 3, 0), (2048, 40, 1)]
    keep, cases, dims, ld, ptr, ctl = [], [], [], [], [], []
    for (m, n, ct) in shapes:
        S = crandn(rng, m, n).astype(nps)
        lds = m + 3
        Sp = np.zeros((lds, max(n, 1)), dtype=nps)
        Sp[:m, :n] = S
        dm, dn = (n, m) if ct else (m, n)
        ldd = dm + 5
        Dp = np.full((ldd, max(dn, 1)), 7.0 - 3.0j, dtype=npd)
        tS = torch.from_numpy(np.ascontiguousarray(Sp.T)).to(DEV)
        tD = torch.from_numpy(np.ascontiguousarray(Dp.T)).to(DEV)
        keep += [tS, tD]
        ref = Dp.copy()
        ref[:dm, :dn] = (S.conj().T if ct else S).astype(npd)
        cases.append((tD, ref, ldd, max(dn, 1)))
        dims += [m, n]
        ld += [lds, ldd]
        ptr += [tS.data_ptr(), tD.data_ptr()]
        ctl.append(ct)
    a1, p1 = i32(dims)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    a4, p4 = i32(ctl)
    assert lib.nudft2_test_copy(pd, ps, len(shapes), p1, p2, p3, p4) == 0
    for tD, ref, ldd, dn in cases:
        got = tD.cpu().numpy().reshape(dn, ldd).T
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("opa,opb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_stream_k(prec, opa, opb):
    """Stream-K shares forced on a ragged batch: each descriptor's tiles x k
    stages dealt out in equal pieces that start and end inside tiles, added
    atomically to a pre-scaled C.  Shapes around the tile (64) and k stage
    (16), one with k = 1 stage, an empty k and an empty output in the same
    launch; beta = 0.5, alpha complex.  Also a single long product (the QR
    V^H C shape class at reduced size)."""
    rng = np.random.default_rng(140 + 8 * prec + 2 * opa + opb)
    batches = [[(300, 200, 5000), (129, 77, 3001), (64, 64, 16), (65, 63, 17), (200, 100, 0),
                (0, 40, 100), (1, 1, 999)],
               [(256, 1500, 3000)]]
    alpha, beta = 0.7 - 0.4j, 0.5
    for shapes in batches:
        mats, keep, mnk, ld, ptr = [], [], [], [], []
        for (m, n, k) in shapes:
            A = crandn(rng, *((m, k) if opa == 0 else (k, m)))
            B = crandn(rng, *((k, n) if opb == 0 else (n, k)))
            Cm = crandn(rng, m, n)
            ta, tb, tc = (to_dev(A, prec) if A.size else torch.zeros(1, dtype=CT[prec][1], device=DEV),
                          to_dev(B, prec) if B.size else torch.zeros(1, dtype=CT[prec][1], device=DEV),
                          to_dev(Cm, prec) if Cm.size else torch.zeros(1, dtype=CT[prec][1], device=DEV))
            keep += [ta, tb, tc]
            mats.append((A, B, Cm, tc))
            mnk += [m, n, k]
            ld += [max(1, A.shape[0]), max(1, B.shape[0]), max(1, m)]
            ptr += [ta.data_ptr(), tb.data_ptr(), tc.data_ptr()]
        a1, p1 = i32(mnk)
        a2, p2 = i32(ld)
        a3, p3 = i64(ptr)
        st = lib.nudft2_test_gemm_cfg(prec, opa, opb, len(shapes), p1, p2, p3, alpha.real,
                                      alpha.imag, beta, -3, None)
        assert st == 0, lib.nudft2_last_error()
        for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
            if m == 0 or n == 0:
                continue
            oA = A if opa == 0 else A.conj().T
            oB = B if opb == 0 else B.conj().T
            ref = alpha * (oA @ oB) + beta * Cm
            got = from_dev(tc, m, n)
            scale = max(1.0, np.abs(ref).max())
            assert np.abs(got - ref).max() < TOL[prec] * scale * max(k, 1) ** 0.5 * 10, (m, n, k)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("opa,opb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_partial_tile_splits(prec, opa, opb):
    """k splits kept as partial tiles in scratch and summed in split order by a
    second kernel (forced, splits = -4): ragged outputs of one to a few tiles,
    k long and short (splits past k hold nothing), k = 0 and an empty output
    in the same launch, beta = 0.5 and 0, alpha complex.  Then the library's
    own choice on a batch of tall-panel Gram shapes (128 x 128, k = 9000),
    which takes this path."""
    rng = np.random.default_rng(160 + 8 * prec + 2 * opa + opb)
    alpha = -0.6 + 0.3j
    runs = [([(128, 128, 5000), (65, 127, 4099), (1, 64, 700), (64, 1, 33), (100, 90, 0),
              (0, 30, 200), (130, 70, 17)], -4, 0.5),
            ([(128, 128, 9000)] * 4 + [(128, 96, 8191)], 0, 0.0)]
    for shapes, sp, beta in runs:
        mats, keep, mnk, ld, ptr = [], [], [], [], []
        for (m, n, k) in shapes:
            A = crandn(rng, *((m, k) if opa == 0 else (k, m)))
            B = crandn(rng, *((k, n) if opb == 0 else (n, k)))
            Cm = crandn(rng, m, n)
            ts = [to_dev(X, prec) if X.size else torch.zeros(1, dtype=CT[prec][1], device=DEV)
                  for X in (A, B, Cm)]
            keep += ts
            mats.append((A, B, Cm, ts[2]))
            mnk += [m, n, k]
            ld += [max(1, A.shape[0]), max(1, B.shape[0]), max(1, m)]
            ptr += [t.data_ptr() for t in ts]
        a1, p1 = i32(mnk)
        a2, p2 = i32(ld)
        a3, p3 = i64(ptr)
        st = lib.nudft2_test_gemm_cfg(prec, opa, opb, len(shapes), p1, p2, p3, alpha.real,
                                      alpha.imag, beta, sp, None)
        assert st == 0, lib.nudft2_last_error()
        for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
            if m == 0 or n == 0:
                continue
            oA = A if opa == 0 else A.conj().T
            oB = B if opb == 0 else B.conj().T
            ref = alpha * (oA @ oB) + beta * Cm
            got = from_dev(tc, m, n)
            scale = max(1.0, np.abs(ref).max())
            assert np.abs(got - ref).max() < TOL[prec] * scale * max(k, 1) ** 0.5 * 10, (m, n, k)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("code", [-5, -6])
def test_gemm_forced_small_tiles(prec, code):
    """The small-output tile shapes the autotuner can pick for A^H B with
    m <= 32 (-5: 32 x 128 tiles, -6: 16- or 32-square tiles), forced on ragged
    batches with short and long k, k = 0 and an empty output in the same
    launch, beta = 0.5, alpha complex; shapes the tiles do not cover are
    rejected with E_INVAL and leave C untouched."""
    rng = np.random.default_rng(180 + 4 * prec - code)
    nmax = 128 if code == -5 else 32
    shapes = [(32, nmax, 5000), (17, nmax - 3, 333), (1, 9, 70), (32, 12, 1), (20, 20, 0),
              (0, 16, 100)]
    alpha, beta = 0.4 + 0.9j, 0.5
    mats, keep, mnk, ld, ptr = [], [], [], [], []
    for (m, n, k) in shapes:
        A = crandn(rng, k, m)
        B = crandn(rng, k, n)
        Cm = crandn(rng, m, n)
        ts = [to_dev(X, prec) if X.size else torch.zeros(1, dtype=CT[prec][1], device=DEV)
              for X in (A, B, Cm)]
        keep += ts
        mats.append((A, B, Cm, ts[2]))
        mnk += [m, n, k]
        ld += [max(1, k), max(1, k), max(1, m)]
        ptr += [t.data_ptr() for t in ts]
    a1, p1 = i32(mnk)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    st = lib.nudft2_test_gemm_cfg(prec, 1, 0, len(shapes), p1, p2, p3, alpha.real, alpha.imag,
                                  beta, code, None)
    assert st == 0, lib.nudft2_last_error()
    for (m, n, k), (A, B, Cm, tc) in zip(shapes, mats):
        if m == 0 or n == 0:
            continue
        ref = alpha * (A.conj().T @ B) + beta * Cm
        got = from_dev(tc, m, n)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() < TOL[prec] * scale * max(k, 1) ** 0.5 * 10, (m, n, k)
    # out of range: m > 32, n above the tile, op(A) = N
    for (m, n, k, opa) in [(33, 16, 100, 1), (16, nmax + 1, 100, 1), (16, 16, 100, 0)]:
        A = crandn(rng, *((k, m) if opa else (m, k)))
        B = crandn(rng, k, n)
        Cm = crandn(rng, m, n)
        ta, tb, tc = to_dev(A, prec), to_dev(B, prec), to_dev(Cm, prec)
        b1, q1 = i32([m, n, k])
        b2, q2 = i32([A.shape[0], k, m])
        b3, q3 = i64([ta.data_ptr(), tb.data_ptr(), tc.data_ptr()])
        st = lib.nudft2_test_gemm_cfg(prec, opa, 0, 1, q1, q2, q3, 1.0, 0.0, 0.0, code, None)
        assert st == 1 and b"forced small tile" in lib.nudft2_last_error()
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(tc, m, n), Cm.astype(CT[prec][0]))


@pytest.mark.parametrize("prec", [0, 1])
def test_trtri_inverts_upper_triangles(prec):
    """Batched in-place inversion of upper-triangular matrices (the solves'
    stored D11^{-1} and root R^{-1}) against LAPACK's inverse, for orders
    around the 128-row diagonal blocks and the doubling joins."""
    rng = np.random.default_rng(77 + prec)
    ks = [1, 5, 128, 129, 300, 1000, 1537]
    keep, ref, kk, ld, ptr = [], [], [], [], []
    for k in ks:
        R = np.triu(crandn(rng, k, k)) / np.sqrt(k)
        R[np.diag_indices(k)] = 1.0 + 0.5 * rng.random(k) * np.exp(2j * np.pi * rng.random(k))
        t = to_dev(R, prec)
        keep.append(t)
        ref.append(np.linalg.inv(R))
        kk.append(k)
        ld.append(k)
        ptr.append(t.data_ptr())
    a1, p1 = i32(kk)
    a2, p2 = i32(ld)
    a3, p3 = i64(ptr)
    assert lib.nudft2_test_trtri(prec, len(ks), p1, p2, p3) == 0, lib.nudft2_last_error()
    for k, t, X in zip(ks, keep, ref):
        got = from_dev(t, k, k)
        err = np.linalg.norm(got - X) / np.linalg.norm(X)
        print(f"trtri k={k} prec{prec}: {err:.1e}")
        assert np.abs(np.tril(got, -1)).max() == 0
        assert err < (1e-13 if prec == 0 else 2e-5) * max(1.0, np.log2(k))
