"""The 2D type-II NUDFT, its adjoint and its least-squares inverse (FP64).

Oracle (test infrastructure only).  Every function follows a definition of the
paper:

* apply / apply_adj / dense_matrix: Section 1, the 2D type-II NUDFT sum and its
  matrix A(j, (k^x, k^y)) = exp(-2 pi i (k^x x_j + k^y y_j)), written here with
  centred frequencies (see the package docstring for the phase relation).
* lstsq: Section 1, the inverse problem min_c ||A c - f||_2, solved by a dense
  Householder QR (the O(M N^2) method the paper cites as the dense baseline).
* kernel_1d / dense_G: Section 2.5 (1D Cauchy-like matrix G = A F^{-1}, eq. for
  its entries) and Section 3.1 (separable 2D kernel, G = G^x face-split G^y),
  with the paper's 0-based frequencies.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

TWO_PI = 2.0 * np.pi


def centred_freqs(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.int64) - n // 2


def phase_turns(k: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(k * x) reduced mod 1 into [-1/2, 1/2), computed exactly.

    k is an integer array (|k| < 2^10), x a float64 array; the product is
    formed in extended precision (64-bit mantissa) where it is exact, so the
    only rounding is the final conversion to float64.  Returns outer(x, k)."""
    kl = np.asarray(k, dtype=np.longdouble)
    xl = np.asarray(x, dtype=np.longdouble)
    t = np.multiply.outer(xl, kl)
    t = t - np.rint(t)
    return t.astype(np.float64)


def expi_turns(t: np.ndarray) -> np.ndarray:
    """exp(-2 pi i t) for t in turns."""
    return np.exp(-1j * TWO_PI * t)


def nudft_1d(x: np.ndarray, n: int, centred: bool = True) -> np.ndarray:
    """A^x(j, k) = exp(-2 pi i k x_j), k centred or 0-based.  Shape (M, n)."""
    k = centred_freqs(n) if centred else np.arange(n, dtype=np.int64)
    return expi_turns(phase_turns(k, x))


def dense_matrix(points: np.ndarray, nx: int, ny: int,
                 centred: bool = True) -> np.ndarray:
    """A (M x N): row j is the Kronecker product of row j of A^x and A^y,
    columns ordered k^y + k^x n^y (Section 1)."""
    Ax = nudft_1d(points[:, 0], nx, centred)
    Ay = nudft_1d(points[:, 1], ny, centred)
    return (Ax[:, :, None] * Ay[:, None, :]).reshape(points.shape[0], nx * ny)


def apply(points: np.ndarray, c: np.ndarray, chunk: int = 8192) -> np.ndarray:
    """f_j = sum_{kx, ky} c[kx, ky] exp(-2 pi i (kx x_j + ky y_j)).

    The double sum is evaluated as an inner sum over k^y (a matrix product
    with the exponentials of y_j) and an outer sum over k^x, row chunk by row
    chunk.  c may be (nx, ny) or (nrhs, nx, ny)."""
    c = np.asarray(c, dtype=np.complex128)
    single = c.ndim == 2
    cc = c[None] if single else c
    nrhs, nx, ny = cc.shape
    M = points.shape[0]
    out = np.empty((nrhs, M), dtype=np.complex128)
    kx = centred_freqs(nx)
    ky = centred_freqs(ny)
    for s in range(0, M, chunk):
        e = min(M, s + chunk)
        Ex = expi_turns(phase_turns(kx, points[s:e, 0]))   # (m, nx)
        Ey = expi_turns(phase_turns(ky, points[s:e, 1]))   # (m, ny)
        for r in range(nrhs):
            inner = Ey @ cc[r].T                             # (m, nx): sum over ky
            out[r, s:e] = np.sum(Ex * inner, axis=1)         # sum over kx
    return out[0] if single else out


def apply_adj(points: np.ndarray, f: np.ndarray, nx: int, ny: int,
              chunk: int = 8192) -> np.ndarray:
    """(A^* f)[kx, ky] = sum_j f_j exp(+2 pi i (kx x_j + ky y_j))."""
    f = np.asarray(f, dtype=np.complex128)
    single = f.ndim == 1
    ff = f[None] if single else f
    nrhs, M = ff.shape
    out = np.zeros((nrhs, nx, ny), dtype=np.complex128)
    kx = centred_freqs(nx)
    ky = centred_freqs(ny)
    for s in range(0, M, chunk):
        e = min(M, s + chunk)
        Ex = expi_turns(phase_turns(kx, points[s:e, 0]))
        Ey = expi_turns(phase_turns(ky, points[s:e, 1]))
        for r in range(nrhs):
            out[r] += (Ex.conj() * ff[r, s:e, None]).T @ Ey.conj()
    return out[0] if single else out


def lstsq(points: np.ndarray, f: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """c* = argmin ||A c - f||_2 by dense Householder QR (economic) and a
    triangular solve.  Returns (nx, ny) (or (nrhs, nx, ny))."""
    A = dense_matrix(points, nx, ny)
    Q, R = sla.qr(A, mode="economic", check_finite=False)
    f = np.asarray(f, dtype=np.complex128)
    single = f.ndim == 1
    ff = f[None] if single else f
    out = np.empty((ff.shape[0], nx, ny), dtype=np.complex128)
    for r in range(ff.shape[0]):
        rhs = Q.conj().T @ ff[r]
        out[r] = sla.solve_triangular(R, rhs, check_finite=False).reshape(nx, ny)
    return out[0] if single else out


def residual(points, c, f) -> float:
    """||A c - f|| / ||f|| (relative residual, Section 5 metric r_s)."""
    return float(np.linalg.norm(apply(points, c) - f) / np.linalg.norm(f))


def rel_err(c, c_ref) -> float:
    """||c - c_ref|| / ||c_ref|| (relative error, Section 5 metric e_s)."""
    return float(np.linalg.norm(np.asarray(c) - c_ref) / np.linalg.norm(c_ref))


# --------------------------------------------------------------------------
# The transformed matrix G = A F^{-1} (paper convention, 0-based frequencies)
# --------------------------------------------------------------------------

def kernel_1d(x: np.ndarray, n: int, cols: np.ndarray | None = None) -> np.ndarray:
    """G^x(j, l) for G^x = A^x (F^x)^{-1}, F(k, l) = exp(-2 pi i k l / n).

    Entry: (1/n) sum_{k<n} exp(-2 pi i k theta), theta = x_j - l/n (mod 1),
    which is the Cauchy-like ratio of Section 2.5, ((g/xi)^n - 1)/(n((g/xi)-1))
    with g = exp(-2 pi i x_j), xi = exp(-2 pi i l/n), and equals 1 where
    g = xi.  It is evaluated in the Dirichlet form
        exp(-i pi (n-1) theta) sin(pi n theta) / (n sin(pi theta)),
    which avoids the cancellation of the ratio near g = xi."""
    if cols is None:
        cols = np.arange(n, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    xl = np.asarray(x, dtype=np.longdouble)
    theta = np.subtract.outer(xl, np.asarray(cols, dtype=np.longdouble) / n)
    theta = theta - np.rint(theta)            # reduce to [-1/2, 1/2]
    th = theta.astype(np.float64)
    out = np.empty(th.shape, dtype=np.complex128)
    small = np.abs(th) < 1e-300
    ths = np.where(small, 1.0, th)
    # n*theta reduced separately for the numerator's accuracy
    nt = (theta * n)
    nt_red = (nt - 2.0 * np.rint(nt / 2.0)).astype(np.float64)   # sin(pi n t) has period 2 in n t
    num = np.sin(np.pi * nt_red)
    den = n * np.sin(np.pi * ths)
    ratio = num / den
    ph_t = ((n - 1) * theta)
    ph_t = (ph_t - 2.0 * np.rint(ph_t / 2.0)).astype(np.float64)
    out[:] = np.exp(-1j * np.pi * ph_t) * ratio
    out[small] = 1.0
    return out


def dft_matrix(n: int) -> np.ndarray:
    """F(k, l) = exp(-2 pi i k l / n) (Section 2.5); the phase k l / n is
    reduced mod 1 in exact integer arithmetic."""
    k = np.arange(n, dtype=np.int64)
    kl = np.mod(np.multiply.outer(k, k), n).astype(np.float64) / n
    return expi_turns(kl)


def dense_G(points: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """G = G^x face-split G^y (Section 3.1), columns l^y + l^x n^y."""
    Gx = kernel_1d(points[:, 0], nx)
    Gy = kernel_1d(points[:, 1], ny)
    return (Gx[:, :, None] * Gy[:, None, :]).reshape(points.shape[0], nx * ny)


def centring_phase(points: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """phi_j = exp(+i pi (nx x_j + ny y_j)) so that A_centred = diag(phi) A_paper."""
    t = phase_turns(np.array([nx // 2]), points[:, 0])[:, 0] + \
        phase_turns(np.array([ny // 2]), points[:, 1])[:, 0]
    return np.exp(1j * TWO_PI * t)
