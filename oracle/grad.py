"""Derivatives of the least-squares inverse NUDFT (oracle, test infrastructure).

c(f, x, y) = argmin_c ||A(x, y) c - f||_2 with A of full column rank, so
c = (A^* A)^{-1} A^* f.  For a real loss L(c) with upstream gradient
g = dL/dc in the convention dL = Re(g^H dc) (PyTorch's convention for complex
tensors), differentiating the normal equations (A^*A) c = A^* f gives

    A^*A dc = dA^* r - A^* dA c,        r = f - A c,

and with z = (A^*A)^{-1} g, w = A z:

    dL/df   = w
    dL/dx_j = 2 pi Im( conj(r_j) t_j - conj(w_j) s_j ),  s = A(k^x o c),
                                                           t = A(k^x o z),
and the same with k^y for y_j, since dA(j, k)/dx_j = -2 pi i k^x A(j, k)
(k centred).  Dense A is used: small problems only.
"""
from __future__ import annotations

import numpy as np

from . import nudft


def lsq_grads(points, f, nx, ny, g):
    """Returns (c, dL/df, dL/dx, dL/dy) for upstream g = dL/dc (nx, ny)."""
    A = nudft.dense_matrix(points, nx, ny)
    AhA = A.conj().T @ A
    c = np.linalg.solve(AhA, A.conj().T @ f)
    z = np.linalg.solve(AhA, np.asarray(g, complex).reshape(-1))
    r = f - A @ c
    w = A @ z
    kx = np.repeat(nudft.centred_freqs(nx), ny).astype(np.float64)
    ky = np.tile(nudft.centred_freqs(ny), nx).astype(np.float64)
    out = []
    for k in (kx, ky):
        s = A @ (k * c)
        t = A @ (k * z)
        out.append(2.0 * np.pi * np.imag(np.conj(r) * t - np.conj(w) * s))
    return c.reshape(nx, ny), w, out[0], out[1]


def loss_target(points, f, nx, ny, c_target):
    """L = ||c(f, x, y) - c_target||^2 and its upstream gradient 2 (c - c_t)."""
    c = nudft.lstsq(points, f, nx, ny)
    d = c - c_target
    return float(np.vdot(d, d).real), 2.0 * d
