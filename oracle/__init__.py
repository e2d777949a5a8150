"""CPU FP64 oracle for the 2D type-II inverse NUDFT (test infrastructure).

This package is the reference that the GPU library is checked against.  It is
plain, slow NumPy/SciPy code written from the paper (Li & Liu, "A superfast
direct solver for the 2D type-II inverse NUDFT based on HSS matrices"):

* ``nudft``  -- the transform itself (Section 1, eq. for the 2D type-II NUDFT
  and its matrix), its adjoint, the dense least-squares solution, and the
  transformed matrix G = A F^{-1} with its closed-form kernel (Section 2.5,
  Cauchy-like entries; Section 3.1, separable 2D kernel).
* ``hss``    -- a small dense-friendly reference of the HSS machinery: HSS
  expansion, 1D HSS by truncated SVD, the face-splitting product generators
  (Theorem 3.3), recompression (Section 2.3) and the URV least-squares solver
  (Section 2.4 / URV section).  Used for tiny problems only.
* ``fadi``   -- factored ADI (fADI) low-rank factors of the 1D HSS row blocks
  from the displacement equation of Section 2.5, with Zolotarev shifts on the
  two arcs of the unit circle, and a 1D HSS whose leaf row bases use them.
* ``grad``   -- derivatives of the least-squares solution with respect to the
  right-hand side and the sample points (chain rule on the normal equations).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never calls it, and it shares no
code with the GPU library; both read their inputs from ``nudft_inputs``.

Conventions fixed here (and restated where used):
* public frequencies are centred, k in [-n/2, n/2) per axis; coefficient
  arrays are C-order (nx, ny) with c[i, j] <-> (k^x, k^y) = (i - nx/2, j - ny/2);
* the paper's matrix uses k in [0, n); the two differ by the row phase
  phi_j = exp(+i pi (nx x_j + ny y_j)):  A_centred = diag(phi) A_paper;
* the column (k^x, k^y) of a vectorised coefficient array is k^y + k^x n^y
  (kx-major), i.e. numpy C-order ``reshape(-1)``.
"""
