"""Reference HSS machinery for small problems (oracle, test infrastructure).

Plain NumPy, dense-friendly, written from the paper's definitions and stated
algorithms.  Every basis is kept explicitly so that expansions are easy to
form; this is only usable at tiny sizes.

* Trees (Definition 2.1 HSS tree; Definition 3.2 face-splitting product of HSS
  trees): 1D trees from dyadic bisection of [0, 1) with half-open intervals;
  the 2D tree is their product (quadrisection).  Node rows are the points in
  the node's interval/box; node columns are the frequencies l with l/n in the
  interval (Theorem 2.2's index sets).
* ``expand``: the matrix an HSS representation stands for (Definition 2.2).
* ``hss_1d``: a 1D HSS approximation of G^x with nested orthonormal bases by
  truncated SVDs of the HSS blocks.  The paper delegates its 1D construction
  to an fADI + interpolative-decomposition method of another work; any valid
  1D HSS approximation with the stated accuracy satisfies the hypothesis of
  Theorem 3.5, so the plainest one (truncated SVD) is used here.
* ``face_split``: the generators of H^x face-split H^y (Theorem 3.3 and its
  constructive proof, extended from the first child to all four children).
* ``recompress``: Section 2.3, stage 1 (bottom-up orthogonalisation) and stage
  2 (top-down truncated SVDs).
* ``urv_factor`` / ``urv_solve``: the URV least-squares solver (Section 2.4,
  "The URV factorization for HSS matrices"), with separate row and column
  ranks (the paper assumes equal ranks for brevity).
* ``direct_solve``: Algorithm 4.1 end to end for one right-hand side.

Truncation rule (the paper fixes only the rank definition, for any unitarily
invariant norm): keep the smallest r with sum_{i>r} s_i^2 <= tol^2 sum_i s_i^2,
i.e. relative Frobenius-norm error tol (the norm of Theorem 3.5).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from . import nudft


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------

def frob_rank(s: np.ndarray, tol: float) -> int:
    """Smallest r with sum_{i>=r} s_i^2 <= tol^2 sum s_i^2 (s descending)."""
    if s.size == 0:
        return 0
    tot = float(np.sum(s * s))
    if tot == 0.0:
        return 0
    tail = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])
    ok = np.nonzero(tail <= (tol * tol) * tot)[0]
    return int(ok[0])


def trunc_left(C: np.ndarray, tol: float):
    """Truncated SVD C ~ P diag(s) X^*: returns (P, s)."""
    if C.shape[0] == 0:
        return np.zeros((0, 0), complex), np.zeros(0)
    if C.shape[1] == 0:
        return np.zeros((C.shape[0], 0), complex), np.zeros(0)
    P, s, _ = np.linalg.svd(C, full_matrices=False)
    r = frob_rank(s, tol) if tol > 0 else int(np.sum(s > s[0] * 1e-14)) if s.size else 0
    return P[:, :r], s[:r]


def thin_qr(X: np.ndarray):
    """Economic QR, k = min(m, n) columns."""
    if X.shape[0] == 0 or X.shape[1] == 0:
        k = min(X.shape)
        return np.zeros((X.shape[0], k), complex), np.zeros((k, X.shape[1]), complex)
    Q, R = np.linalg.qr(X, mode="reduced")
    return Q, R


def face(A1: np.ndarray, A2: np.ndarray) -> np.ndarray:
    """Face-splitting product: row-wise Kronecker product (Section 2.1)."""
    m = A1.shape[0]
    return (A1[:, :, None] * A2[:, None, :]).reshape(m, A1.shape[1] * A2.shape[1])


# --------------------------------------------------------------------------
# trees
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Node:
    key: tuple
    level: int
    rows: np.ndarray        # global row (point) indices, increasing
    cols: np.ndarray        # global column indices, in the node's own order
    children: list
    parent: tuple | None = None


class Tree:
    def __init__(self, nodes: dict, root: tuple, L: int):
        self.nodes = nodes
        self.root = root
        self.L = L

    def level(self, l):
        return [k for k, v in self.nodes.items() if v.level == l]

    def leaves(self):
        return [k for k, v in self.nodes.items() if not v.children]

    def siblings(self, key):
        p = self.nodes[key].parent
        return [c for c in self.nodes[p].children if c != key]


def col_range(n: int, level: int, a: int) -> np.ndarray:
    """Columns l with floor(l 2^level / n) == a, i.e. l/n in [a/2^l,(a+1)/2^l)."""
    lo = -(-a * n // (1 << level))
    hi = -(-(a + 1) * n // (1 << level))
    return np.arange(lo, hi, dtype=np.int64)


def row_bins(x: np.ndarray, level: int) -> np.ndarray:
    b = np.floor(x * (1 << level)).astype(np.int64)
    return np.minimum(b, (1 << level) - 1)


def tree_1d(x: np.ndarray, n: int, L: int) -> Tree:
    nodes = {}
    for l in range(L + 1):
        bins = row_bins(x, l)
        for a in range(1 << l):
            rows = np.nonzero(bins == a)[0]
            ch = [(l + 1, 2 * a), (l + 1, 2 * a + 1)] if l < L else []
            par = (l - 1, a // 2) if l > 0 else None
            nodes[(l, a)] = Node((l, a), l, rows, col_range(n, l, a), ch, par)
    return Tree(nodes, (0, 0), L)


def tree_2d(points: np.ndarray, nx: int, ny: int, L: int) -> Tree:
    """Face-splitting product of the two 1D trees (Definition 3.2), both of
    depth L.  Node (l, a, b): rows = points in the box, columns K^x_a x K^y_b
    in kx-major order, global index ly + lx * ny; children (p, q) in
    lexicographic order."""
    nodes = {}
    for l in range(L + 1):
        bx = row_bins(points[:, 0], l)
        by = row_bins(points[:, 1], l)
        for a in range(1 << l):
            kx = col_range(nx, l, a)
            for b in range(1 << l):
                ky = col_range(ny, l, b)
                rows = np.nonzero((bx == a) & (by == b))[0]
                cols = (kx[:, None] * ny + ky[None, :]).reshape(-1)
                ch = [(l + 1, 2 * a + p, 2 * b + q) for p in (0, 1) for q in (0, 1)] \
                    if l < L else []
                par = (l - 1, a // 2, b // 2) if l > 0 else None
                nodes[(l, a, b)] = Node((l, a, b), l, rows, cols, ch, par)
    return Tree(nodes, (0, 0, 0), L)


def depth_for(nx: int, ny: int, leaf: int = 16) -> int:
    """Common depth of both 1D trees: ceil(log2(max(nx, ny)/leaf)), >= 0."""
    L = 0
    while max(nx, ny) > leaf * (1 << L):
        L += 1
    return L


# --------------------------------------------------------------------------
# HSS representation and expansion
# --------------------------------------------------------------------------

@dataclasses.dataclass
class HSS:
    tree: Tree
    D: dict      # leaf -> dense block (rows x cols in node order)
    U: dict      # leaf -> (|rows| x rU)
    V: dict      # leaf -> (|cols| x rV)
    R: dict      # non-root -> (rU_child x rU_parent)
    W: dict      # non-root -> (rV_child x rV_parent)
    B: dict      # (key, sibling key) -> (rU_key x rV_sib)


def full_bases(h: HSS):
    """Explicit U_tau (|J_tau| x r) and V_tau (|K_tau| x r) for every
    non-root node from the nested relations (Definition 2.2 (2))."""
    t = h.tree
    Uf, Vf = {}, {}
    for l in range(t.L, 0, -1):
        for k in t.level(l):
            nd = t.nodes[k]
            if not nd.children:
                Uf[k], Vf[k] = h.U[k], h.V[k]
                continue
            rpos = {g: i for i, g in enumerate(nd.rows)}
            cpos = {g: i for i, g in enumerate(nd.cols)}
            rU = h.R[nd.children[0]].shape[1]
            rV = h.W[nd.children[0]].shape[1]
            Uk = np.zeros((nd.rows.size, rU), complex)
            Vk = np.zeros((nd.cols.size, rV), complex)
            for c in nd.children:
                cn = t.nodes[c]
                Uk[[rpos[g] for g in cn.rows]] = Uf[c] @ h.R[c]
                Vk[[cpos[g] for g in cn.cols]] = Vf[c] @ h.W[c]
            Uf[k], Vf[k] = Uk, Vk
    return Uf, Vf


def expand(h: HSS, M: int, N: int) -> np.ndarray:
    """Dense matrix represented by the generators (Definition 2.2)."""
    t = h.tree
    H = np.zeros((M, N), complex)
    Uf, Vf = full_bases(h)
    for k in t.leaves():
        nd = t.nodes[k]
        H[np.ix_(nd.rows, nd.cols)] = h.D[k]
    for (a, b), Bab in h.B.items():
        na, nb = t.nodes[a], t.nodes[b]
        H[np.ix_(na.rows, nb.cols)] = Uf[a] @ Bab @ Vf[b].conj().T
    return H


def matvec(h: HSS, x: np.ndarray, M: int) -> np.ndarray:
    return expand(h, M, x.size) @ x


# --------------------------------------------------------------------------
# 1D HSS approximation of G^x by truncated SVD
# --------------------------------------------------------------------------

def hss_1d(x: np.ndarray, n: int, L: int, tol: float, leaf_row_bases=None) -> HSS:
    """Nested orthonormal bases for the HSS blocks G(J_tau, K_tau^c) and
    G(J_tau^c, K_tau)^* of the 1D transformed matrix (Section 2.5), bottom up;
    leaves keep the exact kernel block as D.  tol = 0 keeps every nonzero
    singular direction (an exact representation up to round-off).
    leaf_row_bases: optional {leaf key: orthonormal U} used in place of the
    truncated SVD of the leaf row blocks."""
    t = tree_1d(x, n, L)
    G = nudft.kernel_1d(x, n)
    M = x.size
    D, U, V, R, W, B = {}, {}, {}, {}, {}, {}
    Uf, Vf = {}, {}
    allrows = np.arange(M)
    allcols = np.arange(n)
    for l in range(L, 0, -1):
        for k in t.level(l):
            nd = t.nodes[k]
            rc = np.setdiff1d(allrows, nd.rows)
            cc = np.setdiff1d(allcols, nd.cols)
            if not nd.children:
                D[k] = G[np.ix_(nd.rows, nd.cols)]
                if leaf_row_bases is not None:
                    Uk = leaf_row_bases[k]
                else:
                    Uk, _ = trunc_left(G[np.ix_(nd.rows, cc)], tol)
                Vk, _ = trunc_left(G[np.ix_(rc, nd.cols)].conj().T, tol)
                U[k], V[k] = Uk, Vk
                Uf[k], Vf[k] = Uk, Vk
            else:
                c1, c2 = nd.children
                # row basis: compress the children's projected row blocks
                S = np.vstack([Uf[c].conj().T @ G[np.ix_(t.nodes[c].rows, cc)]
                               for c in (c1, c2)])
                Z, _ = trunc_left(S, tol)
                r1 = Uf[c1].shape[1]
                R[c1], R[c2] = Z[:r1], Z[r1:]
                T = np.vstack([(G[np.ix_(rc, t.nodes[c].cols)] @ Vf[c]).conj().T
                               for c in (c1, c2)])
                Y, _ = trunc_left(T, tol)
                s1 = Vf[c1].shape[1]
                W[c1], W[c2] = Y[:s1], Y[s1:]
                rpos = {g: i for i, g in enumerate(nd.rows)}
                cpos = {g: i for i, g in enumerate(nd.cols)}
                Uk = np.zeros((nd.rows.size, Z.shape[1]), complex)
                Vk = np.zeros((nd.cols.size, Y.shape[1]), complex)
                for c in (c1, c2):
                    Uk[[rpos[g] for g in t.nodes[c].rows]] = Uf[c] @ R[c]
                    Vk[[cpos[g] for g in t.nodes[c].cols]] = Vf[c] @ W[c]
                Uf[k], Vf[k] = Uk, Vk
    for l in range(1, L + 1):
        for k in t.level(l):
            for s in t.siblings(k):
                B[(k, s)] = Uf[k].conj().T @ G[np.ix_(t.nodes[k].rows, t.nodes[s].cols)] @ Vf[s]
    if L == 0:
        D[(0, 0)] = G.copy()
    return HSS(t, D, U, V, R, W, B)


# --------------------------------------------------------------------------
# face-splitting product of two 1D HSS matrices (Theorem 3.3)
# --------------------------------------------------------------------------

def face_split(points: np.ndarray, nx: int, ny: int, hx: HSS, hy: HSS) -> HSS:
    """Generators of H = H^x face-split H^y on the product tree.

    For a node xi = (alpha, beta) (p, q its positions in its parent's 1D
    children), with 1D generators of alpha and beta:
      U_xi = [D^x_xi . U^y_xi | U^x_xi . D^y_xi | U^x_xi . U^y_xi]
      V_xi = [I (x) V^y_beta  | V^x_alpha (x) I  | V^x_alpha (x) V^y_beta]
    where D^x_xi, U^x_xi are the rows J_xi of the 1D diagonal block / basis.
    Sibling interactions: same alpha -> blockdiag(I (x) B^y, 0, 0); same beta
    -> blockdiag(0, B^x (x) I, 0); both differ -> blockdiag(0, 0, B^x (x) B^y).
    Transfer matrices follow from restricting the parent's U, V to the
    child's rows / columns (nested bases of both 1D trees)."""
    L = hx.tree.L
    assert hy.tree.L == L
    t = tree_2d(points, nx, ny, L)
    tx, ty = hx.tree, hy.tree
    Ufx, Vfx = full_bases(hx)
    Ufy, Vfy = full_bases(hy)
    D, U, V, R, W, B = {}, {}, {}, {}, {}, {}

    def rows_in(sub_rows, node_rows):
        pos = {g: i for i, g in enumerate(node_rows)}
        return np.array([pos[g] for g in sub_rows], dtype=np.int64)

    def rU(h, k):
        return h.U[k].shape[1] if k in h.U else h.R[h.tree.nodes[k].children[0]].shape[1]

    def rV(h, k):
        return h.V[k].shape[1] if k in h.V else h.W[h.tree.nodes[k].children[0]].shape[1]

    # leaves
    for k in t.leaves():
        l, a, b = k
        nd = t.nodes[k]
        ax, by = (l, a), (l, b)
        if L == 0:
            D[k] = face(hx.D[ax], hy.D[by])
            continue
        ix = rows_in(nd.rows, tx.nodes[ax].rows)
        iy = rows_in(nd.rows, ty.nodes[by].rows)
        Dx, Dy = hx.D[ax][ix], hy.D[by][iy]
        Ux, Uy = hx.U[ax][ix], hy.U[by][iy]
        D[k] = face(Dx, Dy)
        U[k] = np.hstack([face(Dx, Uy), face(Ux, Dy), face(Ux, Uy)])
        dx, dy = Dx.shape[1], Dy.shape[1]
        Vx, Vy = hx.V[ax], hy.V[by]
        V[k] = np.hstack([np.kron(np.eye(dx), Vy), np.kron(Vx, np.eye(dy)),
                          np.kron(Vx, Vy)])

    for l in range(1, L + 1):
        for k in t.level(l):
            _, a, b = k
            ax, by = (l, a), (l, b)
            dx = tx.nodes[ax].cols.size
            dy = ty.nodes[by].cols.size
            rxU, ryU = rU(hx, ax), rU(hy, by)
            rxV, ryV = rV(hx, ax), rV(hy, by)
            # interactions with siblings
            for s in t.siblings(k):
                _, a2, b2 = s
                ax2, by2 = (l, a2), (l, b2)
                dx2 = tx.nodes[ax2].cols.size
                dy2 = ty.nodes[by2].cols.size
                rxV2, ryV2 = rV(hx, ax2), rV(hy, by2)
                wU = [dx * ryU, rxU * dy, rxU * ryU]
                wV = [dx2 * ryV2, rxV2 * dy2, rxV2 * ryV2]
                Bk = np.zeros((sum(wU), sum(wV)), complex)
                if a == a2:
                    Bk[:wU[0], :wV[0]] = np.kron(np.eye(dx), hy.B[(by, by2)])
                elif b == b2:
                    Bk[wU[0]:wU[0] + wU[1], wV[0]:wV[0] + wV[1]] = \
                        np.kron(hx.B[(ax, ax2)], np.eye(dy))
                else:
                    Bk[wU[0] + wU[1]:, wV[0] + wV[1]:] = \
                        np.kron(hx.B[(ax, ax2)], hy.B[(by, by2)])
                B[(k, s)] = Bk
            if l == 1:
                continue
            # transfer matrices to the parent lam = (tau, sigma)
            pa, pb = a // 2, b // 2
            tau, sig = (l - 1, pa), (l - 1, pb)
            p, q = a - 2 * pa, b - 2 * pb
            ax_s, by_s = (l, 2 * pa + 1 - p), (l, 2 * pb + 1 - q)     # 1D siblings
            Kx_t = tx.nodes[tau].cols
            Ky_s = ty.nodes[sig].cols
            dxt, dys = Kx_t.size, Ky_s.size
            own_x = np.searchsorted(Kx_t, tx.nodes[ax].cols)
            sib_x = np.searchsorted(Kx_t, tx.nodes[ax_s].cols)
            own_y = np.searchsorted(Ky_s, ty.nodes[by].cols)
            sib_y = np.searchsorted(Ky_s, ty.nodes[by_s].cols)
            rxtU, rysU = rU(hx, tau), rU(hy, sig)
            rxtV, rysV = rV(hx, tau), rV(hy, sig)
            Rx, Ry = hx.R[ax], hy.R[by]
            Wx, Wy = hx.W[ax], hy.W[by]
            # ---- R_xi: rows [blk1 dx*ryU | blk2 rxU*dy | blk3 rxU*ryU],
            #            cols [blk1 dxt*rysU | blk2 rxtU*dys | blk3 rxtU*rysU]
            cU = [dxt * rysU, rxtU * dys, rxtU * rysU]
            oU = np.cumsum([0] + cU)
            rwU = [dx * ryU, rxU * dy, rxU * ryU]
            orU = np.cumsum([0] + rwU)
            Rk = np.zeros((sum(rwU), sum(cU)), complex)
            # block1 own x-columns:  I (x) R^y_beta
            E_own_x = np.zeros((dx, dxt))
            E_own_x[np.arange(dx), own_x] = 1.0
            Rk[orU[0]:orU[1], oU[0]:oU[1]] = np.kron(E_own_x, Ry)
            # block1 sibling x-columns from U-block 3: (B^x V^x*_{sib}) (x) R^y
            BVx = hx.B[(ax, ax_s)] @ Vfx[ax_s].conj().T          # rxU x dx_sib
            BVx_full = np.zeros((rxU, dxt), complex)
            BVx_full[:, sib_x] = BVx
            Rk[orU[2]:orU[3], oU[0]:oU[1]] = np.kron(BVx_full, Ry)
            # block2 own y-columns: R^x (x) E_own_y
            E_own_y = np.zeros((dy, dys))
            E_own_y[np.arange(dy), own_y] = 1.0
            Rk[orU[1]:orU[2], oU[1]:oU[2]] = np.kron(Rx, E_own_y)
            # block2 sibling y-columns from U-block 3: R^x (x) (B^y V^y*_{sib})
            BVy = hy.B[(by, by_s)] @ Vfy[by_s].conj().T
            BVy_full = np.zeros((ryU, dys), complex)
            BVy_full[:, sib_y] = BVy
            Rk[orU[2]:orU[3], oU[1]:oU[2]] = np.kron(Rx, BVy_full)
            # block3: R^x (x) R^y
            Rk[orU[2]:orU[3], oU[2]:oU[3]] = np.kron(Rx, Ry)
            R[k] = Rk
            # ---- W_xi = blockdiag(E_x (x) W^y, W^x (x) E_y, W^x (x) W^y)
            cV = [dxt * rysV, rxtV * dys, rxtV * rysV]
            oV = np.cumsum([0] + cV)
            rwV = [dx * ryV, rxV * dy, rxV * ryV]
            orV = np.cumsum([0] + rwV)
            Wk = np.zeros((sum(rwV), sum(cV)), complex)
            Wk[orV[0]:orV[1], oV[0]:oV[1]] = np.kron(E_own_x, Wy)
            Wk[orV[1]:orV[2], oV[1]:oV[2]] = np.kron(Wx, E_own_y)
            Wk[orV[2]:orV[3], oV[2]:oV[3]] = np.kron(Wx, Wy)
            W[k] = Wk
    return HSS(t, D, U, V, R, W, B)


# --------------------------------------------------------------------------
# recompression (Section 2.3)
# --------------------------------------------------------------------------

def recompress(h: HSS, eps: float) -> HSS:
    t = h.tree
    L = t.L
    if L == 0:
        return HSS(t, dict(h.D), {}, {}, {}, {}, {})
    U, V = dict(h.U), dict(h.V)
    R, W, B = dict(h.R), dict(h.W), dict(h.B)
    F, Gf = {}, {}
    # stage 1: bottom-up orthogonalisation (exact)
    for l in range(L, -1, -1):
        for k in t.level(l):
            nd = t.nodes[k]
            if not nd.children:
                U[k], F[k] = thin_qr(U[k])
                V[k], Gf[k] = thin_qr(V[k])
                continue
            ch = nd.children
            for c1 in ch:
                for c2 in ch:
                    if c1 != c2:
                        B[(c1, c2)] = F[c1] @ B[(c1, c2)] @ Gf[c2].conj().T
            if k == t.root:
                continue
            SR = np.vstack([F[c] @ R[c] for c in ch])
            SW = np.vstack([Gf[c] @ W[c] for c in ch])
            QR_, F[k] = thin_qr(SR)
            QW_, Gf[k] = thin_qr(SW)
            o = 0
            for c in ch:
                r = F[c].shape[0]
                R[c] = QR_[o:o + r]
                o += r
            o = 0
            for c in ch:
                r = Gf[c].shape[0]
                W[c] = QW_[o:o + r]
                o += r
    # stage 2: top-down truncation
    SU = {t.root: None}
    SV = {t.root: None}
    for l in range(0, L):
        for k in t.level(l):
            ch = t.nodes[k].children
            P, Q, sU, sV = {}, {}, {}, {}
            for a in ch:
                blocksU = [B[(a, b)] for b in ch if b != a]
                blocksV = [B[(b, a)].conj().T for b in ch if b != a]
                if SU[k] is not None:
                    blocksU.append(R[a] * SU[k][None, :])
                    blocksV.append(W[a] * SV[k][None, :])
                P[a], sU[a] = trunc_left(np.hstack(blocksU), eps)
                Q[a], sV[a] = trunc_left(np.hstack(blocksV), eps)
            for a in ch:
                for b in ch:
                    if a != b:
                        B[(a, b)] = P[a].conj().T @ B[(a, b)] @ Q[b]
            for a in ch:
                if k != t.root:
                    R[a] = P[a].conj().T @ R[a]
                    W[a] = Q[a].conj().T @ W[a]
                an = t.nodes[a]
                if not an.children:
                    U[a] = U[a] @ P[a]
                    V[a] = V[a] @ Q[a]
                else:
                    for c in an.children:
                        R[c] = R[c] @ P[a]
                        W[c] = W[c] @ Q[a]
                SU[a], SV[a] = sU[a], sV[a]
    for a in t.nodes[t.root].children:
        R.pop(a, None)
        W.pop(a, None)
    return HSS(t, dict(h.D), U, V, R, W, B)


# --------------------------------------------------------------------------
# URV factorization and solution
# --------------------------------------------------------------------------

def full_qr(X):
    Q, R = np.linalg.qr(X, mode="complete")
    return Q, R


@dataclasses.dataclass
class URVNode:
    Omega: np.ndarray | None
    mchk: int
    Q: np.ndarray
    P: np.ndarray
    k: int
    D11: np.ndarray
    D12: np.ndarray
    U1: np.ndarray
    V2: np.ndarray
    U2: np.ndarray
    D22: np.ndarray


def urv_node(D, U, V) -> URVNode:
    """Size reduction, basis elimination and partial decomposition of one
    node (leaf or merged)."""
    m, n = D.shape
    rU, rV = U.shape[1], V.shape[1]
    if m >= n + rU:
        Om, T = full_qr(np.hstack([U, D]))
        mc = n + rU
        Uc, Dc = T[:mc, :rU], T[:mc, rU:]
    else:
        Om, mc, Uc, Dc = None, m, U, D
    k = n - rV
    if k > 0:
        Q0, R0 = full_qr(V)
        Q = np.hstack([Q0[:, rV:], Q0[:, :rV]])
        V2 = R0[:rV]
    else:
        k = 0
        Q = np.eye(n, dtype=complex)
        V2 = V
    if mc < k:
        raise ValueError("node has fewer rows than unknowns to eliminate")
    Dt = Dc @ Q
    P, _ = full_qr(Dt[:, :k]) if k > 0 else (np.eye(mc, dtype=complex), None)
    Dh = P.conj().T @ Dt
    Uh = P.conj().T @ Uc
    return URVNode(Om, mc, Q, P, k, Dh[:k, :k], Dh[:k, k:], Uh[:k], V2, Uh[k:],
                   Dh[k:, k:])


@dataclasses.dataclass
class URV:
    h: HSS
    nodes: dict
    root_Q: np.ndarray
    root_R: np.ndarray


def urv_factor(h: HSS) -> URV:
    t = h.tree
    L = t.L
    cur = {}      # node -> (D, U, V) of the (merged) node
    for k in t.leaves():
        if L == 0:
            break
        cur[k] = (h.D[k], h.U[k], h.V[k])
    fac = {}
    for l in range(L, 0, -1):
        for k in t.level(l):
            D, U, V = cur[k]
            fac[k] = urv_node(D, U, V)
        for k in t.level(l - 1):
            ch = t.nodes[k].children
            blocks = []
            for i in ch:
                row = []
                for j in ch:
                    if i == j:
                        row.append(fac[i].D22)
                    else:
                        row.append(fac[i].U2 @ h.B[(i, j)] @ fac[j].V2.conj().T)
                blocks.append(row)
            Dp = np.block(blocks)
            if k == t.root:
                cur[k] = (Dp, None, None)
            else:
                Up = np.vstack([fac[i].U2 @ h.R[i] for i in ch])
                Vp = np.vstack([fac[i].V2 @ h.W[i] for i in ch])
                cur[k] = (Dp, Up, Vp)
    Droot = h.D[t.root] if L == 0 else cur[t.root][0]
    Qr, Rr = np.linalg.qr(Droot, mode="reduced")
    return URV(h, fac, Qr, Rr)


def urv_solve(u: URV, f: np.ndarray, N: int) -> np.ndarray:
    """Least-squares solution of H c = f using the URV factors (bottom-up
    transform of f, root least squares, top-down back substitution)."""
    h, t = u.h, u.h.tree
    L = t.L
    fh1, fh2 = {}, {}
    cur = {k: f[t.nodes[k].rows] for k in t.leaves()}
    for l in range(L, 0, -1):
        for k in t.level(l):
            nd = u.nodes[k]
            fk = cur[k]
            if nd.Omega is not None:
                fk = (nd.Omega.conj().T @ fk)[:nd.mchk]
            fh = nd.P.conj().T @ fk
            fh1[k], fh2[k] = fh[:nd.k], fh[nd.k:]
        for k in t.level(l - 1):
            cur[k] = np.concatenate([fh2[c] for c in t.nodes[k].children])
    froot = cur[t.root]
    croot = sla.solve_triangular(u.root_R, u.root_Q.conj().T @ froot)
    c = np.zeros(N, complex)
    if L == 0:
        c[t.nodes[t.root].cols] = croot
        return c
    cplus = {t.root: croot}
    bhat = {t.root: None}
    for l in range(0, L):
        for k in t.level(l):
            ch = t.nodes[k].children
            c2, o = {}, 0
            for i in ch:
                r = u.nodes[i].V2.shape[0]
                c2[i] = cplus[k][o:o + r]
                o += r
            for i in ch:
                nd = u.nodes[i]
                b = np.zeros(nd.U2.shape[1], complex)
                for j in ch:
                    if j != i:
                        b = b + h.B[(i, j)] @ (u.nodes[j].V2.conj().T @ c2[j])
                if bhat[k] is not None:
                    b = b + h.R[i] @ bhat[k]
                bhat[i] = b
                rhs = fh1[i] - nd.D12 @ c2[i] - nd.U1 @ b
                c1 = sla.solve_triangular(nd.D11, rhs) if nd.k > 0 else np.zeros(0, complex)
                cplus[i] = nd.Q @ np.concatenate([c1, c2[i]])
                if not t.nodes[i].children:
                    c[t.nodes[i].cols] = cplus[i]
    return c


# --------------------------------------------------------------------------
# Algorithm 4.1 end to end
# --------------------------------------------------------------------------

def build(points, nx, ny, eps, leaf=16, recomp=True):
    L = depth_for(nx, ny, leaf)
    hx = hss_1d(points[:, 0], nx, L, eps / 10.0)
    hy = hss_1d(points[:, 1], ny, L, eps / 10.0)
    h = face_split(points, nx, ny, hx, hy)
    return recompress(h, eps) if recomp else h


def direct_solve(points, f, nx, ny, eps, leaf=16):
    """c = F^{-1} H~^+ (phi^* f): the online stage of Algorithm 4.1 with the
    centring phase applied to f; returns the (nx, ny) centred coefficients."""
    h = build(points, nx, ny, eps, leaf)
    u = urv_factor(h)
    phi = nudft.centring_phase(points, nx, ny)
    chat = urv_solve(u, phi.conj() * f, nx * ny)
    return np.fft.ifft2(chat.reshape(nx, ny))
