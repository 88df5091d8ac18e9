"""Algebraic recompression of the interpolation H2 matrix (oracle; test only).

Section 4 of the paper: the matrix is turned into an H2 matrix by a purely
algebraic recompression, with ranks adapted to the accuracy needed instead of
fixed by the analytic construction (the paper notes that analytic ranks are
larger than necessary).  Reproduced here on the interpolation H2 matrix of
h2.py (the same cluster tree, block tree and exact blocks): the nested cluster
bases V (rows) and W (columns) are replaced by orthonormal nested bases of
adaptive rank, chosen by truncated singular value decompositions that are
weighted by every low-rank block the basis serves, and each coupling matrix
is projected onto the new bases.  Every step is a QR or SVD of an explicit
matrix; nothing is squared.

Rows (the columns take the same steps with W, V and S^T in place of V, W, S):

1. Orthogonalisation factors of the other side's basis, from the leaves up:
   R'_s = R factor of QR(W_s) at a leaf, of QR([R'_c1 E_c1; R'_c2 E_c2]) above,
   so that W_s = (orthonormal) R'_s and |W_s^T v| = |R'_s v|.
2. Weights, from the root down: the low-rank blocks that the row basis of t
   serves are V_t B_t Q^T for some orthonormal Q, with
       B_t = [E_t L_parent, S_ts1 R'_s1^T, S_ts2 R'_s2^T, ...]
   over the admissible blocks (t, s) of t; L_t = R^T of QR(B_t^T) keeps
   L_t L_t^T = B_t B_t^T in k x k.
3. Truncation, from the leaves up:
       Y_t = V_t (leaf)  or  [P_c1 E_c1; P_c2 E_c2]  (children c1, c2 done),
   thin SVD of Y_t L_t = U diag(sigma) Z^T, rank r_t = #{i : sigma_i > eps sigma_1};
   U_r is the new leaf basis Q_t (leaf) or, split by the children's ranks, the
   new transfers F_c1 (r_c1 x r_t), F_c2 (r_c2 x r_t); P_t = U_r^T Y_t (r_t x k)
   is the old basis in the new one: V_t ~ (new basis of t) P_t.
4. Coupling: S'_ts = P_t S_ts P'_s^T (r_t x r'_s).

The new basis of t is Q_t at a leaf and diag(basis c1, basis c2) [F_c1; F_c2]
above: orthonormal and nested.  The matvec runs the passes of h2.py with Q, F
and S' in place of V or W, E and S:

    xh_s = Q'_s^T x|_s (leaves),  xh_t = sum_c F'_c^T xh_c (upwards),
    yh_t = sum_s S'_ts xh_s,  yh_c += F_c yh_t (downwards),  y|_t += Q_t yh_t,

plus the exact blocks and the diagonal of h2.py.  eps = 0 keeps every nonzero
singular value: the interpolation H2 matrix up to rounding.  eps is relative
to the largest singular value of the cluster's weighted basis.
"""
from __future__ import annotations

import numpy as np


def r_factor(X: np.ndarray) -> np.ndarray:
    """R of a thin QR of X (min(rows, cols) x cols)."""
    if X.shape[0] == 0:
        return np.zeros((0, X.shape[1]))
    return np.linalg.qr(X, mode="r")


class Recompressed:
    """Recompressed H2 matrix of an h2.H2Oracle (same trees and exact blocks)."""

    def __init__(self, H, eps: float, cache_coupling: bool = True):
        if not eps >= 0.0:
            raise ValueError("eps must be >= 0")
        self.H, self.eps = H, float(eps)
        self.cache_coupling = cache_coupling
        self._S = {}
        Rv = self._orth_factors(H.V)
        Rw = self._orth_factors(H.W)
        self.row = self._truncate(H.V, self._weights(Rw, transpose=False))
        self.col = self._truncate(H.W, self._weights(Rv, transpose=True))

    # -- construction -----------------------------------------------------------
    def _orth_factors(self, leaf_basis) -> dict:
        H = self.H
        R = {}
        for c in range(H.n_clusters - 1, -1, -1):        # children have larger preorder ids
            if H.is_leaf(c):
                R[c] = r_factor(leaf_basis(c))
            else:
                c0, c1 = H.child0[c], H.child1[c]
                R[c] = r_factor(np.vstack([R[c0] @ H.E(c0), R[c1] @ H.E(c1)]))
        return R

    def _weights(self, R_other: dict, transpose: bool) -> dict:
        """L_t (k x w_t) with L_t L_t^T = B_t B_t^T, from the root down."""
        H = self.H
        served = [[] for _ in range(H.n_clusters)]
        for t, s in H.far:
            if transpose:
                served[s].append(int(t))
            else:
                served[t].append(int(s))
        L = {}
        for t in range(H.n_clusters):                     # parents precede children
            parts = []
            p = H.parent[t]
            if p >= 0 and L[p].shape[1] > 0:
                parts.append(H.E(t) @ L[p])
            for s in served[t]:
                S = H.S(s, t).T if transpose else H.S(t, s)
                parts.append(S @ R_other[s].T)
            L[t] = r_factor(np.hstack(parts).T).T if parts else np.zeros((H.k, 0))
        return L

    def _truncate(self, leaf_basis, L: dict) -> dict:
        H = self.H
        Q, F, P, sig = {}, {}, {}, {}
        rank = np.zeros(H.n_clusters, dtype=np.int64)
        for c in range(H.n_clusters - 1, -1, -1):
            if H.is_leaf(c):
                Y = leaf_basis(c)
            else:
                c0, c1 = H.child0[c], H.child1[c]
                Y = np.vstack([P[c0] @ H.E(c0), P[c1] @ H.E(c1)])
            if L[c].shape[1] > 0:
                U, s, _ = np.linalg.svd(Y @ L[c], full_matrices=False)
                r = int(np.count_nonzero(s > self.eps * s[0])) if s[0] > 0.0 else 0
            else:                                          # the basis serves no block
                U, s, r = np.zeros((Y.shape[0], 0)), np.zeros(0), 0
            U = U[:, :r]
            rank[c], sig[c], P[c] = r, s, U.T @ Y
            if H.is_leaf(c):
                Q[c] = U
            else:
                F[c0], F[c1] = U[:rank[c0]], U[rank[c0]:]
        return {"Q": Q, "F": F, "P": P, "rank": rank, "sigma": sig}

    # -- pieces -----------------------------------------------------------------
    def S(self, t, s):
        """Projected coupling matrix S'_ts = P_t S_ts P'_s^T (r_t x r'_s)."""
        key = (t, s)
        if key in self._S:
            return self._S[key]
        out = self.row["P"][t] @ self.H.S(t, s) @ self.col["P"][s].T
        if self.cache_coupling:
            self._S[key] = out
        return out

    def basis(self, side: str, c):
        """The explicit new basis of cluster c (its rows x rank), from Q and F."""
        d = self.row if side == "row" else self.col
        H = self.H
        if H.is_leaf(c):
            return d["Q"][c]
        c0, c1 = H.child0[c], H.child1[c]
        return np.vstack([self.basis(side, c0) @ d["F"][c0], self.basis(side, c1) @ d["F"][c1]])

    # -- matvec -----------------------------------------------------------------
    def apply(self, u1: np.ndarray) -> np.ndarray:
        """u2 = (K_rec + D) u1 for u1 of shape (r, N) (or (N,)); returns the same shape."""
        H = self.H
        u = np.asarray(u1, dtype=np.float64)
        squeeze = u.ndim == 1
        x = np.atleast_2d(u).T.copy()
        C = H.n_clusters
        Qc, Fc = self.col["Q"], self.col["F"]
        xh = [None] * C
        for c in range(C - 1, -1, -1):
            if H.is_leaf(c):
                xs = x[H.nodes(c)]
                if np.any(xs != 0.0):
                    xh[c] = Qc[c].T @ xs
            else:
                acc = None
                for ch in (H.child0[c], H.child1[c]):
                    if xh[ch] is not None:
                        v = Fc[ch].T @ xh[ch]
                        acc = v if acc is None else acc + v
                xh[c] = acc
        yh = [None] * C
        for t in range(C):
            for s in H.far_of[t]:
                if xh[s] is not None:
                    v = self.S(t, s) @ xh[s]
                    yh[t] = v if yh[t] is None else yh[t] + v
        Qr, Fr = self.row["Q"], self.row["F"]
        for c in range(1, C):
            p = H.parent[c]
            if yh[p] is not None:
                v = Fr[c] @ yh[p]
                yh[c] = v if yh[c] is None else yh[c] + v
        y = np.zeros_like(x)
        for c in range(C):
            if H.is_leaf(c) and yh[c] is not None:
                y[H.nodes(c)] += Qr[c] @ yh[c]
        y = H.near_field(x, y)
        y += H.D[:, None] * x
        out = y.T
        return out[0] if squeeze else out

    # -- sizes ------------------------------------------------------------------
    def counts(self) -> dict:
        """Ranks and the entries of every stored piece."""
        H = self.H
        rr, rc = self.row["rank"], self.col["rank"]
        size = H.end - H.begin
        leaves = H.child0 < 0
        transfer = sum(rr[c] * rr[H.parent[c]] + rc[c] * rc[H.parent[c]] for c in range(1, H.n_clusters))
        return dict(coupling_entries=int(sum(rr[t] * rc[s] for t, s in H.far)),
                    basis_entries=int(np.sum(size[leaves] * (rr[leaves] + rc[leaves]))),
                    transfer_entries=int(transfer),
                    rank_row_max=int(rr.max()), rank_col_max=int(rc.max()),
                    rank_row_mean=float(rr.mean()), rank_col_mean=float(rc.mean()))
