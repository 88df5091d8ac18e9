"""The dense collocation matrix M = K + D (oracle; test infrastructure only).

Section 3, eqs. (matrix_definition) and (denseMat): with P1 hat functions
phi_j on the surface mesh and collocation at the nodes xi_i,

    m_ij = (1/4pi) integral phi_j(y) n(y).(xi_i - y)/|xi_i - y|^3 dS_y
           + (Psi(xi_i)/(4 pi) - 1) delta_ij,

u2 = M u1.  The kernel sign is the one under which M maps a constant to minus
itself (u1 = const gives u = 0, so u2 = -u1) and under which the uniformly
magnetised sphere gives u2 = -2z/3; the paper's literal G = -1/(4 pi r)
combined with dG/dn' has the opposite sign, which would give M 1 = 0 on smooth
parts -- that reading contradicts the paper's own physics and is not used.

Triangles incident to xi_i contribute nothing to row i: n.(xi_i - y) = 0 on
them.  Incidence is decided by index.
"""
from __future__ import annotations

import numpy as np

from . import geometry, lindholm


def k_rows(xyz: np.ndarray, tri: np.ndarray, rows) -> np.ndarray:
    """Rows `rows` of the dense double-layer matrix K (len(rows) x N), exact."""
    t = np.asarray(tri, dtype=np.int64)
    n = xyz.shape[0]
    rows = np.atleast_1d(np.asarray(rows, dtype=np.int64))
    r1, r2, r3 = xyz[t[:, 0]], xyz[t[:, 1]], xyz[t[:, 2]]
    out = np.zeros((rows.size, n))
    for q, i in enumerate(rows):
        keep = ~np.any(t == i, axis=1)
        L = lindholm.weights(xyz[i][None, :], r1[keep], r2[keep], r3[keep])
        out[q] = np.bincount(t[keep].ravel(), weights=L.ravel(), minlength=n)
    return out


def m_rows(xyz: np.ndarray, tri: np.ndarray, rows, diag=None) -> np.ndarray:
    """Rows of M = K + D."""
    rows = np.atleast_1d(np.asarray(rows, dtype=np.int64))
    out = k_rows(xyz, tri, rows)
    d = geometry.diagonal(xyz, tri) if diag is None else diag
    out[np.arange(rows.size), rows] += d[rows]
    return out


def dense_m(xyz: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """The full N x N matrix M (small meshes only)."""
    return m_rows(xyz, tri, np.arange(xyz.shape[0]))


def apply_rows(xyz: np.ndarray, tri: np.ndarray, u1: np.ndarray, rows) -> np.ndarray:
    """(M u1)[rows] for u1 of shape (r, N): returns (r, len(rows))."""
    return (m_rows(xyz, tri, rows) @ np.atleast_2d(u1).T).T
