"""Mesh geometry for the collocation matrix (oracle; test infrastructure only).

Section 3 of the paper places the collocation points xi_i at the mesh nodes,
with piecewise linear hat functions phi_i, and eq. (matrix_definition) puts
(Psi(xi_i)/(4 pi) - 1) on the diagonal, Psi being the solid angle subtended at
xi_i (Section 2, after eq. mainInt).  The paper does not say how Psi is
evaluated on a polyhedral surface; here it is the interior solid angle of the
polyhedral cone at the node, i.e. the area of the spherical polygon cut from the
unit sphere, by Gauss-Bonnet:

    Psi_i = 2 pi - sum over edges (i, k) of theta_e,

theta_e being the signed angle between the outward normals of the two
triangles sharing the edge (positive where the edge is convex).
"""
from __future__ import annotations

import numpy as np


def triangle_normals_areas(xyz: np.ndarray, tri: np.ndarray):
    """Unit outward normals (T x 3) and areas (T) of flat triangles."""
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cr = np.cross(b - a, c - a)
    two_area = np.linalg.norm(cr, axis=1)
    return cr / two_area[:, None], 0.5 * two_area


def check_mesh(xyz: np.ndarray, tri: np.ndarray) -> None:
    """Raise ValueError unless the mesh is a closed, consistently oriented 2-manifold.

    Conditions: indices in range; no triangle repeats a vertex or has zero
    area; every directed edge occurs exactly once and its reverse exactly once;
    the enclosed (signed) volume is positive, i.e. normals point outward.
    """
    n = xyz.shape[0]
    t = np.asarray(tri, dtype=np.int64)
    if t.ndim != 2 or t.shape[1] != 3 or t.shape[0] == 0:
        raise ValueError("triangles must be a non-empty T x 3 array")
    if t.min() < 0 or t.max() >= n:
        raise ValueError("triangle index out of range")
    if np.any((t[:, 0] == t[:, 1]) | (t[:, 1] == t[:, 2]) | (t[:, 0] == t[:, 2])):
        raise ValueError("degenerate triangle (repeated vertex)")
    _, area = triangle_normals_areas(xyz, t)
    if np.any(~(area > 0.0)):
        raise ValueError("degenerate triangle (zero area)")
    d = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    key = d[:, 0] * n + d[:, 1]
    rkey = d[:, 1] * n + d[:, 0]
    uk, cnt = np.unique(key, return_counts=True)
    if np.any(cnt != 1):
        raise ValueError("directed edge used twice (inconsistent orientation or non-manifold)")
    if not np.all(np.isin(rkey, uk)):
        raise ValueError("open or non-manifold edge")
    if signed_volume(xyz, t) <= 0.0:
        raise ValueError("signed volume is not positive (inward orientation)")


def signed_volume(xyz: np.ndarray, tri: np.ndarray) -> float:
    """Volume enclosed by the polyhedron, (1/6) sum_T r1 . (r2 x r3)."""
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    return float(np.sum(np.einsum("ij,ij->i", a, np.cross(b, c))) / 6.0)


def node_solid_angles(xyz: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Interior solid angle Psi_i at every node (steradian).

    For each undirected edge {i, k}: T_a is the triangle that runs i -> k in
    its counter-clockwise order and T_b the one that runs k -> i; with
    e = (xi_k - xi_i)/|.|, theta = atan2((n_a x n_b) . e, n_a . n_b).  theta is
    symmetric in the two end nodes and is subtracted from 2 pi at both.
    """
    n = xyz.shape[0]
    t = np.asarray(tri, dtype=np.int64)
    nrm, _ = triangle_normals_areas(xyz, t)
    T = t.shape[0]
    src = np.concatenate([t[:, 0], t[:, 1], t[:, 2]])
    dst = np.concatenate([t[:, 1], t[:, 2], t[:, 0]])
    owner = np.concatenate([np.arange(T)] * 3)
    fwd = src < dst                                 # one directed copy per undirected edge
    key_all = src * n + dst
    order = np.argsort(key_all)
    sorted_keys = key_all[order]
    i, k, ta = src[fwd], dst[fwd], owner[fwd]
    pos = np.searchsorted(sorted_keys, k * n + i)   # the reverse edge k -> i
    tb = owner[order[pos]]
    e = xyz[k] - xyz[i]
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    na, nb = nrm[ta], nrm[tb]
    theta = np.arctan2(np.einsum("ij,ij->i", np.cross(na, nb), e), np.einsum("ij,ij->i", na, nb))
    psi = np.full(n, 2.0 * np.pi)
    np.subtract.at(psi, i, theta)
    np.subtract.at(psi, k, theta)
    return psi


def diagonal(xyz: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """D_ii = Psi_i/(4 pi) - 1 (eq. matrix_definition, second term)."""
    return node_solid_angles(xyz, tri) / (4.0 * np.pi) - 1.0


def incidence(n_nodes: int, tri: np.ndarray):
    """CSR of node -> incident triangles: (offsets (N+1), triangle ids, local vertex 0..2)."""
    t = np.asarray(tri, dtype=np.int64)
    node = t.ravel()
    tid = np.repeat(np.arange(t.shape[0]), 3)
    loc = np.tile(np.arange(3), t.shape[0])
    order = np.argsort(node, kind="stable")
    off = np.zeros(n_nodes + 1, dtype=np.int64)
    np.add.at(off, node + 1, 1)
    off = np.cumsum(off)
    return off, tid[order], loc[order]
