"""P1 finite-element solves either side of the boundary matvec (oracle; test only).

Section 2 of the paper splits the magnetostatic potential u = u1 + u2 in the
body Omega (eqs. u1Poiss, u1Neumann, mainInt, u2diri):

    Delta u1 = div M in Omega,   du1/dn = M.n on the boundary;
    u2 = (K + D) u1 on the boundary (the boundary operator of dense.py / h2.py);
    Delta u2 = 0 in Omega with those Dirichlet values;
    H = -grad u,   E = -(mu0 / 2) int_Omega M.H  (here mu0 = Ms = 1).

Discretisation: continuous piecewise-linear u on a tetrahedral mesh, M
constant per tetrahedron.  Multiplying the u1 equation by a test function v
and integrating by parts, the boundary terms cancel by the Neumann condition:

    int grad u1 . grad v = int M . grad v      for every P1 v,

a singular system (constants solve the homogeneous one) whose right side sums
to zero; u1 is taken with zero node sum (H does not depend on that constant:
the boundary operator maps a constant c to -c, so u2 moves by -c).  u2 solves
the same stiffness matrix on the interior nodes with the boundary nodes fixed.

Everything is FP64 and direct: sparse LU (scipy) for both solves.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def element_geometry(xyz: np.ndarray, tets: np.ndarray):
    """Volumes (T,) and the gradients of the four P1 hat functions (T, 4, 3).

    With J = [x1 - x0, x2 - x0, x3 - x0] (columns), the barycentric
    coordinates of vertices 1..3 are the rows of J^{-1} applied to x - x0, so
    their gradients are the rows of J^{-1}; vertex 0's is minus their sum.
    """
    x = xyz[tets]
    J = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    g = np.empty((tets.shape[0], 4, 3))
    g[:, 1:] = Jinv
    g[:, 0] = -Jinv.sum(axis=1)
    return np.abs(det) / 6.0, g


def stiffness(xyz: np.ndarray, tets: np.ndarray) -> sp.csr_matrix:
    """A_ij = int grad phi_i . grad phi_j (sum over tetrahedra of vol g_a . g_b)."""
    vol, g = element_geometry(xyz, tets)
    loc = vol[:, None, None] * np.einsum("tad,tbd->tab", g, g)
    rows = np.repeat(tets, 4, axis=1).ravel()
    cols = np.tile(tets, (1, 4)).ravel()
    n = xyz.shape[0]
    return sp.coo_matrix((loc.ravel(), (rows, cols)), shape=(n, n)).tocsr()


def neumann_rhs(xyz: np.ndarray, tets: np.ndarray, m: np.ndarray) -> np.ndarray:
    """b_i = int M . grad phi_i (M constant per tetrahedron)."""
    vol, g = element_geometry(xyz, tets)
    loc = vol[:, None] * np.einsum("tad,td->ta", g, m)
    b = np.zeros(xyz.shape[0])
    np.add.at(b, tets.ravel(), loc.ravel())
    return b


def boundary_surface(tets: np.ndarray, xyz: np.ndarray):
    """The faces that belong to one tetrahedron only, oriented outward.

    Returns (nodes, tri): the boundary node indices (sorted) and the triangles
    as indices into `nodes`, counter-clockwise seen from outside (the normal
    (b - a) x (c - a) points away from the tetrahedron's fourth vertex).
    """
    faces, opposite = [], []
    for q in range(4):
        keep = [r for r in range(4) if r != q]
        faces.append(tets[:, keep])
        opposite.append(tets[:, q])
    faces = np.concatenate(faces)
    opposite = np.concatenate(opposite)
    key = np.sort(faces, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    once = cnt[inv.ravel()] == 1
    f, d = faces[once], opposite[once]
    a, b, c = xyz[f[:, 0]], xyz[f[:, 1]], xyz[f[:, 2]]
    inward = np.einsum("ij,ij->i", np.cross(b - a, c - a), xyz[d] - a) > 0
    f[inward] = f[inward][:, [0, 2, 1]]
    nodes = np.unique(f)
    local = np.searchsorted(nodes, f).astype(np.int32)
    return nodes, local


def solve_neumann(A: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    """The solution of A u = b with zero node sum: the bordered system
    [[A, 1], [1^T, 0]] [u; lambda] = [b; 0] (lambda = 0 when b sums to zero)."""
    n = A.shape[0]
    one = sp.csr_matrix(np.ones((n, 1)))
    K = sp.bmat([[A, one], [one.T, None]], format="csc")
    sol = spla.spsolve(K, np.concatenate([b, [0.0]]))
    return sol[:n]


def solve_dirichlet(A: sp.csr_matrix, fixed: np.ndarray, values: np.ndarray) -> np.ndarray:
    """A u = 0 on the free nodes with u = values on the `fixed` nodes."""
    n = A.shape[0]
    free = np.setdiff1d(np.arange(n), fixed)
    u = np.zeros(n)
    u[fixed] = values
    rhs = -A[free][:, fixed] @ values
    u[free] = spla.spsolve(A[free][:, free].tocsc(), rhs)
    return u


def field(xyz: np.ndarray, tets: np.ndarray, u: np.ndarray) -> np.ndarray:
    """H = -grad u per tetrahedron (T, 3)."""
    _, g = element_geometry(xyz, tets)
    return -np.einsum("ta,tad->td", u[tets], g)


def energy(xyz: np.ndarray, tets: np.ndarray, m: np.ndarray, h: np.ndarray) -> float:
    """E = -(1/2) int M . H over the body."""
    vol, _ = element_geometry(xyz, tets)
    return float(-0.5 * np.sum(vol * np.einsum("td,td->t", m, h)))


def demag(xyz: np.ndarray, tets: np.ndarray, m: np.ndarray, boundary_op) -> dict:
    """The whole evaluation of Section 2 for magnetisation m (T, 3).

    boundary_op(nodes_xyz, tri, u1_boundary) -> u2_boundary applies (K + D) on
    the boundary surface (nodes in the order of `nodes`)."""
    A = stiffness(xyz, tets)
    b = neumann_rhs(xyz, tets, m)
    u1 = solve_neumann(A, b)
    nodes, tri = boundary_surface(tets, xyz)
    u2b = boundary_op(xyz[nodes], tri, u1[nodes])
    u2 = solve_dirichlet(A, nodes, u2b)
    h = field(xyz, tets, u1 + u2)
    return {"u1": u1, "u2": u2, "h": h, "energy": energy(xyz, tets, m, h), "nodes": nodes, "tri": tri}
