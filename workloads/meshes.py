"""Seeded synthetic closed triangle meshes.

These generators hold no part of the boundary-operator arithmetic: they only
produce node coordinates (float64, N x 3) and triangles (int32, T x 3, 0-based,
counter-clockwise when seen from outside, i.e. outward normals) for the three
shape families the paper tests on (Section 5: sphere, flat rectangular prism,
torus).  Both the oracle and the GPU library consume them.
"""
from __future__ import annotations

import numpy as np

__all__ = ["icosphere", "cuboid", "torus", "icosahedron"]


def _orient_outward(xyz: np.ndarray, tri: np.ndarray, center: np.ndarray) -> np.ndarray:
    """Flip triangles whose (r2-r1)x(r3-r1) points towards `center` (star-shaped meshes only)."""
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    nrm = np.cross(b - a, c - a)
    inward = np.einsum("ij,ij->i", nrm, (a + b + c) / 3.0 - center) < 0
    out = tri.copy()
    out[inward] = out[inward][:, [0, 2, 1]]
    return out


def icosahedron():
    """The 12 vertices (0, +-1, +-phi) and cyclic permutations, normalised; 20 outward faces.

    Faces are found as the triples of mutually adjacent vertices (edge length 2
    before normalisation), sorted lexicographically, then oriented outward.
    """
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v.append((0.0, s1, s2 * phi))
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v.append((s1, s2 * phi, 0.0))
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v.append((s2 * phi, 0.0, s1))
    v = np.array(v, dtype=np.float64)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    adj = np.abs(d - 2.0) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    tri = np.array(faces, dtype=np.int64)
    assert tri.shape == (20, 3)
    v = v / np.linalg.norm(v, axis=1, keepdims=True)
    tri = _orient_outward(v, tri, np.zeros(3))
    return v, tri.astype(np.int32)


def _subdivide(xyz: np.ndarray, tri: np.ndarray):
    """Midpoint subdivision, re-projected to the unit sphere.

    New (edge-midpoint) vertices are numbered after the old ones in order of
    first appearance, scanning triangles in order and their edges (ab, bc, ca).
    """
    t = tri.astype(np.int64)
    n0 = xyz.shape[0]
    e = np.stack([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]], axis=1).reshape(-1, 2)
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    key = lo * (n0 + 1) + hi
    uniq, first, inv = np.unique(key, return_index=True, return_inverse=True)
    order = np.argsort(first, kind="stable")          # unique edges by first appearance
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    mid_id = n0 + rank[inv]                            # per (triangle, edge) new vertex id
    ue_lo = lo[first[order]]
    ue_hi = hi[first[order]]
    mid = 0.5 * (xyz[ue_lo] + xyz[ue_hi])
    mid /= np.linalg.norm(mid, axis=1, keepdims=True)
    new_xyz = np.concatenate([xyz, mid], axis=0)
    m = mid_id.reshape(-1, 3)                          # ab, bc, ca
    a, b, c = t[:, 0], t[:, 1], t[:, 2]
    ab, bc, ca = m[:, 0], m[:, 1], m[:, 2]
    new_tri = np.stack([
        np.stack([a, ab, ca], 1),
        np.stack([ab, b, bc], 1),
        np.stack([ca, bc, c], 1),
        np.stack([ab, bc, ca], 1),
    ], axis=1).reshape(-1, 3)
    return new_xyz, new_tri


def icosphere(level: int, jitter: float = 0.0, seed: int = 0):
    """Unit-sphere triangulation: icosahedron subdivided `level` times.

    N = 10*4**level + 2 nodes, T = 20*4**level triangles.  With jitter a > 0
    every vertex is moved radially, x <- x*(1 + d), d ~ U(-a, a) drawn from
    numpy default_rng(seed) in vertex-index order.
    """
    xyz, tri = icosahedron()
    tri = tri.astype(np.int64)
    for _ in range(level):
        xyz, tri = _subdivide(xyz, tri)
    if jitter > 0.0:
        d = np.random.default_rng(seed).uniform(-jitter, jitter, size=xyz.shape[0])
        xyz = xyz * (1.0 + d)[:, None]
    return np.ascontiguousarray(xyz, dtype=np.float64), np.ascontiguousarray(tri, dtype=np.int32)


def cuboid(lx: float = 2000.0, ly: float = 2000.0, lz: float = 20.0, h: float = 5.0,
           jitter: float = 0.0, seed: int = 0):
    """Surface of the box [0,lx]x[0,ly]x[0,lz] on a structured grid of spacing h.

    Each face is a grid of squares split into two right triangles along the
    (i, j) -> (i+1, j+1) diagonal.  With jitter a > 0 every vertex moves in the
    plane of its face by U(-a, a) per free axis (numpy default_rng(seed)):
    face-interior nodes along both in-plane axes, edge nodes along their edge
    only, corners not at all.
    """
    nx, ny, nz = int(round(lx / h)), int(round(ly / h)), int(round(lz / h))
    # surface grid nodes: (i, j, k) with at least one index on the boundary
    I, J, K = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    onb = (I == 0) | (I == nx) | (J == 0) | (J == ny) | (K == 0) | (K == nz)
    gi, gj, gk = I[onb], J[onb], K[onb]
    idmap = -np.ones((nx + 1, ny + 1, nz + 1), dtype=np.int64)
    idmap[gi, gj, gk] = np.arange(gi.size)
    xyz = np.stack([gi * (lx / nx), gj * (ly / ny), gk * (lz / nz)], axis=1).astype(np.float64)

    tris = []

    def face(fixed_axis: int, fixed_val: int, outward_sign: int):
        axes = [a for a in range(3) if a != fixed_axis]
        n = [nx, ny, nz]
        a0, a1 = axes
        u, v = np.meshgrid(np.arange(n[a0]), np.arange(n[a1]), indexing="ij")
        u = u.ravel(); v = v.ravel()

        def node(du, dv):
            idx = [None, None, None]
            idx[fixed_axis] = np.full(u.shape, fixed_val)
            idx[a0] = u + du
            idx[a1] = v + dv
            return idmap[idx[0], idx[1], idx[2]]

        p00, p10, p11, p01 = node(0, 0), node(1, 0), node(1, 1), node(0, 1)
        t1 = np.stack([p00, p10, p11], 1)
        t2 = np.stack([p00, p11, p01], 1)
        # (a0, a1, fixed) right-handed?  e_a0 x e_a1 = +e_fixed when the triple is cyclic
        cyclic = (a0, a1, fixed_axis) in [(0, 1, 2), (1, 2, 0), (2, 0, 1)]
        if (1 if cyclic else -1) != outward_sign:
            t1 = t1[:, [0, 2, 1]]
            t2 = t2[:, [0, 2, 1]]
        tris.append(np.stack([t1, t2], 1).reshape(-1, 3))

    face(2, 0, -1); face(2, nz, +1)
    face(1, 0, -1); face(1, ny, +1)
    face(0, 0, -1); face(0, nx, +1)
    tri = np.concatenate(tris, axis=0)

    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter, jitter, size=xyz.shape)
        lim = np.array([nx, ny, nz])
        g = np.stack([gi, gj, gk], 1)
        on_face = (g == 0) | (g == lim)          # per axis: node lies on a face normal to it
        free = ~on_face                          # a node moves only along axes it is not pinned on
        xyz = xyz + np.where(free, d, 0.0)
    return np.ascontiguousarray(xyz), np.ascontiguousarray(tri, dtype=np.int32)


def torus(R: float = 1.0, r: float = 0.3, n_tor: int = 256, n_pol: int = 64):
    """Torus of revolution about z: major radius R, minor radius r.

    n_tor x n_pol quads (toroidal x poloidal), each split along the
    (i, j) -> (i+1, j+1) diagonal; N = n_tor*n_pol, T = 2N.
    """
    i, j = np.meshgrid(np.arange(n_tor), np.arange(n_pol), indexing="ij")
    th = 2.0 * np.pi * i / n_tor
    ph = 2.0 * np.pi * j / n_pol
    rho = R + r * np.cos(ph)
    xyz = np.stack([rho * np.cos(th), rho * np.sin(th), r * np.sin(ph)], -1).reshape(-1, 3)

    def nid(a, b):
        return (a % n_tor) * n_pol + (b % n_pol)

    i = i.ravel(); j = j.ravel()
    p00, p10, p11, p01 = nid(i, j), nid(i + 1, j), nid(i + 1, j + 1), nid(i, j + 1)
    t = np.stack([np.stack([p00, p10, p11], 1), np.stack([p00, p11, p01], 1)], 1).reshape(-1, 3)
    # orient: outward = away from the tube centre line
    a, b, c = xyz[t[:, 0]], xyz[t[:, 1]], xyz[t[:, 2]]
    cen = (a + b + c) / 3.0
    ang = np.arctan2(cen[:, 1], cen[:, 0])
    core = np.stack([R * np.cos(ang), R * np.sin(ang), np.zeros_like(ang)], 1)
    nrm = np.cross(b - a, c - a)
    inward = np.einsum("ij,ij->i", nrm, cen - core) < 0
    t[inward] = t[inward][:, [0, 2, 1]]
    return np.ascontiguousarray(xyz, dtype=np.float64), np.ascontiguousarray(t, dtype=np.int32)
