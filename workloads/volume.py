"""Seeded synthetic tetrahedral volume meshes and magnetisations.

No part of the method's arithmetic lives here: the generators only produce
node coordinates (float64, N x 3), tetrahedra (int32, T x 4, 0-based, positive
orientation: (b - a) . ((c - a) x (d - a)) > 0) and per-tetrahedron
magnetisations (float64, T x 3).  They stand in for the paper's volume meshes
of its test bodies (Section 5: a rectangular prism among them); both the
oracle and the GPU library consume them.
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = ["box_tets", "uniform_m", "vortex_m"]

# the six tetrahedra of a unit cube along its main diagonal (corner bits x, y, z):
# the paths 000 -> e_a -> e_a + e_b -> 111 over the orders (a, b, c) of the axes.
# Every cube uses the same diagonal direction, so neighbouring cubes share
# their face triangulations and the mesh is conforming.
_KUHN = []
for order in itertools.permutations(range(3)):
    corner, path = [0, 0, 0], [0]
    for axis in order:
        corner[axis] = 1
        path.append(corner[0] + 2 * corner[1] + 4 * corner[2])
    _KUHN.append(path)


def box_tets(lx: float, ly: float, lz: float, nx: int, ny: int, nz: int, jitter: float = 0.0, seed: int = 0):
    """The box [0, lx] x [0, ly] x [0, lz] cut into nx x ny x nz cells of 6 tetrahedra each.

    Nodes are numbered x fastest.  jitter > 0 moves every interior node by a
    seeded uniform offset of up to jitter times the cell size along each axis
    (below 0.25 no tetrahedron turns over); boundary nodes stay on the box.
    """
    if min(nx, ny, nz) < 1:
        raise ValueError("at least one cell per axis")
    gx, gy, gz = np.linspace(0.0, lx, nx + 1), np.linspace(0.0, ly, ny + 1), np.linspace(0.0, lz, nz + 1)
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    if jitter > 0.0:
        if jitter >= 0.25:
            raise ValueError("jitter must stay below 0.25 of a cell")
        rng = np.random.default_rng(seed)
        h = np.array([lx / nx, ly / ny, lz / nz])
        ii = np.arange(xyz.shape[0])
        i, j, k = ii % (nx + 1), (ii // (nx + 1)) % (ny + 1), ii // ((nx + 1) * (ny + 1))
        inner = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
        xyz[inner] += rng.uniform(-jitter, jitter, size=(int(inner.sum()), 3)) * h
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = (ci + (nx + 1) * (cj + (ny + 1) * ck)).ravel()
    offs = np.array([dx + (nx + 1) * (dy + (ny + 1) * dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)])
    tets = np.concatenate([base[:, None] + offs[np.array(p)][None, :] for p in _KUHN], axis=0).astype(np.int32)
    a, b, c, d = (xyz[tets[:, q]] for q in range(4))
    vol6 = np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a))
    flip = vol6 < 0
    tets[flip] = tets[flip][:, [0, 2, 1, 3]]
    return xyz, tets


def uniform_m(n_tets: int, direction=(0.0, 0.0, 1.0)) -> np.ndarray:
    """The same unit magnetisation in every tetrahedron."""
    d = np.asarray(direction, dtype=np.float64)
    return np.tile(d / np.linalg.norm(d), (n_tets, 1))


def vortex_m(xyz: np.ndarray, tets: np.ndarray, center=None, core: float = 0.1, seed: int = 0) -> np.ndarray:
    """A unit vortex magnetisation about the z axis through `center` (default: the
    bounding-box centre), out of plane within `core` of the axis, with a seeded
    1 % random tilt per tetrahedron, evaluated at the tetrahedra's centroids."""
    cen = xyz[tets].mean(axis=1)
    c = (xyz.min(axis=0) + xyz.max(axis=0)) / 2.0 if center is None else np.asarray(center, dtype=np.float64)
    d = cen - c
    r = np.hypot(d[:, 0], d[:, 1])
    mz = np.exp(-(r / core) ** 2)
    inplane = np.sqrt(np.maximum(0.0, 1.0 - mz ** 2))
    safe = np.where(r > 0.0, r, 1.0)
    m = np.stack([-d[:, 1] / safe * inplane, d[:, 0] / safe * inplane, mz], axis=1)
    m += 0.01 * np.random.default_rng(seed).normal(size=m.shape)
    return m / np.linalg.norm(m, axis=1, keepdims=True)
