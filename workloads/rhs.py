"""Seeded right-hand sides (boundary traces u1) and request streams.

No operator arithmetic lives here: these only draw the inputs of the matvec.
Every array is (r, N) float64, one contiguous length-N vector per right-hand
side, in the mesh's own node order.
"""
from __future__ import annotations

import numpy as np

__all__ = ["normal_rhs", "z_rhs", "smooth_fields", "poisson_requests"]


def normal_rhs(n_nodes: int, r: int, seed: int = 0) -> np.ndarray:
    """r standard-normal vectors from numpy default_rng(seed).normal(size=(r, N))."""
    return np.random.default_rng(seed).normal(size=(r, n_nodes))


def z_rhs(xyz: np.ndarray) -> np.ndarray:
    """u1 = z: the boundary trace of the uniformly z-magnetised body (Ms = 1), shape (1, N)."""
    return np.ascontiguousarray(xyz[:, 2][None, :], dtype=np.float64)


def smooth_fields(xyz: np.ndarray, r: int = 4, n_terms: int = 16,
                  lam_min: float = 50.0, lam_max: float = 2000.0, seed0: int = 0) -> np.ndarray:
    """r smooth random fields f = sum_q a_q sin(2 pi d_q.x / lam_q + phi_q).

    Field p uses default_rng(seed0 + p): lam_q log-uniform on [lam_min, lam_max],
    d_q uniform on the unit sphere, phi_q ~ U[0, 2 pi), a_q ~ N(0, 1).
    """
    out = np.empty((r, xyz.shape[0]))
    for p in range(r):
        g = np.random.default_rng(seed0 + p)
        lam = np.exp(g.uniform(np.log(lam_min), np.log(lam_max), size=n_terms))
        d = g.normal(size=(n_terms, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        ph = g.uniform(0.0, 2.0 * np.pi, size=n_terms)
        a = g.normal(size=n_terms)
        arg = 2.0 * np.pi * (xyz @ d.T) / lam[None, :] + ph[None, :]
        out[p] = np.sin(arg) @ a
    return out


def poisson_requests(n_requests: int, rate_hz: float, n_meshes: int, max_rhs: int = 16, seed: int = 1):
    """A Poisson arrival stream: list of (arrival_s, mesh_index, n_rhs, rhs_seed).

    Exponential inter-arrival times with mean 1/rate_hz, mesh uniform over
    n_meshes, n_rhs uniform on {1..max_rhs}; all from default_rng(seed).  The
    right-hand sides of request q are drawn later from default_rng(1000 + q).
    """
    g = np.random.default_rng(seed)
    gaps = g.exponential(1.0 / rate_hz, size=n_requests)
    mesh = g.integers(0, n_meshes, size=n_requests)
    nr = g.integers(1, max_rhs + 1, size=n_requests)
    t = np.cumsum(gaps)
    return [(float(t[q]), int(mesh[q]), int(nr[q]), 1000 + q) for q in range(n_requests)]
