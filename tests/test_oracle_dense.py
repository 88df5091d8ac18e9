"""Pins for the dense collocation matrix M = K + D (Section 3, eqs. matrix_definition, denseMat)."""
import json
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import dense, energy, geometry
from workloads import meshes

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


@pytest.mark.parametrize("mesh", [
    lambda: meshes.icosphere(2),
    lambda: meshes.icosphere(3, 0.02, 5),
    lambda: meshes.cuboid(4.0, 3.0, 1.0, 0.5, 0.1, 2),
    lambda: meshes.torus(1.0, 0.3, 24, 10),
])
def test_constant_maps_to_minus_itself(mesh):
    xyz, tri = mesh()
    M = dense.dense_m(xyz, tri)
    np.testing.assert_allclose(M.sum(axis=1), GOLD["constant_row_sum"]["value"], rtol=0, atol=1e-13)


def test_incident_row_entries():
    xyz, tri = meshes.icosphere(2, 0.02, 1)
    K = dense.k_rows(xyz, tri, np.arange(xyz.shape[0]))
    assert np.all(np.diag(K) == 0.0)
    # every off-diagonal entry is a positive weight seen from the inside of a convex body? no:
    # entries are solid-angle-like and negative from the inner side
    off = K[~np.eye(K.shape[0], dtype=bool)]
    assert np.all(off <= 0.0)


def _k_entry_brute(xyz, tri, i, j):
    """K_ij by adaptive quadrature over the triangles of phi_j's support (i not a vertex)."""
    tot = 0.0
    for T in np.where(np.any(tri == j, axis=1))[0]:
        v = tri[T]
        if i in v:
            continue
        loc = int(np.where(v == j)[0][0])
        r1, r2, r3 = xyz[v[0]], xyz[v[1]], xyz[v[2]]
        e1, e2 = r2 - r1, r3 - r1
        cr = np.cross(e1, e2)
        n = cr / np.linalg.norm(cr)

        def f(vv, uu):
            y = r1 + uu * e1 + vv * e2
            phi = (1.0 - uu - vv, uu, vv)[loc]
            d = xyz[i] - y
            return phi * np.dot(n, d) / np.linalg.norm(d) ** 3

        val, _ = integrate.dblquad(f, 0, 1, 0, lambda uu: 1 - uu, epsabs=1e-13, epsrel=1e-11)
        tot += val * np.linalg.norm(cr) / (4 * np.pi)
    return tot


def test_entries_match_quadrature_of_definition():
    xyz, tri = meshes.icosphere(2, 0.02, 1)
    K = dense.k_rows(xyz, tri, [0, 17, 90])
    rng = np.random.default_rng(0)
    for q, i in enumerate([0, 17, 90]):
        for j in rng.choice(xyz.shape[0], 5, replace=False).tolist() + [int(tri[np.any(tri == i, 1)][0][1])]:
            if j == i:
                continue
            ref = _k_entry_brute(xyz, tri, i, j)
            assert abs(K[q, j] - ref) < 1e-10, (i, j, K[q, j], ref)


def test_sphere_uniform_magnetisation_converges():
    errs, eerr = [], []
    for L in (2, 3, 4):
        xyz, tri = meshes.icosphere(L)
        z = xyz[:, 2]
        if L < 4:
            u2 = dense.dense_m(xyz, tri) @ z
        else:
            u2 = np.concatenate([dense.apply_rows(xyz, tri, z[None], r)[0]
                                 for r in np.array_split(np.arange(xyz.shape[0]), 8)])
        exact = -(1.0 - GOLD["sphere_demag_factor"]["value"]) * z       # u2 = -2z/3
        errs.append(np.linalg.norm(u2 - exact) / np.linalg.norm(exact))
        vol = geometry.signed_volume(xyz, tri)
        e = energy.demag_energy_z(xyz, tri, u2)
        eerr.append(abs(e / (GOLD["sphere_energy_over_volume"]["value"] * vol) - 1.0))
    assert errs[0] < 0.012 and errs[0] > errs[1] > errs[2]
    assert errs[2] < 3e-3
    assert eerr[0] > eerr[1] > eerr[2] and eerr[2] < 2e-3


def test_half_identity_diagonal_is_worse_on_polyhedra():
    # replacing Psi/(4 pi) - 1 by the smooth value -1/2 spoils u1 = z at O(h)
    xyz, tri = meshes.icosphere(3)
    z = xyz[:, 2]
    K = dense.k_rows(xyz, tri, np.arange(xyz.shape[0]))
    exact = -2.0 * z / 3.0
    good = np.linalg.norm(K @ z + geometry.diagonal(xyz, tri) * z - exact)
    half = np.linalg.norm(K @ z - 0.5 * z - exact)
    assert half > 5 * good


def test_scale_rotation_permutation():
    xyz, tri = meshes.icosphere(2, 0.03, 2)
    M = dense.dense_m(xyz, tri)
    q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    np.testing.assert_allclose(dense.dense_m(3.7 * xyz @ q.T + 1.0, tri), M, atol=1e-13)
    p = np.random.default_rng(4).permutation(xyz.shape[0])
    inv = np.argsort(p)
    Mp = dense.dense_m(xyz[p], inv[tri].astype(np.int32))
    np.testing.assert_allclose(Mp, M[np.ix_(p, p)], atol=1e-14)


def test_torus_azimuthal_gives_zero_potential():
    # azimuthal M: M.n = 0 and div M = 0, so u1 = const solves the Neumann problem and u = 0
    xyz, tri = meshes.torus(1.0, 0.5, 32, 12)
    M = dense.dense_m(xyz, tri)
    u1 = np.full(xyz.shape[0], 0.7)
    np.testing.assert_allclose(M @ u1 + u1, 0.0, atol=1e-13)


def test_stored_dense_rows_are_the_oracles():
    # the 1000-row fixture of the 163842-node sphere: spot-check three rows
    # against a fresh evaluation (tests/golden/make_dense_rows.py wrote it)
    import os
    from workloads import cases, rhs
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sphere_l7_dense_rows.npz"))
    c = cases.CASES["sphere_l7"]
    xyz, tri = cases.mesh_of(c.mesh)
    rows = np.random.default_rng(2).choice(xyz.shape[0], 1000, replace=False)
    assert np.array_equal(g["rows"], rows)
    u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(xyz.shape[0], 8, 0)])
    pick = [0, 499, 999]
    fresh = dense.m_rows(xyz, tri, rows[pick]) @ u.T
    np.testing.assert_allclose(fresh.T, g["values"][:, pick], rtol=1e-12, atol=1e-14)
