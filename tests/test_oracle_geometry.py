"""Pins for the oracle's solid angle Psi and mesh checks (closed forms, tests/golden)."""
import json
import os

import numpy as np
import pytest

from oracle import geometry, lindholm
from workloads import meshes

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def test_icosahedron_vertex_solid_angle():
    xyz, tri = meshes.icosahedron()
    psi = geometry.node_solid_angles(xyz, tri)
    np.testing.assert_allclose(psi, GOLD["icosahedron_vertex_solid_angle"]["value"], rtol=0, atol=1e-13)


def test_cube_corner_edge_face():
    xyz, tri = meshes.cuboid(3.0, 3.0, 3.0, 1.0)
    psi = geometry.node_solid_angles(xyz, tri)
    g = np.round(xyz).astype(int)
    on = ((g == 0) | (g == 3)).sum(axis=1)
    np.testing.assert_allclose(psi[on == 3], GOLD["cube_corner_solid_angle"]["value"], atol=1e-13)
    np.testing.assert_allclose(psi[on == 2], GOLD["cube_edge_solid_angle"]["value"], atol=1e-13)
    np.testing.assert_allclose(psi[on == 1], GOLD["flat_solid_angle"]["value"], atol=1e-13)


@pytest.mark.parametrize("mesh", [
    lambda: meshes.icosphere(2, 0.03, 0),
    lambda: meshes.cuboid(3.0, 2.0, 1.0, 0.5, 0.1, 1),
    lambda: meshes.torus(1.0, 0.3, 32, 12),               # saddle-shaped, non-convex vertices
])
def test_psi_equals_solid_angle_of_the_rest_of_the_surface(mesh):
    # Gauss: seen from a surface point, the triangles not touching it subtend -Psi
    # (the VO-S solid angle is negative from the inner side); independent of the dihedral sum
    xyz, tri = mesh()
    psi = geometry.node_solid_angles(xyz, tri)
    r1, r2, r3 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    for i in np.random.default_rng(0).choice(xyz.shape[0], 25, replace=False):
        keep = ~np.any(tri == i, axis=1)
        om = lindholm.solid_angle(xyz[i][None], r1[keep], r2[keep], r3[keep]).sum()
        assert abs(-om - psi[i]) < 1e-11


def test_psi_is_rotation_and_scale_invariant():
    xyz, tri = meshes.icosphere(2, 0.03, 4)
    q, _ = np.linalg.qr(np.random.default_rng(1).normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    a = geometry.node_solid_angles(xyz, tri)
    b = geometry.node_solid_angles(7.5 * xyz @ q.T, tri)
    np.testing.assert_allclose(a, b, atol=1e-12)


def test_check_mesh_accepts_and_rejects():
    xyz, tri = meshes.icosphere(1)
    geometry.check_mesh(xyz, tri)
    bad = tri.copy(); bad[0] = bad[0][[0, 2, 1]]
    with pytest.raises(ValueError):
        geometry.check_mesh(xyz, bad)                              # one flipped triangle
    with pytest.raises(ValueError):
        geometry.check_mesh(xyz, tri[1:])                          # open surface
    with pytest.raises(ValueError):
        geometry.check_mesh(xyz, tri[:, [0, 2, 1]])                # inward
    bad = tri.copy(); bad[3, 1] = bad[3, 0]
    with pytest.raises(ValueError):
        geometry.check_mesh(xyz, bad)                              # degenerate
    bad = tri.copy(); bad[0, 0] = xyz.shape[0]
    with pytest.raises(ValueError):
        geometry.check_mesh(xyz, bad)                              # out of range


def test_diagonal_smooth_limit():
    # on finer spheres Psi -> 2 pi, so D -> -1/2 (the smooth-surface value)
    devs = []
    for L in (2, 3, 4):
        xyz, tri = meshes.icosphere(L)
        devs.append(np.max(np.abs(geometry.diagonal(xyz, tri) + 0.5)))
    assert devs[0] > devs[1] > devs[2]
