"""The seeded mesh and right-hand-side generators (no operator arithmetic)."""
import numpy as np
import pytest

from workloads import cases, meshes, rhs


def _euler(tri):
    t = tri.astype(np.int64)
    V = np.unique(t).size
    e = np.sort(np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]]), axis=1)
    E = np.unique(e, axis=0).shape[0]
    return V - E + t.shape[0]


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_icosphere_counts_and_topology(level):
    xyz, tri = meshes.icosphere(level)
    assert xyz.shape == (10 * 4 ** level + 2, 3)
    assert tri.shape == (20 * 4 ** level, 3)
    assert tri.dtype == np.int32 and xyz.dtype == np.float64
    assert _euler(tri) == 2
    np.testing.assert_allclose(np.linalg.norm(xyz, axis=1), 1.0, atol=1e-15)


def test_icosphere_jitter_is_radial_and_bounded():
    a, ta = meshes.icosphere(3)
    b, tb = meshes.icosphere(3, 0.01, 0)
    assert np.array_equal(ta, tb)
    r = np.linalg.norm(b, axis=1)
    assert np.all(np.abs(r - 1.0) <= 0.01 + 1e-15)
    np.testing.assert_allclose(b / r[:, None], a, atol=1e-14)
    c, _ = meshes.icosphere(3, 0.01, 0)
    assert np.array_equal(b, c)                       # seeded


def test_outward_orientation():
    for xyz, tri in (meshes.icosphere(2), meshes.cuboid(4.0, 3.0, 2.0, 1.0), meshes.torus(1.0, 0.3, 16, 8)):
        a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
        vol = np.sum(np.einsum("ij,ij->i", a, np.cross(b, c))) / 6.0
        assert vol > 0


def test_film_counts():
    xyz, tri = meshes.cuboid(2000.0, 2000.0, 20.0, 5.0, 0.5, 0)
    assert xyz.shape[0] == 326402 and tri.shape[0] == 652800
    assert _euler(tri) == 2


def test_film_jitter_in_plane():
    g, _ = meshes.cuboid(40.0, 30.0, 10.0, 5.0)
    j, _ = meshes.cuboid(40.0, 30.0, 10.0, 5.0, 0.5, 0)
    d = j - g
    assert np.all(np.abs(d) <= 0.5)
    lim = np.array([40.0, 30.0, 10.0])
    on = (np.abs(g) < 1e-12) | (np.abs(g - lim) < 1e-12)
    assert np.all(d[on] == 0.0)                       # never moves off its face(s)
    corners = on.sum(axis=1) == 3
    assert corners.sum() == 8 and np.all(d[corners] == 0.0)


def test_torus_counts():
    xyz, tri = meshes.torus()
    assert xyz.shape == (16384, 3) and tri.shape == (32768, 3)
    assert _euler(tri) == 0


def test_rhs_generators():
    x = np.random.default_rng(3).normal(size=(50, 3))
    u = rhs.normal_rhs(50, 4, 0)
    assert u.shape == (4, 50)
    assert np.array_equal(u, np.random.default_rng(0).normal(size=(4, 50)))
    assert np.array_equal(rhs.z_rhs(x)[0], x[:, 2])
    f = rhs.smooth_fields(x * 100, 3)
    assert f.shape == (3, 50) and np.all(np.isfinite(f))
    req = rhs.poisson_requests(512, 200.0, 6)
    assert len(req) == 512
    t = np.array([r[0] for r in req])
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 0.005) < 0.001
    assert all(1 <= r[2] <= 16 and 0 <= r[1] < 6 for r in req)


def test_cases_sizes():
    assert cases.CASES["sphere_l4"].mesh.level == 4
    assert cases.CASES["sphere_l8"].nrhs == 16
    assert len(cases.SERVING_MESHES) == 6
