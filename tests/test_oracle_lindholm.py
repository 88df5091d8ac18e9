"""Pins for the oracle's closed-form triangle integrals (re-derived; the paper only cites them).

Each check compares against something other than the formula itself: adaptive
numerical integration (scipy), Gauss's theorem, and the partition of unity of
the hat functions.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import lindholm
from workloads import meshes

TRI = np.array([[0.1, -0.2, 0.05], [1.3, 0.1, -0.1], [0.2, 0.9, 0.3]])


def _brute(x, r1, r2, r3, a):
    """(1/4pi) int_T phi_a(y) n.(x - y)/|x - y|^3 dS by adaptive 2D quadrature."""
    e1, e2 = r2 - r1, r3 - r1
    cr = np.cross(e1, e2)
    n = cr / np.linalg.norm(cr)
    jac = np.linalg.norm(cr)

    def f(v, u):
        y = r1 + u * e1 + v * e2
        phi = (1.0 - u - v, u, v)[a]
        d = x - y
        return phi * np.dot(n, d) / np.linalg.norm(d) ** 3 * jac / (4 * np.pi)

    val, _ = integrate.dblquad(f, 0.0, 1.0, 0.0, lambda u: 1.0 - u, epsabs=1e-13, epsrel=1e-11)
    return val


@pytest.mark.parametrize("x", [
    [0.4, 0.3, 0.8],        # above the interior
    [0.5, 0.2, -0.5],       # below
    [3.0, -2.0, 1.5],       # far
    [1.5, 1.2, 0.2],        # beside, near the plane
    [0.5, 0.3, 0.2],        # close above the interior
])
def test_weights_match_adaptive_quadrature(x):
    x = np.array(x)
    L = lindholm.weights(x[None], TRI[0][None], TRI[1][None], TRI[2][None])[0]
    for a in range(3):
        ref = _brute(x, TRI[0], TRI[1], TRI[2], a)
        assert abs(L[a] - ref) <= 1e-9 * max(1.0, abs(ref)), (a, L[a], ref)


def test_partition_of_unity():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(200, 3)) * 2.0
    L = lindholm.weights(x, TRI[0], TRI[1], TRI[2])
    om = lindholm.solid_angle(x, TRI[0], TRI[1], TRI[2])
    np.testing.assert_allclose(L.sum(axis=1), om / (4 * np.pi), atol=1e-15)


def test_solid_angle_matches_quadrature_and_sign():
    for x in ([0.4, 0.3, 0.9], [0.4, 0.3, -0.9], [2.0, 2.0, 0.4]):
        x = np.array(x)
        om = lindholm.solid_angle(x, *TRI)
        ref = 4 * np.pi * sum(_brute(x, *TRI, a) for a in range(3))
        assert abs(om - ref) < 1e-9
    n = np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0])
    c = TRI.mean(axis=0)
    assert lindholm.solid_angle(c + 0.1 * n, *TRI) > 0          # outer side positive
    assert lindholm.solid_angle(c - 0.1 * n, *TRI) < 0


def test_gauss_theorem_closed_mesh():
    xyz, tri = meshes.icosphere(2, 0.02, 1)
    r1, r2, r3 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    for p, expect in (([0.1, -0.2, 0.3], -4 * np.pi), ([0.0, 0.0, 0.0], -4 * np.pi),
                      ([1.5, 0.2, 0.1], 0.0), ([0.0, 3.0, -1.0], 0.0)):
        om = lindholm.solid_angle(np.array(p)[None], r1, r2, r3).sum()
        assert abs(om - expect) < 1e-12


def test_coplanar_point_gives_zero():
    x = np.array([2.0, 2.0, 0.0])
    flat = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0]])
    L = lindholm.weights(x[None], flat[0][None], flat[1][None], flat[2][None])[0]
    assert np.all(np.abs(L) == 0.0)


def test_edge_potential_form():
    # P_b = int_edge dl/|x - y|: check the log form used inside weights against quad
    x = np.array([0.3, 0.7, 0.4])
    a, b = TRI[0], TRI[1]
    s = np.linalg.norm(b - a)
    ra, rb = np.linalg.norm(x - a), np.linalg.norm(x - b)
    closed = np.log1p(2 * s / (ra + rb - s))
    ref, _ = integrate.quad(lambda t: s / np.linalg.norm(x - (a + t * (b - a))), 0, 1, epsabs=1e-14)
    assert abs(closed - ref) < 1e-12
