"""Pins of the FEM oracle (oracle/fem.py; Section 2 of the paper, the solves
either side of the boundary operator).  Each function is checked against what
the mathematics fixes: P1 interpolation identities, exactness of the P1
solution for linear potentials, the divergence theorem on the extracted
surface, and the energy of a uniformly magnetised cube, mu0 Ms^2 V / 6 (its
demagnetising factors are 1/3 by symmetry), approached under refinement."""
import numpy as np
import pytest

from oracle import dense, fem
from workloads import volume


def dense_op(x, t, u):
    return dense.dense_m(x, t) @ u


@pytest.fixture(scope="module")
def box():
    return volume.box_tets(1.0, 2.0, 0.5, 3, 5, 2, jitter=0.2, seed=3)


def test_element_geometry_is_the_p1_basis(box):
    xyz, tets = box
    vol, g = fem.element_geometry(xyz, tets)
    x = xyz[tets]
    # grad phi_a . (x_b - x_0) = delta_ab - delta_a0: each hat function is 1 at its vertex, 0 at the others
    d = x - x[:, :1]
    lam = np.einsum("tad,tbd->tab", g, d)
    expect = np.eye(4)[None] - np.eye(4)[None][:, :, :1]
    assert np.allclose(lam, expect, atol=1e-12)
    triple = np.einsum("ij,ij->i", x[:, 1] - x[:, 0], np.cross(x[:, 2] - x[:, 0], x[:, 3] - x[:, 0])) / 6.0
    assert np.allclose(vol, np.abs(triple)) and np.all(triple > 0)      # the generator orients positively
    assert abs(vol.sum() - 1.0) < 1e-12                                  # the box volume


def test_stiffness_and_right_side(box):
    xyz, tets = box
    A = fem.stiffness(xyz, tets)
    assert abs(A - A.T).max() < 1e-14
    assert np.abs(A @ np.ones(len(xyz))).max() < 1e-12                  # constants are in the kernel
    c = np.array([0.3, -1.1, 2.0])
    lin = xyz @ c
    nodes, _ = fem.boundary_surface(tets, xyz)
    inner = np.setdiff1d(np.arange(len(xyz)), nodes)
    assert np.abs((A @ lin)[inner]).max() < 1e-12                       # linear functions are harmonic
    m = volume.uniform_m(len(tets), c)
    b = fem.neumann_rhs(xyz, tets, m)
    assert abs(b.sum()) < 1e-13
    # uniform M: int M . grad phi_i = int grad(M.x) . grad phi_i
    assert np.allclose(b, A @ (xyz @ m[0]), atol=1e-13)
    w = np.linalg.eigvalsh(A.toarray())
    assert w[0] > -1e-12 and w[1] > 1e-6                                 # semidefinite, one-dimensional kernel


def test_boundary_surface_is_closed_and_outward():
    xyz, tets = volume.box_tets(2.0, 1.0, 1.5, 4, 3, 5, jitter=0.15, seed=1)
    nodes, tri = fem.boundary_surface(tets, xyz)
    nx, ny, nz = 4, 3, 5
    assert len(nodes) == (nx + 1) * (ny + 1) * (nz + 1) - (nx - 1) * (ny - 1) * (nz - 1)
    s = xyz[nodes]
    a, b, c = s[tri[:, 0]], s[tri[:, 1]], s[tri[:, 2]]
    # divergence theorem: the volume is (1/6) sum a . (b x c) over outward triangles
    assert abs(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0 - 3.0) < 1e-12
    # every directed edge appears once and its reverse once (closed, consistently oriented)
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    fwd = set(map(tuple, e.tolist()))
    assert len(fwd) == len(e) and all((j, i) in fwd for i, j in fwd)


def test_linear_potentials_are_reproduced(box):
    xyz, tets = box
    A = fem.stiffness(xyz, tets)
    mdir = np.array([0.2, 0.5, -0.8])
    m = volume.uniform_m(len(tets), mdir)
    u1 = fem.solve_neumann(A, fem.neumann_rhs(xyz, tets, m))
    lin = xyz @ m[0]
    assert np.abs(u1 - (lin - lin.mean())).max() < 1e-11               # du1/dn = M.n, div M = 0: u1 = M.x
    nodes, _ = fem.boundary_surface(tets, xyz)
    c = np.array([1.0, -2.0, 0.5])
    u = fem.solve_dirichlet(A, nodes, xyz[nodes] @ c + 4.0)
    assert np.abs(u - (xyz @ c + 4.0)).max() < 1e-11
    assert np.allclose(fem.field(xyz, tets, xyz @ c), -c[None, :], atol=1e-12)


def test_uniformly_magnetised_cube_energy():
    # N = 1/3 for a cube: E = V / 6 (mu0 = Ms = 1); the P1 error falls with refinement
    errs = []
    for n in (4, 6, 8):
        xyz, tets = volume.box_tets(1.0, 1.0, 1.0, n, n, n)
        es = [fem.demag(xyz, tets, volume.uniform_m(len(tets), d), dense_op)["energy"]
              for d in ((1, 0, 0), (0, 0, 1))]
        assert abs(es[0] - es[1]) < 1e-9 * es[0]
        errs.append(abs(es[1] * 6.0 - 1.0))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.025, errs


def test_trace_of_the_demagnetising_tensor():
    # N_xx + N_yy + N_zz = 1 for any body: the energies of the three axis
    # magnetisations add up to V / 2, up to the discretisation error
    errs = []
    for n in (1, 2):
        xyz, tets = volume.box_tets(2.0, 1.0, 0.5, 8 * n, 4 * n, 2 * n)
        es = [fem.demag(xyz, tets, volume.uniform_m(len(tets), d), dense_op)["energy"]
              for d in ((1, 0, 0), (0, 1, 0), (0, 0, 1))]
        assert es[0] < es[1] < es[2]                                      # the thinnest axis has the largest factor
        errs.append(abs(2.0 * sum(es) / 1.0 - 1.0))                       # V = 1
    assert errs[1] < errs[0] / 2 and errs[1] < 0.025, errs


def test_demag_pieces_fit_together(box):
    xyz, tets = box
    m = volume.vortex_m(xyz, tets, core=0.3, seed=2)
    r = fem.demag(xyz, tets, m, dense_op)
    assert abs(r["u1"].sum()) < 1e-10
    nodes, tri = r["nodes"], r["tri"]
    assert np.allclose(r["u2"][nodes], dense.dense_m(xyz[nodes], tri) @ r["u1"][nodes])
    A = fem.stiffness(xyz, tets)
    inner = np.setdiff1d(np.arange(len(xyz)), nodes)
    assert np.abs((A @ r["u2"])[inner]).max() < 1e-10
    assert np.allclose(r["h"], fem.field(xyz, tets, r["u1"] + r["u2"]))
