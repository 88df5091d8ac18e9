"""Full-size GPU checks in the launch configuration the benchmark times.

* Sampled parity: 16 right-hand sides that are unit vectors at seeded nodes.
  The oracle then needs only the clusters, blocks and bases those nodes touch,
  yet every output entry (all N rows of each column) is compared.
* Dense rows: at 163842 nodes, 1000 seeded rows of the exact dense matrix
  (Section 3), stored by tests/golden/make_dense_rows.py, bound the H2
  approximation error.
* Physics at 655362 nodes: u1 = z gives u2 ~ -2z/3 and the sphere's energy
  mu0 Ms^2 V/6 (Section 6.2); M 1 = -1 up to the far-field approximation.
"""
import os

import numpy as np
import pytest

from oracle import energy, geometry, h2
from workloads import cases, rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1811_05731_amd import h2dlp
    return h2dlp


def run(op, u1):
    d1 = torch.tensor(np.atleast_2d(u1), dtype=torch.float64, device="cuda")
    d2 = torch.full_like(d1, float("nan"))
    op.apply(d1, d2)
    torch.cuda.synchronize()
    return d2.cpu().numpy()


GOLDEN_ROWS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sphere_l7_dense_rows.npz")


def relerr(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def unit_columns(n, count, seed):
    cols = np.random.default_rng(seed).choice(n, count, replace=False)
    u = np.zeros((count, n))
    u[np.arange(count), cols] = 1.0
    return u


@pytest.fixture(scope="module")
def sphere_l7():
    c = cases.CASES["sphere_l7"]
    xyz, tri = cases.mesh_of(c.mesh)
    H = h2.H2Oracle(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, cache_coupling=False)
    u = unit_columns(xyz.shape[0], 16, 11)
    return c, xyz, tri, u, H.apply(u)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_sphere_l7_sampled_columns(lib, sphere_l7, prec, tol):
    c, xyz, tri, u, ref = sphere_l7
    op = lib.Operator(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, precision=prec)
    err = relerr(run(op, u), ref)
    assert np.all(err <= tol), err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sphere_l7_dense_rows(lib, sphere_l7, prec):
    # 1000 exact rows of M u1 (tests/golden/make_dense_rows.py, oracle only)
    c, xyz, tri, _, _ = sphere_l7
    g = np.load(GOLDEN_ROWS)
    rows, ref = g["rows"], g["values"]
    n = xyz.shape[0]
    assert int(g["n_nodes"]) == n
    u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(n, 8, 0)])
    op = lib.Operator(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, precision=prec)
    err = relerr(run(op, u)[:, rows], ref)
    print(f"{prec}: H2 vs 1000 dense rows, per column: {np.array2string(err, precision=2)}")
    # interpolation error of the H2 approximation at order 4, not arithmetic
    # (FP32 and FP64 agree to 3e-7): ~2.4e-4 for the smooth u1 = z and ~3e-5
    # for N(0,1) columns; the paper fixes no bound here
    assert err[0] <= 5e-4 and np.all(err[1:] <= 1e-4), err


@pytest.fixture(scope="module")
def sphere_l8():
    c = cases.CASES["sphere_l8"]
    xyz, tri = cases.mesh_of(c.mesh)
    return c, xyz, tri


def test_sphere_l8_sampled_columns_fp32(lib, sphere_l8):
    c, xyz, tri = sphere_l8
    H = h2.H2Oracle(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, cache_coupling=False)
    u = unit_columns(xyz.shape[0], 16, 12)
    ref = H.apply(u)
    op = lib.Operator(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, precision="fp32")
    err = relerr(run(op, u), ref)
    assert np.all(err <= 1e-6), err


def test_sphere_l8_uniform_magnetisation(lib, sphere_l8):
    c, xyz, tri = sphere_l8
    op = lib.Operator(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, precision="fp32")
    z = xyz[:, 2]
    out = run(op, np.vstack([z, np.ones_like(z)]))
    exact = -2.0 * z / 3.0
    assert np.linalg.norm(out[0] - exact) / np.linalg.norm(exact) < 1e-2
    vol = geometry.signed_volume(xyz, tri)
    e = energy.demag_energy_z(xyz, tri, out[0])
    assert abs(e / (vol / 6.0) - 1.0) < 1e-3
    assert np.max(np.abs(out[1] + 1.0)) < 2e-3


@pytest.fixture(scope="module")
def film():
    c = cases.CASES["film"]
    xyz, tri = cases.mesh_of(c.mesh)
    return c, xyz, tri


def test_film_sampled_columns_fp64(lib, film):
    c, xyz, tri = film
    H = h2.H2Oracle(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, cache_coupling=False)
    u = unit_columns(xyz.shape[0], 16, 13)
    ref = H.apply(u)
    op = lib.Operator(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, precision="fp64")
    err = relerr(run(op, u), ref)
    assert np.all(err <= 1e-12), err


def test_film_fp32_smooth_fields(lib, film):
    # FP32 against the FP64 path (itself the oracle's to 1e-12) on the four
    # smooth fields.  On the flat faces the far field of coplanar clusters is
    # a sum of large terms that cancel (the normal derivative of the kernel
    # taken through Chebyshev points across a box only alpha = 0.1 of its
    # length thick), so FP32 rounding is amplified: measured 4.5e-6, against
    # 2e-7 on the sphere
    c, xyz, tri = film
    u = rhs.smooth_fields(xyz, c.nrhs)
    outs = {}
    for prec in ("fp64", "fp32"):
        op = lib.Operator(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, precision=prec)
        outs[prec] = run(op, u)
        op.close()
    err = relerr(outs["fp32"], outs["fp64"])
    print(f"film fp32 vs fp64: {np.array2string(err, precision=2)}")
    assert np.all(err <= 1e-5), err


def test_unjittered_sphere_l8_energy(lib):
    # the same energy check on the level-8 sphere without jitter: the jittered
    # polyhedron is rough (jitter ~0.3 edge lengths), the smooth one is not
    xyz, tri = cases.mesh_of(cases.MeshSpec("icosphere", 8, 0.0, 0))
    c = cases.CASES["sphere_l8"]
    op = lib.Operator(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, precision="fp32", coupling="generated")
    out = run(op, xyz[:, 2])
    vol = geometry.signed_volume(xyz, tri)
    e = energy.demag_energy_z(xyz, tri, out[0])
    print(f"unjittered L8: E/(V/6) - 1 = {e / (vol / 6.0) - 1.0:.3e}")
    assert abs(e / (vol / 6.0) - 1.0) < 1e-3


def test_sphere_l8_bench_configuration(lib, sphere_l8):
    # the configuration bench.py times: generated coupling, admissible blocks
    # with |t||s| <= k^2/2 kept exact, FP32; sampled unit columns against the
    # oracle built with the same block choice
    c, xyz, tri = sphere_l8
    dmax = (c.order ** 3) ** 2 // 2
    H = h2.H2Oracle(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, cache_coupling=False, dense_far_max=dmax)
    u = unit_columns(xyz.shape[0], 16, 14)
    ref = H.apply(u)
    op = lib.Operator(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, precision="fp32", coupling="generated",
                      dense_far_max=dmax)
    assert op.stats.n_far_dense == H.counts()["far_dense"]
    err = relerr(run(op, u), ref)
    print(f"bench configuration vs oracle: {np.array2string(err, precision=2)}")
    assert np.all(err <= 1e-6), err
