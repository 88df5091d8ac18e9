"""GPU parity: the HIP library against the FP64 oracle on the same seeded inputs.

Tolerances (relative l2 per right-hand side, against the oracle's H2 product
unless stated): FP64 path 1e-12; FP32 path 1e-6 (FP32 storage of 24-bit
mantissa values and FP32 accumulation over a few hundred terms give ~1e-7);
BF16X3 path 5e-6: a coupling entry split into two bfloat16 terms keeps about
16 bits (|S - hi - lo| <= 2^-16 |S|), the same holds for xhat, and the dropped
lo*lo term is of that size too, so each far-field term carries ~1e-5 relative
error; measured 1.1e-6 .. 2.5e-6 on these cases, above the 1e-6 the FP32 path
meets.  BF16X6 1e-6: three-term splits leave ~2^-25 of each factor and the
dropped products are of that order too, so FP32 accumulation dominates as on
the FP32 path.
"""
import numpy as np
import pytest

from oracle import dense, geometry, h2
from workloads import meshes, rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 5e-6, "bf16x6": 1e-6}


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1811_05731_amd import h2dlp
    return h2dlp


def run(op, u1, dtype=torch.float64, nrhs=None):
    d_u1 = torch.tensor(np.atleast_2d(u1), dtype=dtype, device="cuda")
    d_u2 = torch.full_like(d_u1, float("nan"))
    op.apply(d_u1, d_u2, nrhs=nrhs)
    torch.cuda.synchronize()
    return d_u2.double().cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


@pytest.fixture(scope="module")
def sphere_l4():
    xyz, tri = meshes.icosphere(4, 0.01, 0)
    H = h2.H2Oracle(xyz, tri, order=4, leaf=32, eta=2.0)
    u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(xyz.shape[0], 1, 0)])
    return xyz, tri, H, u, H.apply(u)


def test_diagonal_matches_oracle(lib):
    xyz, tri = meshes.icosphere(3, 0.02, 1)
    op = lib.Operator(xyz, tri, order=3, leaf=16)
    np.testing.assert_allclose(op.export_diagonal(), geometry.diagonal(xyz, tri), rtol=0, atol=1e-14)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_near_field_only_single_leaf(lib, prec):
    # 42 nodes <= leaf: the root is one leaf, M is one exact near block plus D
    xyz, tri = meshes.icosphere(1, 0.05, 3)
    op = lib.Operator(xyz, tri, order=2, leaf=64, precision=prec)
    assert op.stats.n_far == 0 and op.stats.n_near == 1
    u = rhs.normal_rhs(xyz.shape[0], 3, 1)
    ref = u @ dense.dense_m(xyz, tri).T
    assert np.all(relerr(run(op, u), ref) <= TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_all_near_ragged_leaves(lib, prec):
    # eta tiny: nothing admissible, M = all near blocks; 162 nodes in ragged leaves
    xyz, tri = meshes.icosphere(2, 0.03, 2)
    op = lib.Operator(xyz, tri, order=2, leaf=24, eta=1e-3, precision=prec)
    assert op.stats.n_far == 0
    u = rhs.normal_rhs(xyz.shape[0], 4, 2)
    ref = u @ dense.dense_m(xyz, tri).T
    assert np.all(relerr(run(op, u), ref) <= TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_sphere_l4_matches_oracle(lib, sphere_l4, prec):
    xyz, tri, H, u, ref = sphere_l4
    op = lib.Operator(xyz, tri, order=4, leaf=32, eta=2.0, precision=prec)
    out = run(op, u)
    err = relerr(out, ref)
    assert np.all(err <= TOL[prec]), err
    # and against the dense matrix: the H2 approximation error at order 4
    M = dense.dense_m(xyz, tri)
    assert np.all(relerr(out, u @ M.T) <= 1e-4)


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5, 6, 7, 8])
def test_every_order_matches_oracle(lib, order):
    xyz, tri = meshes.icosphere(3, 0.01, 4)
    H = h2.H2Oracle(xyz, tri, order=order, leaf=16, eta=2.0)
    u = rhs.normal_rhs(xyz.shape[0], 3, order)
    ref = H.apply(u)
    op = lib.Operator(xyz, tri, order=order, leaf=16, eta=2.0)
    assert op.stats.n_far > 0
    assert np.all(relerr(run(op, u), ref) <= TOL["fp64"])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_multi_rhs_columns_are_independent(lib, sphere_l4, prec):
    xyz, tri, H, _, _ = sphere_l4
    op = lib.Operator(xyz, tri, order=4, leaf=32, eta=2.0, precision=prec)
    u = rhs.normal_rhs(xyz.shape[0], 37, 5)            # three 16-column passes, ragged last
    ref = H.apply(u)
    full = run(op, u)
    assert np.all(relerr(full, ref) <= TOL[prec])
    for q in (0, 15, 16, 36):
        single = run(op, u[q])[0]
        assert np.array_equal(single, full[q])          # same arithmetic whatever the batch
    assert np.array_equal(run(op, u), full)              # bitwise reproducible


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_split_bf16_orders(lib, order, prec):
    xyz, tri = meshes.icosphere(3, 0.01, 4)
    H = h2.H2Oracle(xyz, tri, order=order, leaf=16, eta=2.0)
    u = rhs.normal_rhs(xyz.shape[0], 3, order)
    ref = H.apply(u)
    op = lib.Operator(xyz, tri, order=order, leaf=16, eta=2.0, precision=prec)
    err = relerr(run(op, u), ref)
    print(f"{prec} order {order}: max rel err {err.max():.3e}")
    assert np.all(err <= TOL[prec]), err


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
def test_split_bf16_rejects_high_order(lib, prec):
    xyz, tri = meshes.icosphere(2)
    with pytest.raises(lib.H2dlpError) as e:
        lib.Operator(xyz, tri, order=6, leaf=16, precision=prec)
    assert e.value.code == lib.ENOTSUP


def test_fp32_io(lib, sphere_l4):
    xyz, tri, H, u, ref = sphere_l4
    op = lib.Operator(xyz, tri, order=4, leaf=32, eta=2.0, precision="fp32")
    out = run(op, u.astype(np.float32), dtype=torch.float32)
    assert np.all(relerr(out, ref) <= 1e-6)


@pytest.mark.parametrize("mesh,order", [
    (lambda: meshes.cuboid(200.0, 150.0, 20.0, 5.0, 0.5, 0), 4),
    (lambda: meshes.torus(1.0, 0.3, 64, 16), 3),
])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_other_geometries(lib, mesh, order, prec):
    xyz, tri = mesh()
    H = h2.H2Oracle(xyz, tri, order=order, leaf=48, eta=2.0)
    u = np.vstack([np.ones(xyz.shape[0]), rhs.normal_rhs(xyz.shape[0], 2, 7)])
    ref = H.apply(u)
    op = lib.Operator(xyz, tri, order=order, leaf=48, eta=2.0, precision=prec)
    assert np.all(relerr(run(op, u), ref) <= TOL[prec])


def test_workspace_and_streams(lib, sphere_l4):
    xyz, tri, H, u, ref = sphere_l4
    op = lib.Operator(xyz, tri, order=4, leaf=32, eta=2.0)
    _, wbytes = op.bytes()
    ws = [torch.empty(wbytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
    streams = [torch.cuda.Stream() for _ in range(2)]
    d_u1 = torch.tensor(u, device="cuda")
    outs = [torch.empty_like(d_u1) for _ in range(2)]
    torch.cuda.synchronize()
    for q in range(2):
        op.apply(d_u1, outs[q], stream=streams[q], workspace=ws[q])
    torch.cuda.synchronize()
    for q in range(2):
        assert np.all(relerr(outs[q].cpu().numpy(), ref) <= TOL["fp64"])
    small = torch.empty(wbytes - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(lib.H2dlpError) as e:
        op.apply(d_u1, outs[0], workspace=small)
    assert e.value.code == lib.ENOMEM


# generated coupling: S_ts computed inside the apply from the box geometry
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_generated_coupling_every_order(lib, order, prec):
    xyz, tri = meshes.icosphere(3, 0.01, 4)
    H = h2.H2Oracle(xyz, tri, order=order, leaf=16, eta=2.0)
    u = rhs.normal_rhs(xyz.shape[0], 3, order)
    ref = H.apply(u)
    op = lib.Operator(xyz, tri, order=order, leaf=16, eta=2.0, precision=prec, coupling="generated")
    assert op.stats.n_far > 0 and op.stats.bytes_coupling == 0
    err = relerr(run(op, u), ref)
    print(f"generated {prec} order {order}: max rel err {err.max():.3e}")
    assert np.all(err <= TOL[prec]), err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_generated_coupling_columns(lib, sphere_l4, prec):
    xyz, tri, H, _, _ = sphere_l4
    op = lib.Operator(xyz, tri, order=4, leaf=32, eta=2.0, precision=prec, coupling="generated")
    u = rhs.normal_rhs(xyz.shape[0], 37, 5)
    ref = H.apply(u)
    full = run(op, u)
    assert np.all(relerr(full, ref) <= TOL[prec])
    for q in (0, 15, 16, 36):
        assert np.array_equal(run(op, u[q])[0], full[q])
    assert np.array_equal(run(op, u), full)


@pytest.mark.parametrize("mesh,order", [
    (lambda: meshes.cuboid(200.0, 150.0, 20.0, 5.0, 0.5, 0), 4),
    (lambda: meshes.torus(1.0, 0.3, 64, 16), 3),
])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_generated_coupling_other_geometries(lib, mesh, order, prec):
    xyz, tri = mesh()
    H = h2.H2Oracle(xyz, tri, order=order, leaf=48, eta=2.0)
    u = np.vstack([np.ones(xyz.shape[0]), rhs.normal_rhs(xyz.shape[0], 2, 7)])
    ref = H.apply(u)
    op = lib.Operator(xyz, tri, order=order, leaf=48, eta=2.0, precision=prec, coupling="generated")
    assert np.all(relerr(run(op, u), ref) <= TOL[prec])


# admissible blocks kept as exact entries (dense_far_max)
@pytest.mark.parametrize("coupling", ["stored", "generated"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dense_far_blocks_match_oracle(lib, sphere_l4, prec, coupling):
    xyz, tri, H_plain, u, ref_plain = sphere_l4
    H = h2.H2Oracle(xyz, tri, order=4, leaf=32, eta=2.0, dense_far_max=4096)
    ref = H.apply(u)
    op = lib.Operator(xyz, tri, order=4, leaf=32, eta=2.0, precision=prec, coupling=coupling, dense_far_max=4096)
    assert op.stats.n_far_dense == H.counts()["far_dense"] > 0
    out = run(op, u)
    assert np.all(relerr(out, ref) <= TOL[prec])
    M = dense.dense_m(xyz, tri)
    assert np.all(relerr(out, u @ M.T) < relerr(ref_plain, u @ M.T))   # closer to the exact operator


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_every_block_dense_is_the_dense_matrix(lib, prec):
    xyz, tri = meshes.icosphere(3, 0.01, 5)
    op = lib.Operator(xyz, tri, order=3, leaf=16, eta=2.0, precision=prec, dense_far_max=xyz.shape[0] ** 2)
    assert op.stats.n_far == 0 and op.stats.n_far_dense > 0
    u = rhs.normal_rhs(xyz.shape[0], 5, 9)
    assert np.all(relerr(run(op, u), u @ dense.dense_m(xyz, tri).T) <= TOL[prec])
