"""The recompressed operator on the GPU (Section 4: the algebraic conversion
to an H2 matrix of adaptive rank) against the oracle's recompression of the
same interpolation matrix (oracle/recompress.py).

The ranks are integers decided by floating point: both sides take them from
FP64 singular values of the same weighted bases, computed without squaring,
and the tests check that they agree before comparing values.  FP64 to 1e-12,
FP32 to 1e-6 (relative l2 per right-hand side), as for the interpolation
matrix; and the recompressed product stays within its truncation error of
the interpolation product it came from."""
import numpy as np
import pytest

from oracle import h2, recompress
from workloads import meshes, rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6}


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1811_05731_amd import h2dlp
    return h2dlp


def run(op, u1, dtype=torch.float64):
    d1 = torch.tensor(np.atleast_2d(u1), dtype=dtype, device="cuda")
    d2 = torch.full_like(d1, float("nan"))
    op.apply(d1, d2)
    torch.cuda.synchronize()
    return d2.double().cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


MESHES = {
    "sphere": lambda: meshes.icosphere(3, 0.01, 4),
    "film": lambda: meshes.cuboid(200.0, 150.0, 20.0, 5.0, 0.5, 0),
    "torus": lambda: meshes.torus(1.0, 0.3, 64, 16),
}


@pytest.fixture(scope="module")
def oracles():
    cache = {}

    def get(name, order, leaf, eps, dmax=0):
        key = (name, order, leaf, eps, dmax)
        if key not in cache:
            xyz, tri = MESHES[name]()
            H = h2.H2Oracle(xyz, tri, order=order, leaf=leaf, eta=2.0, dense_far_max=dmax)
            R = recompress.Recompressed(H, eps)
            u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(xyz.shape[0], 3, 7)])
            cache[key] = (xyz, tri, H, R, u, R.apply(u), H.apply(u))
        return cache[key]
    return get


@pytest.mark.parametrize("name,order,leaf", [("sphere", 4, 16), ("sphere", 5, 32), ("film", 4, 32),
                                             ("torus", 3, 24)])
@pytest.mark.parametrize("eps", [1e-4, 1e-6])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_recompressed_matches_oracle(lib, oracles, name, order, leaf, eps, prec):
    xyz, tri, H, R, u, ref, ref_interp = oracles(name, order, leaf, eps)
    op = lib.Operator(xyz, tri, order=order, leaf=leaf, eta=2.0, precision=prec, recompress_eps=eps)
    st = op.stats
    assert (st.rank_sum_row, st.rank_sum_col) == (int(R.row["rank"].sum()), int(R.col["rank"].sum()))
    assert (st.rank_max_row, st.rank_max_col) == (int(R.row["rank"].max()), int(R.col["rank"].max()))
    assert st.coupling_entries == R.counts()["coupling_entries"]
    out = run(op, u)
    err = relerr(out, ref)
    print(f"recompressed {name} m={order} eps={eps:g} {prec}: vs oracle {err.max():.2e}, vs interpolation "
          f"{relerr(out, ref_interp).max():.2e}; ranks {st.rank_sum_row}/{st.n_clusters * st.k}")
    assert np.all(err <= TOL[prec]), err
    # the truncation error against the interpolation matrix, relative to K u (as in the oracle's pins)
    k_ref = ref_interp - H.D[None, :] * u
    assert np.all(relerr(out - H.D[None, :] * u, k_ref) <= 10 * eps + (3e-6 if prec == "fp32" else 0.0))


def test_recompressed_with_exact_small_blocks(lib, oracles):
    xyz, tri, H, R, u, ref, _ = oracles("sphere", 4, 16, 1e-6, 16 * 16)
    op = lib.Operator(xyz, tri, order=4, leaf=16, eta=2.0, precision="fp64", recompress_eps=1e-6,
                      dense_far_max=16 * 16)
    assert op.stats.n_far_dense == H.far_dense.shape[0] > 0
    assert np.all(relerr(run(op, u), ref) <= 1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_recompressed_columns_and_workspace(lib, oracles, prec):
    xyz, tri, H, R, _, _, _ = oracles("sphere", 4, 16, 1e-6)
    op = lib.Operator(xyz, tri, order=4, leaf=16, eta=2.0, precision=prec, recompress_eps=1e-6)
    u = rhs.normal_rhs(xyz.shape[0], 37, 5)              # three 16-column passes, ragged last
    full = run(op, u)
    assert np.all(relerr(full, R.apply(u)) <= TOL[prec])
    for q in (0, 15, 16, 36):
        assert np.array_equal(run(op, u[q])[0], full[q])
    assert np.array_equal(run(op, u), full)
    # the workspace shrinks with the ranks; a caller workspace of that size works
    _, wbytes = op.bytes()
    assert wbytes == op.stats.workspace_bytes
    plan = lib.plan(xyz, tri, order=4, leaf=16, eta=2.0, precision=prec, recompress_eps=1e-6)
    assert wbytes <= plan.stats.workspace_bytes
    ws = torch.empty(wbytes, dtype=torch.uint8, device="cuda")
    d1 = torch.tensor(u, device="cuda")
    d2 = torch.empty_like(d1)
    op.apply(d1, d2, workspace=ws)
    torch.cuda.synchronize()
    assert np.array_equal(d2.cpu().numpy(), full)


def test_recompressed_offload_roundtrip(lib, oracles):
    xyz, tri, _, _, u, ref, _ = oracles("sphere", 4, 16, 1e-4)
    op = lib.Operator(xyz, tri, order=4, leaf=16, eta=2.0, precision="fp32", recompress_eps=1e-4)
    before = run(op, u)
    op.offload()
    op.reload()
    assert np.array_equal(run(op, u), before)
