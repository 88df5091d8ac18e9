"""The allocation-free apply (h2dlp_apply_noalloc, workspace in the library's
device array) against h2dlp_apply_ex on the same operator: the same kernels,
so the same bits, on two calls in a row, the second with a smaller input."""
import numpy as np
import pytest

from oracle import h2
from workloads import meshes, rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1811_05731_amd import h2dlp
    return h2dlp


def both(op, u, stream=None):
    """(apply_ex result, apply_noalloc result) for the host array u."""
    d1 = torch.tensor(u, device="cuda")
    ex = torch.full_like(d1, float("nan"))
    na = torch.full_like(d1, float("nan"))
    op.apply(d1, ex, stream=stream)
    torch.cuda.synchronize()
    op.apply_noalloc(d1, na, stream=stream)
    torch.cuda.synchronize()
    return ex.cpu().numpy(), na.cpu().numpy()


def test_noalloc_equals_apply_ex_two_calls(lib):
    # first call: 10242 nodes, FP32, 20 columns (two 16-column passes)
    xyz, tri = meshes.icosphere(5, 0.01, 0)
    big = lib.Operator(xyz, tri, order=4, leaf=32, eta=2.0, precision="fp32", coupling="generated")
    assert big.stats.workspace_bytes <= lib.NOALLOC_SCRATCH_BYTES
    ex, na = both(big, rhs.normal_rhs(xyz.shape[0], 20, 3))
    assert np.array_equal(ex, na)
    # second call, smaller: 642 nodes, FP64, 3 columns, on a side stream; the
    # scratch still holds the first call's values
    xyz2, tri2 = meshes.icosphere(3, 0.01, 1)
    small = lib.Operator(xyz2, tri2, order=3, leaf=16, eta=2.0, precision="fp64")
    assert small.stats.workspace_bytes < big.stats.workspace_bytes
    u = rhs.normal_rhs(xyz2.shape[0], 3, 4)
    ex2, na2 = both(small, u, stream=torch.cuda.Stream())
    assert np.array_equal(ex2, na2)
    ref = h2.H2Oracle(xyz2, tri2, order=3, leaf=16, eta=2.0).apply(u)
    assert np.max(np.linalg.norm(na2 - ref, axis=1) / np.linalg.norm(ref, axis=1)) <= 1e-12
    # and the larger operator again after the smaller one
    ex3, na3 = both(big, rhs.normal_rhs(xyz.shape[0], 5, 6))
    assert np.array_equal(ex3, na3)


def test_noalloc_rejects_a_workspace_beyond_the_scratch(lib):
    # 163842 nodes in FP64: about 160 MB of workspace against 128 MiB
    xyz, tri = meshes.icosphere(7, 0.005, 0)
    op = lib.Operator(xyz, tri, order=4, leaf=64, eta=2.0, precision="fp64", coupling="generated")
    assert op.stats.workspace_bytes > lib.NOALLOC_SCRATCH_BYTES
    d1 = torch.zeros((1, xyz.shape[0]), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.H2dlpError) as e:
        op.apply_noalloc(d1, torch.empty_like(d1))
    assert e.value.code == lib.ENOMEM and "scratch" in str(e.value)
