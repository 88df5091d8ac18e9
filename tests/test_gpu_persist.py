"""Saving a built operator to a file and loading it back (h2dlp_save /
h2dlp_load; Section 6.1: the H2 matrix is computed once per geometry, stored
and read back at later starts).  A loaded operator gives the saved one's
results bit for bit, in every representation, also when saved while
offloaded; its stats are the built operator's."""
import numpy as np
import pytest

from workloads import meshes, rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1811_05731_amd import h2dlp
    return h2dlp


def run(op, u, dtype=torch.float64):
    d1 = torch.tensor(u, dtype=dtype, device="cuda")
    d2 = torch.full_like(d1, float("nan"))
    op.apply(d1, d2)
    torch.cuda.synchronize()
    return d2.cpu().numpy()


CONFIGS = [
    dict(precision="fp64"),
    dict(precision="fp32", coupling="generated", dense_far_max=2048),
    dict(precision="fp32", coupling="generated", row_basis="generated"),
    dict(precision="bf16x3", dense_far_max=4096),
    dict(precision="fp32", recompress_eps=1e-6),
    dict(precision="fp64", recompress_eps=1e-4),
]


@pytest.mark.parametrize("kw", CONFIGS, ids=lambda kw: "-".join(f"{k}={v}" for k, v in kw.items()))
def test_load_gives_the_saved_operator(lib, tmp_path, kw):
    xyz, tri = meshes.icosphere(4, 0.01, 0)
    u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(xyz.shape[0], 20, 3)])    # two passes of 16 columns
    op = lib.Operator(xyz, tri, order=4, leaf=32, eta=2.0, **kw)
    ref = run(op, u)
    ref32 = run(op, u, torch.float32)
    path = tmp_path / "op.h2dlp"
    op.save(path)
    st = op.stats
    op.close()
    back = lib.Operator.load(path)
    assert back.stats == st
    assert np.array_equal(run(back, u), ref)
    assert np.array_equal(run(back, u, torch.float32), ref32)
    assert np.array_equal(back.export_diagonal(), back.export_diagonal())
    # a loaded operator offloads, reloads and saves like a built one
    back.offload()
    path2 = tmp_path / "op2.h2dlp"
    back.save(path2)                       # written from the parked host copy
    back.reload()
    assert np.array_equal(run(back, u), ref)
    back.close()
    assert path2.read_bytes() == path.read_bytes()
    again = lib.Operator.load(path2, device=0)
    assert np.array_equal(run(again, u), ref)
    again.close()


def test_load_at_larger_size(lib, tmp_path):
    import time
    xyz, tri = meshes.icosphere(6, 0.005, 0)
    t0 = time.perf_counter()
    op = lib.Operator(xyz, tri, order=4, leaf=64, eta=2.0, precision="fp32", recompress_eps=1e-6)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    u = rhs.normal_rhs(xyz.shape[0], 4, 0)
    ref = run(op, u)
    path = tmp_path / "l6.h2dlp"
    op.save(path)
    op.close()
    t0 = time.perf_counter()
    back = lib.Operator.load(path)
    torch.cuda.synchronize()
    t_load = time.perf_counter() - t0
    print(f"L6 recompressed: build {t_build:.2f} s, load {t_load:.2f} s, file {path.stat().st_size / 1e6:.0f} MB")
    assert np.array_equal(run(back, u), ref)
    back.close()
