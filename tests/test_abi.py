"""The C ABI without a GPU: symbols, argument checks, host-only planning and
structure identity with the oracle (cluster tree, boxes, block lists)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import h2
from paper_1811_05731_amd import h2dlp
from workloads import cases, meshes

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "h2dlp.h")


def test_every_declared_symbol_is_exported():
    names = set(re.findall(r"\b(h2dlp_[a-z_]+)\s*\(", open(HEADER).read()))
    assert len(names) >= 14
    lib = ctypes.CDLL(h2dlp.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(h2dlp.EXPORTED) == names


def test_default_options():
    o = h2dlp.default_options()
    assert (o["order"], o["leaf"], o["eta"], o["precision"], o["alpha"], o["device"]) == (4, 32, 2.0, 0, 0.1, -1)
    assert (o["coupling"], o["dense_far_max"], o["recompress_eps"], o["row_basis"]) == (0, 0, 0.0, 0)


def _plan_rc(xyz, tri, **kw):
    try:
        h2dlp.plan(xyz, tri, **kw)
        return 0
    except h2dlp.H2dlpError as e:
        return e.code


def test_argument_errors():
    xyz, tri = meshes.icosphere(2)
    assert _plan_rc(xyz, tri, order=0) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, order=9) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, leaf=0) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, leaf=65) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, eta=0.0) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, eta=float("nan")) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, alpha=-0.1) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, order=6, precision="bf16x3") == h2dlp.ENOTSUP
    assert _plan_rc(xyz, tri, order=6, precision="bf16x6") == h2dlp.ENOTSUP
    assert _plan_rc(xyz, tri, order=5, precision="bf16x6") == 0
    assert _plan_rc(xyz, tri, order=6, coupling="generated") == h2dlp.ENOTSUP
    assert _plan_rc(xyz, tri, order=4, precision="bf16x3", coupling="generated") == h2dlp.ENOTSUP
    assert _plan_rc(xyz, tri, order=5, precision="fp32", coupling="generated") == 0
    lib = h2dlp.library()
    out = ctypes.c_void_p()
    opt = h2dlp._Options()
    lib.h2dlp_default_options(ctypes.byref(opt))
    assert lib.h2dlp_plan(None, ctypes.byref(opt), ctypes.byref(out)) == h2dlp.EINVAL
    assert lib.h2dlp_build(None, 4, 32, 2.0) is None
    assert lib.h2dlp_apply(None, None, None, 1) == h2dlp.EINVAL
    assert lib.h2dlp_info(None, None) == h2dlp.EINVAL
    assert "NULL" in h2dlp.last_error()


def test_mesh_errors():
    xyz, tri = meshes.icosphere(2)
    bad = tri.copy(); bad[0] = bad[0][[0, 2, 1]]
    assert _plan_rc(xyz, bad) == h2dlp.EINVAL and "orientation" in h2dlp.last_error()
    assert _plan_rc(xyz, tri[1:]) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri[:, [0, 2, 1]]) == h2dlp.EINVAL and "volume" in h2dlp.last_error()
    bad = tri.copy(); bad[5, 2] = bad[5, 0]
    assert _plan_rc(xyz, bad) == h2dlp.EINVAL and "degenerate" in h2dlp.last_error()
    bad = tri.copy(); bad[0, 0] = xyz.shape[0]
    assert _plan_rc(xyz, bad) == h2dlp.EINVAL and "range" in h2dlp.last_error()
    dup = xyz.copy(); dup[7] = dup[3]
    assert _plan_rc(dup, tri) == h2dlp.EINVAL
    nan = xyz.copy(); nan[2, 1] = np.nan
    assert _plan_rc(nan, tri) == h2dlp.EINVAL


def test_apply_on_plan_handle_is_rejected():
    xyz, tri = meshes.icosphere(2)
    p = h2dlp.plan(xyz, tri)
    lib = h2dlp.library()
    buf = (ctypes.c_double * (2 * xyz.shape[0]))()
    assert lib.h2dlp_apply(p.handle, buf, ctypes.byref(buf, 8 * xyz.shape[0]), 1) == h2dlp.EINVAL


def _same_structure(xyz, tri, order, leaf, eta):
    lib_s = h2dlp.plan(xyz, tri, order=order, leaf=leaf, eta=eta).export_structure()
    ora_s = h2.H2Oracle(xyz, tri, order=order, leaf=leaf, eta=eta).export_structure()
    for key in ora_s:
        assert np.array_equal(np.asarray(ora_s[key]), np.asarray(lib_s[key])), key


@pytest.mark.parametrize("mesh,leaf,eta", [
    (lambda: meshes.icosphere(4, 0.01, 0), 32, 2.0),
    (lambda: meshes.icosphere(5, 0.01, 0), 64, 2.0),
    (lambda: meshes.icosphere(3, 0.0, 0), 16, 1.0),                 # unjittered: many ties
    (lambda: meshes.cuboid(200.0, 200.0, 20.0, 5.0, 0.5, 0), 64, 2.0),  # flat faces: inflated boxes
    (lambda: meshes.torus(1.0, 0.3, 64, 16), 32, 3.0),
])
def test_structure_identical_to_oracle(mesh, leaf, eta):
    xyz, tri = mesh()
    _same_structure(xyz, tri, 4, leaf, eta)


def test_plan_sizes():
    xyz, tri = meshes.icosphere(4, 0.01, 0)
    s = h2dlp.plan(xyz, tri, order=4, leaf=32, eta=2.0).stats
    ora = h2.H2Oracle(xyz, tri, order=4, leaf=32, eta=2.0).counts()
    assert (s.n_clusters, s.n_leaves, s.n_far, s.n_near, s.near_entries) == \
        (ora["clusters"], ora["leaves"], ora["far"], ora["near"], ora["near_entries"])
    assert s.coupling_entries == s.n_far * 64 * 64
    assert s.bytes_coupling == 8 * s.coupling_entries
    s32 = h2dlp.plan(xyz, tri, order=4, leaf=32, eta=2.0, precision="fp32").stats
    assert s32.bytes_coupling == 4 * s.coupling_entries
    assert 10 * xyz.shape[0] < s32.nearsing_entries < 25 * xyz.shape[0]   # the 2-ring, ~18 per node
    s3 = h2dlp.plan(xyz, tri, order=4, leaf=32, eta=2.0, precision="bf16x3").stats
    s6 = h2dlp.plan(xyz, tri, order=4, leaf=32, eta=2.0, precision="bf16x6").stats
    assert s3.bytes_coupling == 4 * s.coupling_entries and s6.bytes_coupling == 6 * s.coupling_entries
    assert s6.bytes_resident - s3.bytes_resident == 2 * s.coupling_entries   # k = 64: no padding columns
    assert s6.bytes_near == s32.bytes_near and s6.bytes_bases == s32.bytes_bases
    sg = h2dlp.plan(xyz, tri, order=4, leaf=32, eta=2.0, precision="fp32", coupling="generated").stats
    assert sg.bytes_coupling == 0 and sg.coupling_entries == s.coupling_entries
    assert s32.bytes_resident - sg.bytes_resident == 4 * s.coupling_entries - 48 * s.n_clusters
    # regenerated row bases: V (N k values) gives way to the node coordinates
    # (24 bytes a node) and a 64-byte record per leaf, and each leaf item loses
    # its V block descriptor (16 bytes); k = 64 leaves no padding to account for
    sr = h2dlp.plan(xyz, tri, order=4, leaf=32, eta=2.0, precision="fp32", row_basis="generated").stats
    n = xyz.shape[0]
    assert s32.bytes_bases - sr.bytes_bases == 4 * n * 64 - 24 * n - 64 * s.n_leaves
    assert s32.bytes_resident - sr.bytes_resident == 4 * n * 64 - 24 * n - 48 * s.n_leaves
    assert (sr.n_far, sr.n_near, sr.coupling_entries, sr.bytes_near) == (s32.n_far, s32.n_near,
                                                                         s32.coupling_entries, s32.bytes_near)
    r, w = h2dlp.plan(xyz, tri).bytes()
    assert w > 0 and r > w


@pytest.mark.parametrize("dmax", [0, 1024, 4096])
def test_dense_far_plan_matches_oracle(dmax):
    xyz, tri = meshes.icosphere(4, 0.01, 0)
    s = h2dlp.plan(xyz, tri, order=4, leaf=32, eta=2.0, dense_far_max=dmax).stats
    ora = h2.H2Oracle(xyz, tri, order=4, leaf=32, eta=2.0, dense_far_max=dmax)
    c = ora.counts()
    assert (s.n_far, s.n_far_dense, s.near_entries, s.dense_far_entries) == \
        (c["far"], c["far_dense"], c["near_entries"], c["dense_far_entries"])
    assert s.coupling_entries == s.n_far * 64 * 64
    assert s.bytes_near == 8 * (s.near_entries + s.dense_far_entries)
    st = h2dlp.plan(xyz, tri, order=4, leaf=32, eta=2.0, dense_far_max=dmax).export_structure()
    assert np.array_equal(st["far"], ora.far)
    if dmax:
        assert s.n_far_dense > 0
    with pytest.raises(h2dlp.H2dlpError):
        h2dlp.plan(xyz, tri, dense_far_max=-1)


def test_build_without_gpu_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    xyz, tri = meshes.icosphere(2)
    with pytest.raises(h2dlp.H2dlpError) as e:
        h2dlp.Operator(xyz, tri)
    assert e.value.code in (h2dlp.ENOTSUP, h2dlp.EDEVICE)


def test_apply_rejects_bad_tensors_before_any_launch():
    # the binding refuses host tensors, tensors on another device, wrong ranks
    # and nrhs beyond the rows before it passes a pointer to the library (a
    # stand-in handle that the library is never given)
    torch = pytest.importorskip("torch")
    op = object.__new__(h2dlp.Operator)
    op._h, op.plan_only, op.n_nodes, op.device = ctypes.c_void_p(0), False, 10, 0
    u = torch.zeros(3, 10, dtype=torch.float64)
    with pytest.raises(ValueError, match="cuda:0"):
        op.apply(u, torch.zeros_like(u))
    with pytest.raises(ValueError, match="nrhs"):
        op.apply(u, torch.zeros_like(u), nrhs=4)
    with pytest.raises(ValueError, match="nrhs"):
        op.apply(u, torch.zeros_like(u), nrhs=0)
    with pytest.raises(ValueError, match="shape"):
        op.apply(torch.zeros(2, 3, 10, dtype=torch.float64), torch.zeros(2, 3, 10, dtype=torch.float64))
    with pytest.raises(ValueError, match="float64 or both float32"):
        op.apply(u, torch.zeros(3, 10, dtype=torch.float32))
    op._h = None                                   # nothing to free
    planned = h2dlp.plan(*meshes.icosphere(2), order=2, leaf=16)
    with pytest.raises(ValueError, match="planned"):
        planned.apply(u, torch.zeros_like(u))


def test_recompression_arguments():
    xyz, tri = meshes.icosphere(2)
    assert _plan_rc(xyz, tri, recompress_eps=-1e-3) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, recompress_eps=1.0) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, recompress_eps=float("nan")) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, recompress_eps=1e-6, coupling="generated") == h2dlp.ENOTSUP
    assert _plan_rc(xyz, tri, recompress_eps=1e-6, precision="bf16x3") == h2dlp.ENOTSUP
    assert _plan_rc(xyz, tri, order=6, recompress_eps=1e-6) == h2dlp.ENOTSUP
    assert _plan_rc(xyz, tri, row_basis=2) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, row_basis=-1) == h2dlp.EINVAL
    assert _plan_rc(xyz, tri, row_basis="generated", recompress_eps=1e-6) == h2dlp.ENOTSUP
    p = h2dlp.plan(xyz, tri, order=3, leaf=16, recompress_eps=1e-6, precision="fp32")
    q = h2dlp.plan(xyz, tri, order=3, leaf=16, precision="fp32")
    # before the build the plan reports the interpolation sizes, an upper bound
    assert p.stats.rank_sum_row == p.stats.n_clusters * 27 and p.stats.rank_max_col == 27
    assert p.stats.n_far == q.stats.n_far and p.stats.coupling_entries == q.stats.coupling_entries


def test_persistence_errors(tmp_path):
    # h2dlp_save / h2dlp_load refuse what they cannot use before touching a device
    lib = h2dlp.library()
    xyz, tri = meshes.icosphere(2)
    op = h2dlp.plan(xyz, tri)
    assert lib.h2dlp_save(op.handle, str(tmp_path / "x.op").encode()) == h2dlp.EINVAL   # nothing on a device
    assert lib.h2dlp_save(None, b"x") == h2dlp.EINVAL
    with pytest.raises(ValueError):
        op.save(tmp_path / "x.op")
    out = ctypes.c_void_p(1)
    assert lib.h2dlp_load(str(tmp_path / "missing.op").encode(), -1, ctypes.byref(out)) == h2dlp.EINVAL
    assert out.value is None
    assert lib.h2dlp_load(None, -1, ctypes.byref(out)) == h2dlp.EINVAL
    assert lib.h2dlp_load(b"x", -1, None) == h2dlp.EINVAL
    junk = tmp_path / "junk.op"
    junk.write_bytes(b"not an operator file at all")
    assert lib.h2dlp_load(str(junk).encode(), -1, ctypes.byref(out)) == h2dlp.EINVAL
    assert "not an h2dlp operator file" in h2dlp.last_error()
    # right magic, another format version
    other = tmp_path / "other.op"
    other.write_bytes(b"H2DLPOPS" + (99).to_bytes(4, "little") + bytes(64))
    assert lib.h2dlp_load(str(other).encode(), -1, ctypes.byref(out)) == h2dlp.ENOTSUP
    # right header, cut short inside the options
    cut = tmp_path / "cut.op"
    cut.write_bytes(b"H2DLPOPS" + (2).to_bytes(4, "little") + (36).to_bytes(4, "little")
                    + ctypes.sizeof(h2dlp._Stats).to_bytes(4, "little") + bytes(10))
    assert lib.h2dlp_load(str(cut).encode(), -1, ctypes.byref(out)) == h2dlp.EINVAL
    assert out.value is None


def test_fem_volume_errors():
    # h2dlp_fem_build checks the volume before it touches a device
    from workloads import volume
    xyz, tets = volume.box_tets(1.0, 1.0, 1.0, 2, 2, 2)
    bad = tets.copy()
    bad[0, 1] = len(xyz)
    flat = tets.copy()
    flat[0, 3] = flat[0, 2]
    for t, what in ((bad, "out of range"), (flat, "degenerate")):
        with pytest.raises(h2dlp.H2dlpError) as e:
            h2dlp.FemField(xyz, t)
        assert e.value.code == h2dlp.EINVAL and what in str(e.value)
    lib = h2dlp.library()
    out = ctypes.c_void_p()
    assert lib.h2dlp_fem_build(None, None, ctypes.byref(out)) == h2dlp.EINVAL
    assert lib.h2dlp_fem_field(None, None, None, None, None, 1e-10, 10, None, None) == h2dlp.EINVAL
