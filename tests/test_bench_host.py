"""Host-side logic of bench.py: exact-block thresholds, the roofline
arithmetic of the reported records, and the one-GPU contract."""
import os
import subprocess
import sys
import types

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_default_thresholds():
    assert bench.default_dense_far_max(5, "stored") == 125 ** 2
    assert bench.default_dense_far_max(5, "generated") == 125 ** 2 // 2
    assert bench.default_dense_far_max(4, "generated") == 64 ** 2 // 2


def test_coupling_records():
    st = types.SimpleNamespace(coupling_entries=10 * 125 ** 2, n_clusters=7, k=125, rank_sum_row=7 * 125,
                               rank_sum_col=7 * 125)
    # generated: 2 flops per entry and right-hand side, 16 right-hand sides per pass
    flops = 2.0 * 10 * 125 ** 2 * 16
    assert bench.coupling_flops(st) == flops
    r = bench.roofline_of(st, "fp32", "generated", {"coupling": (4.0, 2)}, 1000, 2)    # 2 ms per apply
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert abs(r["achieved"] - flops / 2e-3 / 1e12) < 0.01
    assert abs(r["roofline_ms"] - flops / 157.3e12 * 1e3) < 1e-4
    # stored: every entry once, xhat read and yhat written once per cluster
    b = 10 * 125 ** 2 * 4 + 2 * 7 * 125 * 16 * 4
    assert bench.coupling_alg_bytes(st, 4, 4) == b
    r = bench.roofline_of(st, "fp32", "stored", {"coupling": (1.0, 1)}, 1000, 1)
    assert r["bound"] == "hbm" and r["alg_bytes_per_launch"] == b
    assert abs(r["frac"] - b / 1e-3 / 1e9 / 8000.0) < 1e-4
    # FP64 and BF16X6 entries are 8 and 6 bytes
    assert bench.roofline_of(st, "fp64", "stored", {"coupling": (1.0, 1)}, 1000, 1)["alg_bytes_per_launch"] == \
        10 * 125 ** 2 * 8 + 2 * 7 * 125 * 16 * 8
    assert bench.roofline_of(st, "bf16x6", "stored", {"coupling": (1.0, 1)}, 1000, 1)["alg_bytes_per_launch"] == \
        10 * 125 ** 2 * 6 + 2 * 7 * 125 * 16 * 4


def test_near_field_record():
    st = types.SimpleNamespace(bytes_near=10 ** 6)
    # per node and column: x64 (8 B) read and y64 (8 B) written by the
    # diagonal kernel, x (operator precision) read and y64 read and written by
    # the near-field product; D (8 B) per node
    assert bench.near_field_alg_bytes(st, 4, 100) == 10 ** 6 + 100 * 16 * 36 + 800
    assert bench.near_field_alg_bytes(st, 8, 100) == 10 ** 6 + 100 * 16 * 40 + 800
    r = bench.near_field_roofline(st, "fp32", {"near_field": (3.0, 3)}, 100, 3)
    assert r["bound"] == "hbm" and abs(r["achieved"] - (10 ** 6 + 57600 + 800) / 1e-3 / 1e9) < 0.1
    # two event intervals per apply (the launches before and after the first
    # coupling launch): still 1 ms per apply
    r2 = bench.near_field_roofline(st, "fp32", {"near_field": (3.0, 6)}, 100, 3)
    assert r2["achieved"] == r["achieved"] and r2["avg_launch_ms"] == 1.0 and r2["event_intervals_per_apply"] == 2


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""


def test_apply_roofline_record():
    st = types.SimpleNamespace(bytes_coupling=0, bytes_near=4 * 10 ** 6, bytes_bases=4 * 2 * 100 * 8,
                               bytes_transfer=0, n_clusters=3, k=8, coupling_entries=10 ** 9, near_entries=10 ** 6,
                               dense_far_entries=0, rank_sum_row=24, rank_sum_col=24)
    r = bench.apply_roofline(st, "fp32", 100, 16, 1.0, "generated")
    flops = 2.0 * (10 ** 9 + 10 ** 6 + 2 * 100 * 8) * 16
    assert r["alg_flops"] == flops and r["bound"] == "mfma"
    assert abs(r["roofline_ms"] - flops / 157.3e9) < 1e-4 and abs(r["frac"] - r["roofline_ms"] / 1.0) < 1e-4
    assert r["alg_bytes"] == bench.apply_alg_bytes(st, 4, 100, 16)
    st.coupling_entries = 0
    assert bench.apply_roofline(st, "fp64", 100, 16, 1.0, "stored")["bound"] == "hbm"


def test_host_cpu_and_sampled_oracle():
    h = bench.host_cpu()
    assert 1 <= h["cores"] <= min(16, h["visible_cpus"])
    from workloads import meshes
    xyz, tri = meshes.icosphere(3, 0.01, 0)
    case = types.SimpleNamespace(order=3, leaf=16, eta=2.0)
    r = bench.oracle_sample(xyz, tri, case, 4, dense_far_max=81, cores=2, frac=0.2)
    assert r["cores"] == 2 and r["kind"] == "oracle" and r["value"] > 0 and r["est_apply_s"] > 0
    assert "dense" in r["sample"] and "far" in r["sample"]


def test_direct_oracle_timing():
    r = bench.oracle_direct("sphere_l4", cores=2, reps=2)
    assert r["nodes"] == 2562 and r["rhs"] == 2 and len(r["apply_s"]) == 2 and r["GDOF_s"] > 0
