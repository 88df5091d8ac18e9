"""Benchmark of the H2 boundary double-layer matvec u2 = (K + D) u1 on one MI355X.

One step = one apply of the whole hot path (permute, leaf forward, upward
transfers, coupling, downward transfers, leaf backward + near field + diagonal)
to 16 right-hand sides on the level-8 icosphere (655362 boundary nodes), order
5, leaf 64, eta 2.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  `value` is boundary degrees of freedom per second
(N * nrhs / t_apply / 1e9).  `rooflines` holds a record for the coupling
products and one for the near field, each from its HIP-event time inside the
timed region; `roofline` is the dominant one, whose algorithmic work at its
own peak takes longer.  `cpu_baseline` times the CPU oracle on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H² DLP matvec boundary GDOF/s + %HBM roofline; serve p50/p99 at 1e-6 rel err"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_1811_05731_amd/csrc/apply_kernels.hip", "paper_1811_05731_amd/csrc/layout.h",
                  "paper_1811_05731_amd/csrc/kernels.h", "paper_1811_05731_amd/csrc/api.cpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sphere_l8.json")
RHS_PER_PASS = 16
DEFAULT_COUPLING = "stored"
DEFAULT_RECOMPRESS_EPS = 1e-6


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def workload(name: str):
    from workloads import cases
    c = cases.CASES[name]
    xyz, tri = cases.mesh_of(c.mesh)
    return c, xyz, tri


def default_dense_far_max(order: int, coupling: str) -> int:
    """Largest |t||s| for which an admissible block is cheaper kept exact.

    Stored coupling: whenever its entries are fewer than the k^2 of a coupling
    matrix (bytes against bytes).  Generated coupling: the exact block costs
    4 |t||s| bytes of HBM (~5 TB/s achieved) while the low-rank block costs
    2 k^2 16 flops of FP32 MFMA (~92 TFLOP/s achieved); alone they would
    balance at |t||s| ~ 0.43 k^2.  The two run side by side, and at L8 the
    apply time is flat within 1 % from 0.5 to 0.63 k^2: k^2 / 2 is taken.
    """
    k2 = order ** 6
    return k2 if coupling == "stored" else k2 // 2


def case_rhs(case, xyz):
    """The right-hand sides each workload is quoted with, and their description."""
    from workloads import rhs
    n = xyz.shape[0]
    if case.name == "film":
        return rhs.smooth_fields(xyz, case.nrhs), f"{case.nrhs} smooth fields (16 sinusoids, wavelengths 50-2000 nm)"
    if case.name in ("sphere_l4", "sphere_l7"):
        return (np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(n, case.nrhs - 1, 0)]),
                f"u1 = z and {case.nrhs - 1} N(0,1) right-hand sides")
    return rhs.normal_rhs(n, case.nrhs, 0), f"{case.nrhs} N(0,1) right-hand sides"


def describe(case, n, n_tri, rhs_text, dense_far_max=0, coupling="stored", recompress_eps=0.0):
    m = case.mesh
    if m.kind == "icosphere":
        geo = f"icosphere level {m.level}, radial jitter +-{m.jitter:g}"
    elif m.kind == "cuboid":
        geo = f"thin-film cuboid 2000 x 2000 x 20 nm on a 5 nm grid, in-plane jitter +-{m.jitter:g} nm"
    else:
        geo = m.kind
    rep = (f"coupling matrices {'recomputed in the apply' if coupling == 'generated' else 'stored'}"
           + (f", admissible blocks with |t||s| <= {dense_far_max} kept exact" if dense_far_max else "")
           + (f", bases recompressed to adaptive ranks (relative tolerance {recompress_eps:g})" if recompress_eps
              else ""))
    return (f"{case.name}: {geo}, {n} boundary nodes, {n_tri} triangles, order {case.order}, leaf {case.leaf}, "
            f"eta {case.eta:g}, {rhs_text}; {rep}")


def coupling_alg_bytes(st, elem_s: int, elem_v: int) -> int:
    """Algorithmic bytes of one coupling launch: every S_ts once (elem_s bytes
    per entry), xhat read once and yhat written once (elem_v bytes per value;
    the ranks summed over the clusters are C k without recompression)."""
    return st.coupling_entries * elem_s + (st.rank_sum_col + st.rank_sum_row) * 16 * elem_v


def apply_alg_bytes(st, elem: int, n_nodes: int, nrhs: int, io_elem: int = 8) -> int:
    """Algorithmic bytes of one apply: the stored operator once, plus compulsory vectors."""
    operator = st.bytes_coupling + st.bytes_near + st.bytes_bases + st.bytes_transfer
    vectors = (8 * n_nodes + 4 * n_nodes + 2 * io_elem * n_nodes * nrhs
               + 2 * (st.rank_sum_col + st.rank_sum_row) * 16 * elem)
    return operator + vectors


def time_path(op, d_u1, d_u2, steps: int, warmup: int, profile):
    """Mean ms per apply over `steps` applies; `profile` = kinds whose launches
    are timed with HIP events inside the same region (None = none)."""
    import torch
    for _ in range(warmup):
        op.apply(d_u1, d_u2)
    torch.cuda.synchronize()
    if profile:
        op.profile(profile)
        op.profile_read(reset=True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        op.apply(d_u1, d_u2)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    kernels = None
    if profile:
        kernels = op.profile_read(reset=True)
        op.profile(False)
    return ms, kernels


def median_apply_ms(op, d_u1, d_u2, n: int) -> float:
    """Median over n applies, each bracketed by its own pair of HIP events (after the timed region)."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for e0, e1 in evs:
        e0.record()
        op.apply(d_u1, d_u2)
        e1.record()
    torch.cuda.synchronize()
    return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))


def copy_bandwidth(dev, reps: int = 10) -> float:
    """Device-to-device copy of 1 GiB: bytes read + written per second (GB/s)."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def sphere_check(op, xyz, dev) -> dict:
    """u1 = z on the unit sphere: u2 should be -2z/3 (demagnetising factor 1/3),
    and u1 = 1 gives u2 = -1.  Also the same with the smooth-surface diagonal
    -1/2 in place of Psi/(4 pi) - 1, for comparison."""
    import torch
    z = xyz[:, 2]
    d1 = torch.tensor(np.vstack([z, np.ones_like(z)]), device=dev)
    d2 = torch.empty_like(d1)
    op.apply(d1, d2)
    torch.cuda.synchronize()
    u2 = d2.cpu().numpy()
    diag = op.export_diagonal()
    exact = -2.0 * z / 3.0
    half = u2[0] - diag * z - 0.5 * z
    rel = lambda a: float(f"{np.linalg.norm(a - exact) / np.linalg.norm(exact):.3e}")  # noqa: E731
    return {"u1_z_rel_err": rel(u2[0]), "u1_z_rel_err_half_identity": rel(half),
            "u1_one_max_err": float(f"{np.max(np.abs(u2[1] + 1.0)):.3e}")}


def host_cpu() -> dict:
    """The host's CPU model and the cores the CPU baseline uses: the CPUs this
    process may run on, at most 16 (one GPU's share of its host)."""
    visible = len(os.sched_getaffinity(0))
    model = None
    with open("/proc/cpuinfo") as f:
        for line in f:
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    return {"cores": min(16, visible), "visible_cpus": visible, "model": model}


_CPU = {}        # state the forked CPU-baseline workers inherit


def _sample_worker(q: int):
    """Worker q of the sampled oracle apply: build its items' pieces (untimed),
    wait for every worker, then time its share of the sampled items."""
    from threadpoolctl import threadpool_limits
    H, x, xh, items = _CPU["H"], _CPU["x"], _CPU["xh"], _CPU["items"][q]
    with threadpool_limits(limits=1):
        for kind, a in items:                       # pieces the oracle builds once per operator
            if kind == "leaf":
                H.W(a), H.V(a)
            elif kind == "up":
                H.E(H.child0[a]), H.E(H.child1[a])
            elif kind == "down":
                H.E(a)
            elif kind in ("near", "dense"):
                H.K_near(*a)
        _CPU["barrier"].wait()
        t0 = time.perf_counter()
        for kind, a in items:
            if kind == "leaf":
                _ = H.W(a).T @ x[H.nodes(a)]
                _ = H.V(a) @ xh
            elif kind == "up":
                _ = H.E(H.child0[a]).T @ xh + H.E(H.child1[a]).T @ xh
            elif kind == "down":
                _ = H.E(a) @ xh
            elif kind == "far":
                _ = H.S(*a) @ xh                    # generated on the fly, as the oracle does here
            else:
                _ = H.K_near(*a) @ x[H.nodes(a[1])]
        t1 = time.perf_counter()
    return t0, t1


def _fill_worker(args):
    """Pieces of the oracle built in a worker for the parent's caches."""
    kind, chunk = args
    H = _CPU["H"]
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        if kind == "W":
            return kind, [(int(c), H.W(c)) for c in chunk]
        if kind == "K":
            return kind, [((int(t), int(s)), H.K_near(t, s)) for t, s in chunk]
        return kind, [((int(t), int(s)), H.S(t, s)) for t, s in chunk]


def oracle_sample(xyz, tri, case, nrhs: int, dense_far_max: int, cores: int, frac: float = 0.05,
                  seed: int = 7) -> dict:
    """The oracle's apply of the benchmarked operator, timed on a sample.

    The oracle's matvec is a loop over work items: leaves (W_s^T x, V_t yhat),
    upward and downward transfers, low-rank far blocks (S_ts generated on the
    fly, as the GPU path does), near blocks and exact admissible blocks.  A
    seeded fraction `frac` of every kind is dealt over `cores` worker
    processes (one BLAS thread each).  Each worker first builds the pieces the
    oracle builds once per operator (bases, transfers, exact blocks; untimed),
    then all time their items together; the whole-apply estimate is that wall
    time divided by `frac`.
    """
    from multiprocessing import get_context

    from oracle import h2
    t0 = time.perf_counter()
    H = h2.H2Oracle(xyz, tri, order=case.order, leaf=case.leaf, eta=case.eta, cache_coupling=False,
                    dense_far_max=dense_far_max)
    t_struct = time.perf_counter() - t0
    rng = np.random.default_rng(seed)
    C = H.n_clusters
    kinds = {"leaf": list(np.where(H.child0 < 0)[0]), "up": list(np.where(H.child0 >= 0)[0]),
             "down": list(range(1, C)), "far": [tuple(b) for b in H.far], "near": [tuple(b) for b in H.near],
             "dense": [tuple(b) for b in H.far_dense]}
    items, counts = [], {}
    for kind, lst in kinds.items():
        if not lst:
            continue
        pick = rng.choice(len(lst), max(1, int(round(frac * len(lst)))), replace=False)
        items += [(kind, lst[p]) for p in pick]
        counts[kind] = (len(pick), len(lst))
    order = rng.permutation(len(items))
    ctx = get_context("fork")
    _CPU.update(H=H, x=rng.normal(size=(xyz.shape[0], nrhs)), xh=rng.normal(size=(H.k, nrhs)),
                items=[[items[o] for o in order[q::cores]] for q in range(cores)], barrier=ctx.Barrier(cores))
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        spans = pool.map(_sample_worker, range(cores))
    t_run = time.perf_counter() - t0
    wall = max(b for _, b in spans) - min(a for a, _ in spans)
    t0 = time.perf_counter()
    _ = H.D[:, None] * _CPU["x"]
    t_diag = time.perf_counter() - t0
    _CPU.clear()
    est = wall / frac + t_diag
    n = xyz.shape[0]
    return {"value": n * nrhs / est / 1e9, "unit": "GDOF/s", "cores": cores, "kind": "oracle",
            "sample": (f"{frac:.0%} of every item kind of the benchmarked operator (seed {seed}): "
                       + ", ".join(f"{k} {a}/{b}" for k, (a, b) in counts.items())
                       + f"; dealt over {cores} processes with one BLAS thread each; whole-apply time = "
                         f"their common wall time / {frac:g}; S_ts generated on the fly"),
            "est_apply_s": round(est, 3), "sample_wall_s": round(wall, 4),
            "oracle_structure_s": round(t_struct, 2), "piece_build_and_sample_s": round(t_run, 2)}


def oracle_direct(case_name: str, cores: int, dense_far_max: int = 0, reps: int = 3) -> dict:
    """The oracle's whole apply timed directly (median of `reps`) on a named
    workload, after one apply that builds its pieces.  Bases, exact blocks and
    coupling matrices of that first apply are computed by `cores` worker
    processes into the oracle's own caches (logged as the oracle's build)."""
    from multiprocessing import get_context

    from threadpoolctl import threadpool_limits

    from oracle import h2
    case, xyz, tri = workload(case_name)
    u1, _ = case_rhs(case, xyz)
    t0 = time.perf_counter()
    H = h2.H2Oracle(xyz, tri, order=case.order, leaf=case.leaf, eta=case.eta, dense_far_max=dense_far_max)
    _CPU["H"] = H
    jobs = [("W", c) for c in np.array_split(np.where(H.child0 < 0)[0], 4 * cores)]
    jobs += [("K", c) for c in np.array_split(np.concatenate([H.near, H.far_dense]), 8 * cores)]
    jobs += [("S", c) for c in np.array_split(H.far, 8 * cores)]
    with get_context("fork").Pool(cores) as pool:
        for kind, part in pool.imap_unordered(_fill_worker, jobs):
            cache = {"W": H._W, "K": H._K, "S": H._S}[kind]
            for key, val in part:
                cache[key] = val
    _CPU.clear()
    with threadpool_limits(limits=cores):
        H.apply(u1)                                            # transfers and V; everything else cached
        t_build = time.perf_counter() - t0
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            H.apply(u1)
            times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    n = xyz.shape[0]
    return {"workload": case_name, "nodes": n, "rhs": u1.shape[0], "dense_far_max": dense_far_max,
            "apply_s_median": round(t, 4), "apply_s": [round(v, 4) for v in times],
            "GDOF_s": n * u1.shape[0] / t / 1e9, "build_s": round(t_build, 1),
            "note": f"coupling matrices cached after the first apply; BLAS at {cores} threads"}


def cpu_baseline(xyz, tri, case, nrhs: int, dense_far_max: int, direct_c2: bool = True,
                 recompress_eps: float = 0.0) -> dict:
    """The CPU oracle beside the GPU: the benchmarked operator on a sample
    (`value`), the 2562-node sphere timed directly (dense matvec and whole H2
    apply, median of 3) and, unless disabled, the 163842-node sphere's whole
    apply timed directly."""
    from threadpoolctl import threadpool_limits

    from oracle import dense, h2, recompress
    from workloads import cases, rhs
    host = host_cpu()
    cores = host["cores"]
    out = oracle_sample(xyz, tri, case, nrhs, dense_far_max, cores)
    if recompress_eps:
        out["operator"] = ("the oracle's interpolation H2 matrix of the same mesh (the matrix the recompressed "
                           "operator approximates to the tolerance; the oracle's own recompression of 655362 "
                           "nodes takes far longer than a baseline may); its recompressed apply is timed "
                           "directly at 2562 nodes under direct.sphere_l4")
    out["cpu_model"] = host["model"]
    out["visible_cpus"] = host["visible_cpus"]
    c1 = cases.CASES["sphere_l4"]
    x1, t1 = cases.mesh_of(c1.mesh)
    M = dense.dense_m(x1, t1)
    u = np.vstack([rhs.z_rhs(x1), rhs.normal_rhs(x1.shape[0], 1, 0)])
    H1 = h2.H2Oracle(x1, t1, order=c1.order, leaf=c1.leaf, eta=c1.eta)
    H1.apply(u)                                            # builds the pieces once
    R1 = None
    if recompress_eps:
        t0 = time.perf_counter()
        R1 = recompress.Recompressed(H1, recompress_eps)
        R1.apply(u)
        t_r1 = time.perf_counter() - t0
    with threadpool_limits(limits=cores):
        td, th, tr = [], [], []
        for _ in range(3):
            t0 = time.perf_counter()
            _ = u @ M.T
            td.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            H1.apply(u)
            th.append(time.perf_counter() - t0)
            if R1 is not None:
                t0 = time.perf_counter()
                R1.apply(u)
                tr.append(time.perf_counter() - t0)
    del M, H1
    out["direct"] = {"sphere_l4": {"nodes": int(x1.shape[0]), "rhs": 2, "dense_matvec_s_median": float(np.median(td)),
                                   "h2_apply_s_median": round(float(np.median(th)), 4),
                                   "h2_GDOF_s": x1.shape[0] * 2 / float(np.median(th)) / 1e9}}
    if R1 is not None:
        out["direct"]["sphere_l4"].update({"recompressed_apply_s_median": round(float(np.median(tr)), 4),
                                           "recompressed_GDOF_s": x1.shape[0] * 2 / float(np.median(tr)) / 1e9,
                                           "recompression_build_s": round(t_r1, 2),
                                           "recompress_eps": recompress_eps})
    if direct_c2:
        c2 = cases.CASES["sphere_l7"]
        # the plain interpolation matrix when the benchmarked operator is its recompression
        dmax_c2 = 0 if recompress_eps else default_dense_far_max(c2.order, DEFAULT_COUPLING)
        out["direct"]["sphere_l7"] = oracle_direct("sphere_l7", cores, dmax_c2)
    return out


def serve_bench(n_requests: int = 512, rate_hz: float = 200.0, n_slots: int = 4, coupling: str = "stored",
                dense_far: bool = False, recompress_eps: float = 0.0, evicting: bool = False) -> dict:
    """The serving mix: Poisson arrivals of 1..16-column requests over six meshes.

    Spheres (levels 4-7), the thin film and a torus, FP32 operators.  The HBM
    budget holds every operator plus the slot workspaces (they take a few GB
    of the 288), or, with `evicting`, the largest operator and 90 % of the
    operators' bytes but not all at once, so idle ones are offloaded and
    reloaded over PCIe.
    """
    from paper_1811_05731_amd import serving
    from workloads import cases, rhs

    backend = serving.GpuBackend(0)
    specs = []
    for spec, order, leaf in cases.SERVING_MESHES:
        xyz, tri = cases.mesh_of(spec)
        specs.append(serving.MeshSpec(spec.name, xyz, tri, order=order, leaf=leaf, eta=2.0, precision="fp32",
                                      coupling=coupling, dense_far_max=order ** 6 if dense_far else 0,
                                      recompress_eps=recompress_eps))
    srv = serving.Server(backend, 0, n_slots=n_slots, max_batch_rhs=64)
    for s in specs:
        srv.add_mesh(s)
    resident = [m.resident_bytes for m in srv.meshes.values()]
    # evicting: the film alone is ~80 % of all operators, and a budget below
    # 90 % would hold the film and nothing else, so every switch to or from it
    # would reload it
    budget = srv.fixed_bytes() + (max(max(resident), int(0.9 * sum(resident))) if evicting else sum(resident))
    srv.budget = budget
    t0 = time.perf_counter()
    srv.prewarm()
    prewarm_s = time.perf_counter() - t0
    reqs = []
    for q, (arr, mi, nr, seed) in enumerate(rhs.poisson_requests(n_requests, rate_hz, len(specs), 16, seed=1)):
        s = specs[mi]
        reqs.append(serving.Request(q, s.mesh_id, np.random.default_rng(seed).normal(size=(nr, s.n_nodes)), arr))
    st = srv.run(reqs)
    srv.close()
    return {"requests": st["requests"], "served": st["served"], "p50_ms": round(st["p50_ms"], 3),
            "p99_ms": round(st["p99_ms"], 3), "max_ms": round(st["max_ms"], 3),
            "throughput_req_s": round(st["throughput_req_s"], 2),
            "throughput_GDOF_s": round(st["throughput_GDOF_s"], 4), "batches": st["batches"],
            "budget_GB": round(budget / 1e9, 2), "operators_GB": round(sum(resident) / 1e9, 2),
            "slots_GB": round(srv.fixed_bytes() / 1e9, 2),
            "budget": "90 % of the operators (evicting)" if evicting else "every operator resident",
            "slots": n_slots, "precision": "fp32", "coupling": coupling, "dense_far_max": "k^2" if dense_far else 0,
            "recompress_eps": recompress_eps,
            "rate_hz": rate_hz, "prewarm_s": round(prewarm_s, 2),
            "reloads": sum(st["reloads"].values()), "offloads": sum(st["offloads"].values()),
            "breakdown_ms": st["breakdown_ms"]}


def fem_bench(reps: int = 3) -> dict:
    """Whole field evaluations (Section 2: the Neumann solve for u1, the boundary
    operator, the Dirichlet solve for u2, H and the energy) on a 10:20:1
    rectangular prism, the paper's test body, cut into 100 x 200 x 10 cells of
    six tetrahedra (1.2 million tetrahedra, seeded interior jitter of 0.1
    cell).  The boundary operator is the benchmarked representation (FP32,
    recompressed at 1e-6; order 4, leaf 64).  Uniform magnetisations along
    the three axes give the demagnetising factors; their sum should be 1."""
    import torch

    from paper_1811_05731_amd import h2dlp
    from workloads import volume
    lx, ly, lz, nx, ny, nz = 2.0, 4.0, 0.2, 100, 200, 10
    xyz, tets = volume.box_tets(lx, ly, lz, nx, ny, nz, jitter=0.1, seed=0)
    t0 = time.perf_counter()
    f = h2dlp.FemField(xyz, tets, order=4, leaf=64, eta=2.0, precision="fp32", recompress_eps=1e-6)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    vol = lx * ly * lz
    dh = torch.empty((len(tets), 3), dtype=torch.float64, device="cuda")
    out = {"workload": f"prism {lx:g} x {ly:g} x {lz:g} (10:20:1), {nx} x {ny} x {nz} cells of 6 tetrahedra, "
                       "interior jitter 0.1 cell; boundary operator FP32 recompressed at 1e-6, order 4, leaf 64",
           "nodes": int(len(xyz)), "tets": int(len(tets)), "boundary_nodes": int(f.n_boundary),
           "stiffness_entries": int(f.nnz), "build_s": round(build_s, 2),
           "boundary_operator_GB": round(f.boundary_stats.bytes_resident / 1e9, 3),
           "fem_device_GB": round(f.device_bytes / 1e9, 3)}
    factors = {}
    for axis, d in (("x", (1, 0, 0)), ("y", (0, 1, 0)), ("z", (0, 0, 1))):
        dm = torch.tensor(volume.uniform_m(len(tets), d), device="cuda")
        ts, r = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            r = f.field(dm, dh, tol=1e-10)
            ts.append(time.perf_counter() - t0)
        factors[axis] = 2.0 * r.energy / vol
        out[f"uniform_{axis}"] = {"energy": r.energy, "demag_factor": round(factors[axis], 6),
                                  "cg_iterations": [r.iters_u1, r.iters_u2],
                                  "field_ms_median": round(1e3 * float(np.median(ts)), 2)}
    out["demag_factor_sum"] = round(sum(factors.values()), 6)
    dm = torch.tensor(volume.vortex_m(xyz, tets, core=0.2, seed=0), device="cuda")
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = f.field(dm, dh, tol=1e-10)
        ts.append(time.perf_counter() - t0)
    out["vortex"] = {"energy": r.energy, "cg_iterations": [r.iters_u1, r.iters_u2],
                     "field_ms_median": round(1e3 * float(np.median(ts)), 2)}
    f.close()
    return out


MFMA_PEAK_TFS = {"fp32": 157.3, "fp64": 78.6}     # dense MFMA peaks of MI355X


def coupling_flops(st) -> float:
    """Algorithmic flops of one coupling launch on 16 right-hand sides: 2 k^2 per column and block."""
    return 2.0 * st.coupling_entries * RHS_PER_PASS


def near_field_alg_bytes(st, elem: int, n_nodes: int) -> int:
    """Algorithmic bytes of the near-field pair of launches (16 columns): the
    diagonal kernel reads x64 and D and the FP64 near-singular entries and
    writes y64; the near-field product reads its blocks and x once and adds
    into y64 (read and written).  st.bytes_near holds the blocks, the
    near-singular entries and their offsets."""
    vec = n_nodes * RHS_PER_PASS * (8 + 8 + elem + 16) + 8 * n_nodes
    return st.bytes_near + vec


def near_field_roofline(st, prec: str, kernels: dict, n_nodes: int, applies: int) -> dict:
    """Roofline record of the near-field kernel from its HIP-event time.  A
    "launch" is the kind's launches of one apply (the diagonal and the two
    near-field launches, the second after the first coupling launch): their
    HIP-event intervals summed over `applies` applies, divided by them."""
    ms_, n_ = kernels["near_field"]
    avg = ms_ / max(applies, 1)
    b = near_field_alg_bytes(st, 8 if prec == "fp64" else 4, n_nodes)
    ach = b / (avg * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "near_field", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": b, "avg_launch_ms": round(avg, 4),
            "event_intervals_per_apply": round(n_ / max(applies, 1), 2),
            "roofline_ms": round(b / HBM_PEAK_GBS / 1e6, 4)}


def roofline_of(st, prec: str, coupling: str, kernels: dict, n_nodes: int, applies: int) -> dict:
    """Roofline record of the coupling kernel from its HIP-event time (one
    interval per apply around its launches: two when recompressed)."""
    cpl_ms, cpl_n = kernels["coupling"]
    avg = cpl_ms / max(applies, 1)
    ev = 8 if prec == "fp64" else 4
    if coupling == "generated":            # no coupling bytes: bound by the MFMA pipe
        fl = coupling_flops(st)
        ach = fl / (avg * 1e-3) / 1e12
        peak = MFMA_PEAK_TFS[prec]
        return {"bound": "mfma", "kernel": "coupling", "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4), "alg_flops_per_launch": fl, "avg_launch_ms": round(avg, 4),
                "roofline_ms": round(fl / peak / 1e9, 4)}
    es = {"fp64": 8, "bf16x6": 6}.get(prec, 4)
    b = coupling_alg_bytes(st, es, ev)
    ach = b / (avg * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "coupling", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": b, "avg_launch_ms": round(avg, 4),
            "roofline_ms": round(b / HBM_PEAK_GBS / 1e6, 4)}


def apply_roofline(st, prec: str, n_nodes: int, nrhs: int, ms: float, coupling: str) -> dict:
    """The whole apply against its own roofline: its algorithmic bytes at
    8 TB/s or its MFMA flops at the precision's dense peak, whichever takes
    longer.  Flops: 2 per entry and column of every block the apply
    multiplies (coupling, exact blocks, both leaf bases); bytes as
    apply_alg_bytes."""
    elem = 8 if prec == "fp64" else 4
    b = apply_alg_bytes(st, elem, n_nodes, nrhs)
    entries = st.coupling_entries + st.near_entries + st.dense_far_entries + st.bytes_bases // elem
    f = 2.0 * entries * nrhs
    peak = MFMA_PEAK_TFS["fp64" if prec == "fp64" else "fp32"]
    t_b, t_f = b / HBM_PEAK_GBS / 1e6, f / peak / 1e9
    return {"alg_bytes": b, "alg_flops": f, "hbm_ms": round(t_b, 4), "mfma_ms": round(t_f, 4),
            "bound": "hbm" if t_b >= t_f else "mfma", "roofline_ms": round(max(t_b, t_f), 4),
            "frac": round(max(t_b, t_f) / ms, 4)}


def rel_err(a, ref) -> float:
    """Largest relative l2 error over the right-hand sides (rows)."""
    return float(f"{np.max(np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)):.3e}")


def other_workload(name: str, configs, steps: int = 10, warmup: int = 2, dense_rows=None) -> dict:
    """Time and check the named workload in each (precision, coupling,
    dense_far_max, recompress_eps) of `configs` with its own right-hand sides;
    each result against the FP64 result of the same operator (a recompressed
    one also against the FP64 interpolation matrix), and against exact dense
    rows when given (rows, values)."""
    import torch

    from paper_1811_05731_amd import h2dlp
    case, xyz, tri = workload(name)
    n = xyz.shape[0]
    u1, rhs_text = case_rhs(case, xyz)
    d1 = torch.tensor(u1, device="cuda:0")
    d2 = torch.empty_like(d1)
    res, outs = {"workload": describe(case, n, tri.shape[0], rhs_text), "nodes": n, "rhs": u1.shape[0]}, {}

    def key(prec, cpl, dmax, eps):
        return f"{prec}_{cpl}_{dmax}" + (f"_recompressed_{eps:g}" if eps else "")

    for prec, cpl, dmax, eps in configs:
        op = h2dlp.Operator(xyz, tri, order=case.order, leaf=case.leaf, eta=case.eta, precision=prec, device=0,
                            coupling=cpl, dense_far_max=dmax, recompress_eps=eps)
        ms, _ = time_path(op, d1, d2, steps, warmup, None)
        outs[(prec, cpl, dmax, eps)] = d2.cpu().numpy()
        res[key(prec, cpl, dmax, eps)] = {"value": round(n * u1.shape[0] / (ms * 1e-3) / 1e9, 4),
                                          "ms_per_step": round(ms, 4),
                                          "resident_GB": round(op.stats.bytes_resident / 1e9, 3)}
        op.close()
    for (prec, cpl, dmax, eps), val in outs.items():
        rec = res[key(prec, cpl, dmax, eps)]
        # against the FP64 result of the same operator (same exact-block
        # threshold and recompression tolerance)
        ref = next((v for (p, c, d, e), v in outs.items() if p == "fp64" and d == dmax and e == eps), None)
        if ref is not None and prec != "fp64":
            rec["vs_fp64_gpu_rel_err"] = rel_err(val, ref)
        if eps:
            ref0 = next((v for (p, c, d, e), v in outs.items() if p == "fp64" and d == 0 and e == 0), None)
            if ref0 is not None:
                rec["vs_fp64_interpolation_rel_err"] = rel_err(val, ref0)
        if dense_rows is not None:
            rows, vals = dense_rows
            rec["vs_dense_rows_rel_err"] = [float(f"{e:.3e}") for e in
                                            np.linalg.norm(val[:, rows] - vals, axis=1) / np.linalg.norm(vals, axis=1)]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sphere_l8")
    ap.add_argument("--precision", default="fp32", choices=("fp32", "fp64"))
    ap.add_argument("--coupling", default=DEFAULT_COUPLING, choices=("stored", "generated"))
    ap.add_argument("--dense-far-max", type=int, default=-1,
                    help="admissible blocks with |t||s| <= this are stored exactly (0: the plain H2 matrix; "
                         "-1: where that is cheaper -- k^2 with stored coupling, k^2/2 with generated coupling)")
    ap.add_argument("--recompress-eps", type=float, default=DEFAULT_RECOMPRESS_EPS,
                    help="recompress the bases to adaptive ranks at this relative tolerance (0: the interpolation "
                         "bases); needs stored coupling")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-cpu-c2", action="store_true", help="skip the direct oracle apply at 163842 nodes")
    ap.add_argument("--no-variants", action="store_true", help="skip the other precisions and coupling modes")
    ap.add_argument("--no-workloads", action="store_true", help="skip the 163842-node sphere and the film")
    ap.add_argument("--copy-calibration", action="store_true", help="also run a 1 GiB device copy (counter scale)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--no-fem", action="store_true", help="skip the finite-element field evaluations")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the apply shards by target "
              "rows with one all-gather of u1; that path is a design, not built here)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1811_05731_amd import h2dlp

    case, xyz, tri = workload(args.workload)
    n = xyz.shape[0]
    nrhs = case.nrhs
    u1, rhs_text = case_rhs(case, xyz)
    dev = torch.device("cuda:0")
    d_u1 = torch.tensor(u1, device=dev)
    d_u2 = torch.empty_like(d_u1)

    dense_far_max = args.dense_far_max if args.dense_far_max >= 0 else default_dense_far_max(case.order, args.coupling)

    def dmax_of(coupling):
        return args.dense_far_max if args.dense_far_max >= 0 else default_dense_far_max(case.order, coupling)

    rec_eps = args.recompress_eps
    if rec_eps > 0 and args.dense_far_max < 0:
        dense_far_max = 0                          # the recompression replaces the exact small blocks

    def build(prec, coupling, dmax=None, eps=0.0, row_basis="stored"):
        return h2dlp.Operator(xyz, tri, order=case.order, leaf=case.leaf, eta=case.eta, precision=prec, device=0,
                              coupling=coupling, dense_far_max=dmax_of(coupling) if dmax is None else dmax,
                              recompress_eps=eps, row_basis=row_basis)

    t0 = time.perf_counter()
    op = build(args.precision, args.coupling, dense_far_max, rec_eps)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    st = op.stats
    elem = 8 if args.precision == "fp64" else 4
    print(f"# built {case.name} {args.precision} {args.coupling}: N={n} clusters={st.n_clusters} far={st.n_far} "
          f"near={st.n_near} resident={st.bytes_resident / 1e9:.2f} GB in {build_s:.1f} s", file=sys.stderr, flush=True)

    # timed region: HIP events around the coupling and near-field launches only
    # (the two candidates for the roofline kernel); the per-kind breakdown comes
    # from a separate profiled pass
    ms, kernels = time_path(op, d_u1, d_u2, args.steps, args.warmup, profile=("coupling", "near_field"))
    u2_main = d_u2.cpu().numpy()
    ms_median = median_apply_ms(op, d_u1, d_u2, max(20, args.steps))
    _, breakdown = time_path(op, d_u1, d_u2, 5, 0, profile=True)
    diag_main = op.export_diagonal()
    value = n * nrhs / (ms * 1e-3) / 1e9
    # the dominant kernel is the one with the longer roofline time (its
    # algorithmic work at its roofline's peak); both records are reported
    rooflines = {"coupling": roofline_of(st, args.precision, args.coupling, kernels, n, args.steps),
                 "near_field": near_field_roofline(st, args.precision, kernels, n, args.steps)}
    dominant = max(rooflines, key=lambda k_: rooflines[k_]["roofline_ms"])
    for kind, roof_k in rooflines.items():
        roof_k["traffic"] = None
        if os.path.exists(TRAFFIC_FILE):
            for rec in json.load(open(TRAFFIC_FILE))["records"]:
                if rec.get("kernel_hash") == kernel_hash() and rec.get("kind", "coupling") == kind \
                        and rec.get("precision") == args.precision and rec.get("workload") == args.workload \
                        and rec.get("coupling") == args.coupling and rec.get("dense_far_max", 0) == dense_far_max \
                        and rec.get("recompress_eps", 0.0) == rec_eps:
                    roof_k["traffic"] = rec.get("bytes_per_launch")
    roof = rooflines[dominant]
    b_apply = apply_alg_bytes(st, elem, n, nrhs)
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "ms_per_step_median": round(ms_median, 4),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": describe(case, n, tri.shape[0], rhs_text, dense_far_max, args.coupling, rec_eps),
                   "nodes": n, "rhs": nrhs, "order": case.order, "leaf": case.leaf, "eta": case.eta,
                   "precision": args.precision, "coupling": args.coupling, "dense_far_max": dense_far_max,
                   "recompress_eps": rec_eps},
        "roofline": roof,
        "rooflines": rooflines,
        "apply_roofline": apply_roofline(st, args.precision, n, nrhs, ms, args.coupling),
        "apply_hbm_frac": round(b_apply / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "copy_GBps": None,
        "apply_alg_bytes": b_apply,
        "kernel_ms_per_apply": {k: round(v[0] / 5, 4) for k, v in breakdown.items()},
        "operator": {"clusters": st.n_clusters, "far_blocks": st.n_far, "near_blocks": st.n_near,
                     "far_blocks_dense": st.n_far_dense, "dense_far_entries": st.dense_far_entries,
                     "coupling_bytes": st.bytes_coupling, "near_bytes": st.bytes_near,
                     "resident_bytes": st.bytes_resident, "compression": round(st.compression, 5),
                     "bytes_per_dof": round(st.bytes_resident / n, 1),
                     "rank_mean_row": round(st.rank_sum_row / st.n_clusters, 2),
                     "rank_mean_col": round(st.rank_sum_col / st.n_clusters, 2),
                     "build_s": round(build_s, 2)},
        "kernel_hash": kernel_hash(),
    }
    if getattr(case.mesh, "kind", "") == "icosphere":
        out["sphere_check"] = sphere_check(op, xyz, dev)
    op.close()
    copy_gbs = copy_bandwidth(dev)
    out["copy_GBps"] = round(copy_gbs, 1)
    out["apply_copy_frac"] = round(b_apply / (ms * 1e-3) / 1e9 / copy_gbs, 4)

    if not args.no_variants:
        print("# other precisions and representations", file=sys.stderr, flush=True)
        variants, outs = {}, {}
        # each in the benchmark's configuration of its coupling mode, and the
        # plain interpolation H2 matrix (no exact admissible blocks); the last
        # two regenerate the leaf row bases in the apply
        configs = [("fp64", "stored", None, 0.0), ("fp64", "generated", None, 0.0), ("fp32", "stored", None, 0.0),
                   ("fp32", "generated", None, 0.0), ("bf16x3", "stored", None, 0.0), ("bf16x6", "stored", None, 0.0),
                   ("fp64", "generated", 0, 0.0), ("fp32", "generated", 0, 0.0), ("bf16x3", "stored", 0, 0.0),
                   ("fp64", "stored", 0, 1e-6), ("fp32", "stored", 0, 1e-6)]
        configs = [c + ("stored",) for c in configs] + [("fp32", "generated", None, 0.0, "generated"),
                                                        ("fp32", "generated", 0, 0.0, "generated")]
        for prec, cpl, dm, eps, rb in configs:
            dmax = dmax_of(cpl) if dm is None else dm
            if (prec, cpl, dmax, eps, rb) == (args.precision, args.coupling, dense_far_max, rec_eps, "stored"):
                continue
            if (prec.startswith("bf16") or cpl == "generated" or eps > 0) and case.order > 5:
                continue
            t0 = time.perf_counter()
            opv = build(prec, cpl, dmax, eps, rb)
            torch.cuda.synchronize()
            bs = time.perf_counter() - t0
            nv = max(3, args.steps // 2)
            msv, kv = time_path(opv, d_u1, d_u2, nv, args.warmup, profile=("coupling",))
            key = ((prec if cpl == "stored" else f"{prec}_generated") + ("_plain" if dm == 0 and dmax == 0 and not eps
                                                                        else "")
                   + ("_recompressed" if eps else "") + ("_regenerated_v" if rb == "generated" else ""))
            outs[key] = d_u2.cpu().numpy()
            ev = 8 if prec == "fp64" else 4
            variants[key] = {"value": round(n * nrhs / (msv * 1e-3) / 1e9, 4), "ms_per_step": round(msv, 4),
                             "dense_far_max": dmax, "recompress_eps": eps, "row_basis": rb, "build_s": round(bs, 2),
                             "coupling": roofline_of(opv.stats, prec, cpl, kv, n, nv),
                             "resident_GB": round(opv.stats.bytes_resident / 1e9, 2),
                             "apply_hbm_frac": round(apply_alg_bytes(opv.stats, ev, n, nrhs) / (msv * 1e-3) / 1e9
                                                     / HBM_PEAK_GBS, 4),
                             "apply_roofline": apply_roofline(opv.stats, prec, n, nrhs, msv, cpl)}
            opv.close()
        # each result against the FP64 result of the same operator (the same
        # exact-block threshold: both coupling modes give the same operator)
        # references: the FP64 result of each operator (exact-block threshold
        # and recompression; both coupling modes give the same operator)
        fp64_of = {}
        for key, val in outs.items():
            if key.startswith("fp64"):
                fp64_of.setdefault((variants[key]["dense_far_max"], variants[key]["recompress_eps"]), val)
        if args.precision == "fp64":
            fp64_of[(dense_far_max, rec_eps)] = u2_main

        def rel(a, ref):
            return None if ref is None else rel_err(a, ref)

        def rel_k(a, ref):
            # the same error relative to |K u1| (without the diagonal)
            if ref is None:
                return None
            k_ref = ref - diag_main[None, :] * u1
            return float(f"{np.max(np.linalg.norm(a - ref, axis=1) / np.linalg.norm(k_ref, axis=1)):.3e}")

        if args.precision != "fp64":
            ref = fp64_of.get((dense_far_max, rec_eps))
            out["vs_fp64_gpu_rel_err"] = rel(u2_main, ref)
            out["vs_fp64_gpu_rel_err_of_K"] = rel_k(u2_main, ref)
        if rec_eps:
            # the recompressed operator against the FP64 interpolation matrix it came from
            ref = fp64_of.get((0, 0.0))
            out["vs_fp64_interpolation_rel_err"] = rel(u2_main, ref)
            out["vs_fp64_interpolation_rel_err_of_K"] = rel_k(u2_main, ref)
        for key, val in outs.items():
            v = variants[key]
            ref = fp64_of.get((v["dense_far_max"], v["recompress_eps"]))
            if ref is not val:
                v["vs_fp64_gpu_rel_err"] = rel(val, ref)
                v["vs_fp64_gpu_rel_err_of_K"] = rel_k(val, ref)
            if v["recompress_eps"]:
                v["vs_fp64_interpolation_rel_err"] = rel(val, fp64_of.get((0, 0.0)))
        out["variants"] = variants

    if not args.no_workloads and args.workload == "sphere_l8":
        print("# the 163842-node sphere and the film", file=sys.stderr, flush=True)
        g = np.load(os.path.join(ROOT, "tests", "golden", "sphere_l7_dense_rows.npz"))
        c2 = workload("sphere_l7")[0]
        k2 = c2.order ** 6
        out["sphere_l7"] = other_workload("sphere_l7", [("fp32", "generated", k2 // 2, 0.0),
                                                        ("fp64", "generated", k2 // 2, 0.0),
                                                        ("fp32", "stored", 0, 0.0), ("fp64", "stored", 0, 0.0),
                                                        ("fp32", "stored", 0, 1e-6), ("fp64", "stored", 0, 1e-6)],
                                          dense_rows=(g["rows"], g["values"]))
        c3 = workload("film")[0]
        k2 = c3.order ** 6
        out["film"] = other_workload("film", [("fp32", "generated", k2 // 2, 0.0), ("fp64", "generated", k2 // 2, 0.0),
                                              ("fp32", "stored", 0, 0.0), ("fp64", "stored", 0, 0.0),
                                              ("fp32", "stored", 0, 1e-6), ("fp64", "stored", 0, 1e-6)])

    if not args.no_fem and args.workload == "sphere_l8":
        print("# finite-element field evaluations", file=sys.stderr, flush=True)
        out["fem"] = fem_bench()

    if not args.no_serve:
        print("# serving the mixed request stream", file=sys.stderr, flush=True)
        # serving keeps operators small (reloads cross PCIe): the benchmarked
        # representation without exact admissible blocks
        out["serving"] = serve_bench(coupling=args.coupling, dense_far=False, recompress_eps=rec_eps)
        out["serving_evicting"] = serve_bench(coupling=args.coupling, dense_far=False, recompress_eps=rec_eps,
                                              evicting=True)

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)        # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = a.numel() * 4

    if not args.no_cpu:
        print("# timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(xyz, tri, case, nrhs, dense_far_max, direct_c2=not args.no_cpu_c2,
                                           recompress_eps=rec_eps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
