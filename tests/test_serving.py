"""The continuous-batching scheduler on a CPU stand-in backend (no GPU).

The stand-in applies a fixed random matrix per mesh with a simulated service
time, tracks "device" bytes, and can be told to fail; the scheduler under test
is the same code the GPU backend runs.
"""
import numpy as np
import pytest

from paper_1811_05731_amd.serving import Backend, MeshSpec, Request, Server


class FakeOp:
    def __init__(self, n, seed):
        self.M = np.random.default_rng(seed).normal(size=(n, n)) / n
        self.on_device = True


class FakeBackend(Backend):
    def __init__(self, sizes, service_s=0.002, fail_launch_on=None):
        self.sizes = sizes                  # mesh_id -> (resident bytes, workspace bytes)
        self.service_s = service_s
        self.fail_launch_on = fail_launch_on
        self.device_bytes = 0
        self.peak_device_bytes = 0
        self.log = []
        import time
        self.clock = time.perf_counter

    def plan_bytes(self, spec):
        return self.sizes[spec.mesh_id]

    def _grow(self, b):
        self.device_bytes += b
        self.peak_device_bytes = max(self.peak_device_bytes, self.device_bytes)

    def build(self, spec):
        self.log.append(("build", spec.mesh_id))
        self._grow(self.sizes[spec.mesh_id][0])
        op = FakeOp(spec.n_nodes, hash(spec.mesh_id) % 1000)
        op.mesh_id = spec.mesh_id
        return op

    def offload(self, op):
        self.log.append(("offload", op.mesh_id))
        op.on_device = False
        self.device_bytes -= self.sizes[op.mesh_id][0]

    def reload(self, op, slot=None):
        self.log.append(("reload", op.mesh_id))
        op.on_device = True
        self._grow(self.sizes[op.mesh_id][0])

    def free(self, op):
        if op.on_device:
            self.device_bytes -= self.sizes[op.mesh_id][0]

    def make_slots(self, n, workspace_bytes, max_values=0):
        self._grow(n * workspace_bytes)
        return [{"id": q} for q in range(n)]

    def launch(self, slot, op, parts):
        u1 = np.concatenate(parts, axis=0)
        assert op.on_device, "apply on an operator that is not resident"
        if self.fail_launch_on is not None and op.mesh_id == self.fail_launch_on:
            raise RuntimeError("injected launch failure")
        self.log.append(("launch", op.mesh_id, u1.shape[0]))
        return (self.clock() + self.service_s, u1 @ op.M.T)

    def poll(self, ticket):
        return self.clock() >= ticket[0]

    def collect(self, ticket):
        return ticket[1]

    def timings(self, ticket):
        return {"reload": 0.0, "h2d": 0.0, "apply": 1e3 * self.service_s, "d2h": 0.0}


def _specs(sizes_nodes):
    return [MeshSpec(mid, np.zeros((n, 3)), np.zeros((1, 3), np.int32)) for mid, n in sizes_nodes]


def _requests(n_req, meshes, rate, seed=1, max_rhs=4):
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, n_req))
    out = []
    for q in range(n_req):
        mid, n = meshes[g.integers(len(meshes))]
        r = int(g.integers(1, max_rhs + 1))
        out.append(Request(q, mid, g.normal(size=(r, n)), float(t[q])))
    return out


MESHES = [("a", 30), ("b", 50), ("c", 20)]
SIZES = {"a": (300, 10), "b": (500, 10), "c": (200, 10)}


def test_all_served_and_equal_to_alone():
    be = FakeBackend(SIZES)
    srv = Server(be, budget_bytes=10_000, n_slots=2)
    for s in _specs(MESHES):
        srv.add_mesh(s)
    reqs = _requests(80, MESHES, rate=2000.0)
    stats = srv.run(reqs)
    assert stats["served"] == 80 and stats["rejected"] == 0
    ops = {m.spec.mesh_id: m.op for m in srv.meshes.values()}
    for r in reqs:
        alone = np.atleast_2d(r.u1) @ ops[r.mesh_id].M.T
        np.testing.assert_allclose(r.result, alone, rtol=0, atol=1e-13)   # BLAS blocking differs by batch
        assert r.latency is not None and r.latency >= 0
    assert stats["batches"] < 80                      # same-mesh requests were coalesced
    assert np.isfinite(stats["p50_ms"]) and stats["p99_ms"] >= stats["p50_ms"]
    # latency parts: queue, device phases, the rest; each request's parts sum to its latency
    b = stats["breakdown_ms"]
    assert set(b) == {"queue", "reload", "h2d", "apply", "d2h", "other"}
    assert b["apply"]["p50"] == pytest.approx(1e3 * be.service_s)
    assert all(v["p99"] >= v["p50"] for v in b.values())
    for r in reqs:
        assert r.latency >= r.launched - r.arrival >= 0
        assert r.done - r.launched >= sum(r.timing.values()) * 1e-3 - 1e-4     # the service time elapsed


def test_batches_respect_column_limit_and_mesh():
    be = FakeBackend(SIZES, service_s=0.01)
    srv = Server(be, budget_bytes=10_000, n_slots=1, max_batch_rhs=5)
    for s in _specs(MESHES):
        srv.add_mesh(s)
    reqs = [Request(q, "a", np.ones((2, 30)) * q, 0.0) for q in range(6)]
    srv.run(reqs)
    launches = [e for e in be.log if e[0] == "launch"]
    assert all(e[1] == "a" and e[2] <= 5 for e in launches)
    assert [e[2] for e in launches] == [4, 4, 4]         # all arrive at once: whole requests, <= 5 columns


def test_budget_forces_offload_and_reload():
    be = FakeBackend(SIZES)
    # budget holds slots + one or two operators but never all three
    srv = Server(be, budget_bytes=20 + 650, n_slots=2)
    for s in _specs(MESHES):
        srv.add_mesh(s)
    reqs = _requests(120, MESHES, rate=500.0, seed=3)
    stats = srv.run(reqs)
    assert stats["served"] == 120
    assert sum(stats["offloads"].values()) > 0 and sum(stats["reloads"].values()) > 0
    assert be.peak_device_bytes <= 670
    assert sum(stats["builds"].values()) == 3            # offloaded operators come back without a rebuild


def test_bad_requests_are_rejected_others_served():
    be = FakeBackend(SIZES)
    srv = Server(be, budget_bytes=10_000, n_slots=2)
    for s in _specs(MESHES):
        srv.add_mesh(s)
    good = _requests(20, MESHES, rate=1000.0)
    bad = [Request(100, "zzz", np.ones((1, 30)), 0.001),
           Request(101, "a", np.ones((1, 31)), 0.001),
           Request(102, "b", np.full((2, 50), np.nan), 0.002)]
    stats = srv.run(good + bad)
    assert stats["rejected"] == 3 and stats["served"] == 20
    assert all(r.error for r in bad) and all(r.error is None for r in good)


def test_operator_above_budget_is_rejected():
    sizes = dict(SIZES, b=(5000, 10))
    be = FakeBackend(sizes)
    srv = Server(be, budget_bytes=1000, n_slots=2)
    for s in _specs(MESHES):
        srv.add_mesh(s)
    reqs = _requests(40, MESHES, rate=1000.0, seed=5)
    stats = srv.run(reqs)
    for r in reqs:
        assert (r.error is not None) == (r.mesh_id == "b")
    assert stats["served"] == sum(r.mesh_id != "b" for r in reqs)


def test_launch_failure_fails_only_that_mesh():
    be = FakeBackend(SIZES, fail_launch_on="c")
    srv = Server(be, budget_bytes=10_000, n_slots=2)
    for s in _specs(MESHES):
        srv.add_mesh(s)
    reqs = _requests(60, MESHES, rate=1000.0, seed=7)
    srv.run(reqs)
    for r in reqs:
        if r.mesh_id == "c":
            assert r.error and "injected" in r.error
        else:
            assert r.error is None and r.result is not None


def test_invalid_server_arguments():
    with pytest.raises(ValueError):
        Server(FakeBackend(SIZES), 100, n_slots=0)


def test_victim_is_smallest_operator_that_makes_room():
    be = FakeBackend(SIZES)
    srv = Server(be, budget_bytes=20 + 800, n_slots=2)
    for s in _specs(MESHES):
        srv.add_mesh(s)
    a, b, c = (srv.meshes[k] for k in "abc")
    assert srv._make_resident(a) and srv._make_resident(b)
    a.last_used, b.last_used = 2.0, 1.0            # b is least recently used, but a alone makes room
    assert srv._make_resident(c)
    assert not a.on_device and b.on_device and c.on_device
    # a (300) needs 200 more bytes: c (200) is the smallest idle operator that makes room
    assert srv._make_resident(a)
    assert not c.on_device and a.on_device and b.on_device
    # c (200) with a budget of 400 next to a and b: no idle operator alone makes
    # room for the 600 bytes over, so the largest (b) goes first, then a
    srv.budget = 20 + 400
    be.log.clear()
    assert srv._make_resident(c)
    assert [e[1] for e in be.log if e[0] == "offload"] == ["b", "a"] and c.on_device


def test_request_wider_than_batch_limit_is_rejected():
    be = FakeBackend(SIZES)
    srv = Server(be, budget_bytes=10_000, n_slots=1, max_batch_rhs=3)
    for s in _specs(MESHES):
        srv.add_mesh(s)
    reqs = [Request(0, "a", np.ones((4, 30)), 0.0), Request(1, "a", np.ones((3, 30)), 0.0)]
    stats = srv.run(reqs)
    assert reqs[0].error and reqs[1].error is None and stats["served"] == 1


def test_host_copy_and_finite_check_large_and_small():
    from paper_1811_05731_amd.serving import all_finite, copy_rows
    g = np.random.default_rng(3)
    for rows, n in ((3, 50), (16, 40000), (64, 5000)):         # below and above the threaded size
        u = g.normal(size=(rows, n))
        dst = np.empty_like(u)
        copy_rows(dst, u)
        assert np.array_equal(dst, u)
        assert all_finite(u)
        for bad in (np.nan, np.inf, -np.inf):
            v = u.copy()
            v[g.integers(rows), g.integers(n)] = bad
            assert not all_finite(v)
    w = np.full((2, 4), 1e308)                                  # finite entries whose sum overflows
    assert not all_finite(w)
