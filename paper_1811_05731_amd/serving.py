"""Continuous-batching service of boundary-operator matvec requests.

A request asks for u2 = M u1 on one of several meshes (Section 3, eq. denseMat:
in a micromagnetic run every effective-field evaluation needs one such product,
Section 1).  The server keeps operators resident on the GPU within an HBM
budget, coalesces the queued requests of one mesh into one multi-column apply,
runs up to `n_slots` applies at once on their own streams with their own
workspaces, and admits new work whenever a slot frees up -- requests that
arrive while others are on the GPU join the next batch of their mesh.
Operators that do not fit are made room for by parking idle ones in pinned
host memory and reloading them later; the victim is the smallest idle operator
whose bytes make enough room (reload time grows with size), least recently
used first among equals.  A reload is enqueued on the stream of the batch that
needs it, so the loop keeps serving resident meshes while it runs.

The scheduler is independent of the GPU: `Backend` is the interface it drives.
`GpuBackend` implements it on the HIP library; tests drive the same scheduler
with a CPU stand-in.
"""
from __future__ import annotations

import os
import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Any, Optional

import numpy as np

__all__ = ["MeshSpec", "Request", "Backend", "GpuBackend", "Server", "percentile"]


# Host-side copies and checks of large batches are split over a few threads
# (NumPy releases the GIL inside them): one thread moves ~10 GB/s, and a batch
# on a large mesh is tens of megabytes.
_PAR_BYTES = 1 << 20
_pool_lock = threading.Lock()
_pool_obj: Optional[ThreadPoolExecutor] = None


def _pool() -> ThreadPoolExecutor:
    global _pool_obj
    with _pool_lock:
        if _pool_obj is None:
            _pool_obj = ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1)))
        return _pool_obj


def _row_chunks(rows: int, nbytes: int):
    n = 1 if nbytes < _PAR_BYTES else min(rows, _pool()._max_workers)
    b = np.linspace(0, rows, n + 1).astype(int)
    return [(int(b[q]), int(b[q + 1])) for q in range(n) if b[q + 1] > b[q]]


def copy_rows(dst: np.ndarray, src: np.ndarray) -> None:
    """dst[...] = src (same 2-D shape), split by rows over the pool when large."""
    chunks = _row_chunks(src.shape[0], src.nbytes)
    if len(chunks) == 1:
        dst[...] = src
        return
    list(_pool().map(lambda c: dst[c[0]:c[1]].__setitem__(Ellipsis, src[c[0]:c[1]]), chunks))


def all_finite(u: np.ndarray) -> bool:
    """No NaN or infinity in u (a sum per row chunk: one pass, no mask array;
    a sum that overflows counts as non-finite too)."""
    def part(c):
        with np.errstate(over="ignore", invalid="ignore"):
            return np.add.reduce(u[c[0]:c[1]], axis=None)
    chunks = _row_chunks(u.shape[0], u.nbytes)
    sums = list(_pool().map(part, chunks)) if len(chunks) > 1 else [part(chunks[0])]
    return bool(np.all(np.isfinite(sums)))


@dataclass
class MeshSpec:
    mesh_id: str
    xyz: np.ndarray
    tri: np.ndarray
    order: int = 4
    leaf: int = 64
    eta: float = 2.0
    precision: str = "fp32"
    coupling: str = "stored"          # "stored" | "generated" (coupling matrices recomputed in the apply)
    dense_far_max: int = 0            # admissible blocks with |t||s| <= this kept as exact entries
    recompress_eps: float = 0.0       # > 0: bases recompressed to adaptive ranks at this tolerance (stored coupling)
    row_basis: str = "stored"         # "generated": leaf row bases evaluated in the apply (interpolation bases)

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])


@dataclass
class Request:
    rid: int
    mesh_id: str
    u1: np.ndarray                 # (r, N) float64, caller's node order
    arrival: float = 0.0           # seconds after the start of Server.run
    result: Optional[np.ndarray] = None
    error: Optional[str] = None
    done: Optional[float] = None   # seconds after the start of Server.run
    batch_id: Optional[int] = None
    launched: Optional[float] = None   # seconds after the start of Server.run: its batch went to a slot
    timing: Optional[dict] = None      # device milliseconds of its batch by phase (backend.timings)

    @property
    def nrhs(self) -> int:
        return int(np.atleast_2d(self.u1).shape[0])

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class Backend:
    """What the scheduler needs from an execution engine."""

    def plan_bytes(self, spec: MeshSpec) -> tuple:             # (resident, workspace) bytes
        raise NotImplementedError

    def build(self, spec: MeshSpec) -> Any:
        raise NotImplementedError

    def offload(self, op) -> None:
        raise NotImplementedError

    def reload(self, op, slot=None) -> None:        # may be asynchronous on the slot's stream
        raise NotImplementedError

    def free(self, op) -> None:
        raise NotImplementedError

    def make_slots(self, n: int, workspace_bytes: int, max_values: int = 0) -> list:
        raise NotImplementedError

    def staging_bytes(self, max_values: int) -> int:            # device bytes per slot beyond the workspace
        return 0

    def launch(self, slot, op, parts: list) -> Any:         # -> ticket
        """Apply op to the batch: `parts` are the requests' (r_i x n) arrays, stacked in order."""
        raise NotImplementedError

    def poll(self, ticket) -> bool:
        raise NotImplementedError

    def collect(self, ticket) -> np.ndarray:
        raise NotImplementedError

    def timings(self, ticket) -> Optional[dict]:
        """Milliseconds of a finished batch by phase (reload, h2d, apply, d2h), if measured."""
        return None


class GpuBackend(Backend):
    """The HIP library on one GPU: torch supplies streams, pinned staging and workspaces."""

    def __init__(self, device: int = 0):
        import torch

        from . import h2dlp
        self.torch = torch
        self.h2dlp = h2dlp
        self.device = torch.device("cuda", device)
        self.dev_index = device

    def plan_bytes(self, spec):
        p = self.h2dlp.plan(spec.xyz, spec.tri, spec.order, spec.leaf, spec.eta, spec.precision,
                            coupling=spec.coupling, dense_far_max=spec.dense_far_max,
                            recompress_eps=spec.recompress_eps, row_basis=spec.row_basis)
        return p.stats.bytes_resident, p.stats.workspace_bytes

    def build(self, spec):
        return self.h2dlp.Operator(spec.xyz, spec.tri, spec.order, spec.leaf, spec.eta, spec.precision,
                                   device=self.dev_index, coupling=spec.coupling, dense_far_max=spec.dense_far_max,
                                   recompress_eps=spec.recompress_eps, row_basis=spec.row_basis)

    def built_bytes(self, op):
        return op.stats.bytes_resident

    def offload(self, op):
        op.offload()

    def reload(self, op, slot=None):
        if slot is not None:                        # the reload's start, for the batch's timing
            ev = self.torch.cuda.Event(enable_timing=True)
            ev.record(slot["stream"])
            slot["reload_ev"] = ev
        op.reload(stream=None if slot is None else slot["stream"])

    def free(self, op):
        op.close()

    def staging_bytes(self, max_values):
        return 2 * 8 * max(1, max_values)

    def make_slots(self, n, workspace_bytes, max_values=0):
        """Per slot: a stream, a workspace, and pinned host and device staging
        for `max_values` input and output values (allocated once)."""
        t = self.torch
        slots = []
        for _ in range(n):
            v = max(1, max_values)
            slots.append({"stream": t.cuda.Stream(device=self.device),
                          "ws": t.empty(max(1, workspace_bytes), dtype=t.uint8, device=self.device),
                          "h_in": t.empty(v, dtype=t.float64, pin_memory=True),
                          "h_out": t.empty(v, dtype=t.float64, pin_memory=True),
                          "d_in": t.empty(v, dtype=t.float64, device=self.device),
                          "d_out": t.empty(v, dtype=t.float64, device=self.device)})
        return slots

    def launch(self, slot, op, parts):
        t = self.torch
        s = slot["stream"]
        r, n = sum(p.shape[0] for p in parts), parts[0].shape[1]
        if r * n > slot["h_in"].numel():
            raise ValueError("batch larger than the slot's staging buffers")
        h_in = slot["h_in"][:r * n].view(r, n)
        staged, c = h_in.numpy(), 0
        for p in parts:                             # each request straight into pinned memory
            copy_rows(staged[c:c + p.shape[0]], p)
            c += p.shape[0]
        d1 = slot["d_in"][:r * n].view(r, n)
        d2 = slot["d_out"][:r * n].view(r, n)
        h_out = slot["h_out"][:r * n].view(r, n)
        ev = [t.cuda.Event(enable_timing=True) for _ in range(4)]
        with t.cuda.stream(s):
            ev[0].record(s)
            d1.copy_(h_in, non_blocking=True)
            ev[1].record(s)
            op.apply(d1, d2, stream=s, workspace=slot["ws"])
            ev[2].record(s)
            h_out.copy_(d2, non_blocking=True)
            ev[3].record(s)
        return {"ev": ev, "reload_ev": slot.pop("reload_ev", None), "h_out": h_out}

    def poll(self, ticket):
        return ticket["ev"][3].query()

    def collect(self, ticket):
        ticket["ev"][3].synchronize()
        src = ticket["h_out"].numpy()
        out = np.empty(src.shape, dtype=src.dtype)
        copy_rows(out, src)
        return out

    def timings(self, ticket):
        ev, rel = ticket["ev"], ticket["reload_ev"]
        return {"reload": rel.elapsed_time(ev[0]) if rel is not None else 0.0,
                "h2d": ev[0].elapsed_time(ev[1]), "apply": ev[1].elapsed_time(ev[2]),
                "d2h": ev[2].elapsed_time(ev[3])}


@dataclass
class _Mesh:
    spec: MeshSpec
    resident_bytes: int
    workspace_bytes: int
    op: Any = None
    on_device: bool = False
    inflight: int = 0
    last_used: float = 0.0
    queue: deque = field(default_factory=deque)
    builds: int = 0
    reloads: int = 0
    offloads: int = 0


def percentile(values, q: float) -> float:
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        return float("nan")
    return float(np.percentile(v, q))


class Server:
    """Continuous batching over resident operators within an HBM budget."""

    def __init__(self, backend: Backend, budget_bytes: int, n_slots: int = 4, max_batch_rhs: int = 64,
                 aging: float = 0.05, reload_bytes_per_s: float = 20e9, clock=time.perf_counter):
        if n_slots < 1 or max_batch_rhs < 1:
            raise ValueError("n_slots and max_batch_rhs must be >= 1")
        self.backend = backend
        self.budget = int(budget_bytes)
        self.n_slots = n_slots
        self.max_batch_rhs = max_batch_rhs
        self.aging = aging
        self.reload_bytes_per_s = reload_bytes_per_s
        self.clock = clock
        self.t0 = 0.0
        self.meshes: dict = {}
        self.slots = None
        self.free_slots = []
        self.inflight = []                 # (ticket, slot, mesh, [requests], column offsets)
        self.batches = 0
        self.rejected = 0

    # -- registration and memory ----------------------------------------------------
    def add_mesh(self, spec: MeshSpec):
        resident, ws = self.backend.plan_bytes(spec)
        m = _Mesh(spec, int(resident), int(ws))
        self.meshes[spec.mesh_id] = m
        built = getattr(self.backend, "built_bytes", None)
        if spec.recompress_eps > 0 and built is not None:
            # a recompressed operator's ranks are known only once built, and the
            # plan's full-rank count can be many times its size: build it now for
            # the exact size, and park it in host memory until it is admitted
            m.op = self.backend.build(spec)
            m.builds += 1
            m.resident_bytes = int(built(m.op))
            self.backend.offload(m.op)
            m.offloads += 1

    def _max_values(self) -> int:
        return self.max_batch_rhs * max((m.spec.n_nodes for m in self.meshes.values()), default=1)

    def _slot_bytes(self) -> int:
        ws = max((m.workspace_bytes for m in self.meshes.values()), default=0)
        return self.n_slots * (ws + self.backend.staging_bytes(self._max_values()))

    def fixed_bytes(self) -> int:
        """Device bytes the slots hold whatever is resident (workspaces and staging)."""
        return self._slot_bytes()

    def _used(self) -> int:
        return self._slot_bytes() + sum(m.resident_bytes for m in self.meshes.values() if m.on_device)

    def _fits(self, m: _Mesh) -> bool:
        return self._slot_bytes() + m.resident_bytes <= self.budget

    def _patience(self, m: _Mesh) -> float:
        return self.aging + 2.0 * m.resident_bytes / self.reload_bytes_per_s

    def _victim(self, need: int) -> Optional[_Mesh]:
        """The idle operator to offload next when `need` more bytes are wanted:
        the smallest one that makes enough room on its own, else the largest
        (fewest evictions); least recently used first among equal sizes."""
        idle = [x for x in self.meshes.values() if x.on_device and x.inflight == 0]
        if not idle:
            return None
        enough = [x for x in idle if x.resident_bytes >= need]
        if enough:
            return min(enough, key=lambda x: (x.resident_bytes, x.last_used))
        return max(idle, key=lambda x: (x.resident_bytes, -x.last_used))

    def _make_resident(self, m: _Mesh, slot=None) -> bool:
        """Offload idle operators until m fits; then build m, or reload it on the slot's stream."""
        if m.on_device:
            return True
        while self._used() + m.resident_bytes > self.budget:
            victim = self._victim(self._used() + m.resident_bytes - self.budget)
            if victim is None:
                return False
            self.backend.offload(victim.op)
            victim.on_device = False
            victim.offloads += 1
        if m.op is None:
            m.op = self.backend.build(m.spec)
            m.builds += 1
        else:
            self.backend.reload(m.op, slot)
            m.reloads += 1
        m.on_device = True
        return True

    def prewarm(self):
        """Make every registered operator resident before the first request: build
        it, or reload it if it was built and parked when registered (reloads
        without a slot return when the copies are done).  Operators beyond the
        budget end up offloaded."""
        for m in self.meshes.values():
            if not m.on_device and self._fits(m):
                self._make_resident(m)

    # -- the loop -------------------------------------------------------------------
    def _reject(self, req: Request, msg: str):
        req.error = msg
        req.done = self.clock() - self.t0
        self.rejected += 1

    def _accept(self, req: Request):
        m = self.meshes.get(req.mesh_id)
        u = np.atleast_2d(req.u1)
        if m is None:
            return self._reject(req, f"unknown mesh {req.mesh_id!r}")
        if u.ndim != 2 or u.shape[1] != m.spec.n_nodes or u.shape[0] < 1:
            return self._reject(req, f"u1 must have shape (r, {m.spec.n_nodes})")
        if u.shape[0] > self.max_batch_rhs:
            return self._reject(req, f"more than max_batch_rhs = {self.max_batch_rhs} columns")
        if not all_finite(u):
            return self._reject(req, "u1 has non-finite values")
        if not self._fits(m):
            return self._reject(req, "operator larger than the HBM budget")
        m.queue.append(req)

    def _launch_ready(self, now: float) -> bool:
        launched = False
        while self.free_slots:
            waiting = [m for m in self.meshes.values() if m.queue]
            if not waiting:
                break
            # resident meshes first (no load cost); a non-resident mesh goes
            # first once its head request has waited longer than `aging` plus
            # twice its estimated reload time; then the oldest head request
            waiting.sort(key=lambda m: (not m.on_device and now - m.queue[0].arrival < self._patience(m),
                                        m.queue[0].arrival))
            started = False
            for m in waiting:
                slot = self.free_slots[-1]
                try:
                    ok = self._make_resident(m, slot)
                except Exception as e:  # build / reload failure: fail this mesh's queue
                    while m.queue:
                        self._reject(m.queue.popleft(), f"could not make operator resident: {e}")
                    continue
                if not ok:
                    continue
                batch, cols = [], 0
                while m.queue and cols + m.queue[0].nrhs <= self.max_batch_rhs:
                    r = m.queue.popleft()
                    batch.append(r)
                    cols += r.nrhs
                parts = [np.atleast_2d(r.u1) for r in batch]
                self.free_slots.pop()
                try:
                    ticket = self.backend.launch(slot, m.op, parts)
                except Exception as e:
                    self.free_slots.append(slot)
                    for r in batch:
                        self._reject(r, f"apply failed: {e}")
                    continue
                self.batches += 1
                for r in batch:
                    r.batch_id = self.batches
                    r.launched = now
                m.inflight += 1
                m.last_used = now
                self.inflight.append((ticket, slot, m, batch))
                started = launched = True
                break
            if not started:
                break
        return launched

    def _reap(self) -> bool:
        reaped = False
        keep = []
        for ticket, slot, m, batch in self.inflight:
            if self.backend.poll(ticket):
                out = self.backend.collect(ticket)
                t = self.clock()
                tm = self.backend.timings(ticket)
                c = 0
                for r in batch:
                    r.result = out[c:c + r.nrhs]
                    r.done = t - self.t0
                    r.timing = tm
                    c += r.nrhs
                m.inflight -= 1
                self.free_slots.append(slot)
                reaped = True
            else:
                keep.append((ticket, slot, m, batch))
        self.inflight = keep
        return reaped

    def run(self, requests, idle_sleep: float = 5e-5) -> dict:
        """Serve `requests` (Request objects with arrival times relative to the start)."""
        if self.slots is None:
            self.slots = self.backend.make_slots(self.n_slots, max((m.workspace_bytes for m in self.meshes.values()),
                                                                   default=1), self._max_values())
            self.free_slots = list(self.slots)
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        self.t0 = self.clock()
        start = time.perf_counter()
        while pending or self.inflight or any(m.queue for m in self.meshes.values()):
            now = self.clock() - self.t0
            progressed = False
            while pending and pending[0].arrival <= now:
                self._accept(pending.popleft())
                progressed = True
            progressed |= self._reap()
            progressed |= self._launch_ready(now)
            if not progressed:
                if pending and not self.inflight and not any(m.queue for m in self.meshes.values()):
                    time.sleep(max(0.0, min(pending[0].arrival - (self.clock() - self.t0), 0.01)))
                else:
                    time.sleep(idle_sleep)
        wall = time.perf_counter() - start
        ok = [r for r in requests if r.error is None]
        lat = [r.latency for r in ok]
        cols = sum(r.nrhs for r in ok)
        dofs = sum(r.nrhs * self.meshes[r.mesh_id].spec.n_nodes for r in ok)
        return {
            "breakdown_ms": self.breakdown(ok),
            "requests": len(requests), "served": len(ok), "rejected": len(requests) - len(ok),
            "batches": self.batches, "wall_s": wall,
            "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
            "max_ms": 1e3 * (max(lat) if lat else float("nan")),
            "throughput_req_s": len(ok) / wall if wall > 0 else float("nan"),
            "throughput_rhs_s": cols / wall if wall > 0 else float("nan"),
            "throughput_GDOF_s": dofs / wall / 1e9 if wall > 0 else float("nan"),
            "builds": {k: m.builds for k, m in self.meshes.items()},
            "reloads": {k: m.reloads for k, m in self.meshes.items()},
            "offloads": {k: m.offloads for k, m in self.meshes.items()},
        }

    @staticmethod
    def breakdown(reqs) -> dict:
        """p50 / p99 milliseconds of each part of the requests' latency: queue
        (arrival to launch), the device phases of their batch (reload, h2d,
        apply, d2h, where the backend measures them) and the rest (launch to
        result on the host minus the device phases: issue, waiting for the GPU,
        polling)."""
        parts = {"queue": [r.launched - r.arrival for r in reqs if r.launched is not None]}
        timed = [r for r in reqs if r.timing is not None and r.launched is not None]
        for k in ("reload", "h2d", "apply", "d2h"):
            parts[k] = [r.timing[k] * 1e-3 for r in timed]
        parts["other"] = [r.done - r.launched - sum(r.timing.values()) * 1e-3 for r in timed]
        return {k: {"p50": round(1e3 * percentile(v, 50), 3), "p99": round(1e3 * percentile(v, 99), 3)}
                for k, v in parts.items() if v}

    def close(self):
        for m in self.meshes.values():
            if m.op is not None:
                self.backend.free(m.op)
                m.op = None
                m.on_device = False
