"""Python binding of the h2dlp C ABI (include/h2dlp.h): argument marshalling only.

Every step of the operator runs in the HIP library ``libh2dlp.so``; this
module only converts NumPy / torch arguments into pointers and sizes.  Device
memory and streams come from PyTorch.  If the library is missing the import of
this module fails: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libh2dlp.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTSUP = 0, -1, -2, -3, -4
FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
IO_F64, IO_F32 = 0, 1
NOALLOC_SCRATCH_BYTES = 128 * 1024 * 1024      # H2DLP_NOALLOC_SCRATCH_BYTES
NKINDS = 7
KIND_NAMES = ("permute", "leaf_forward", "upward", "coupling", "downward", "leaf_output", "near_field")
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "bf16x6": BF16X6}
COUPLING = {"stored": 0, "generated": 1}        # H2DLP_COUPLING_STORED / _GENERATED
ROW_BASIS = {"stored": 0, "generated": 1}       # H2DLP_ROW_BASIS_STORED / _GENERATED


class H2dlpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"h2dlp error {code}: {msg}")
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("xyz", ctypes.POINTER(ctypes.c_double)),
                ("n_tris", ctypes.c_int64), ("tri", ctypes.POINTER(ctypes.c_int32))]


class _Volume(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("xyz", ctypes.POINTER(ctypes.c_double)),
                ("n_tets", ctypes.c_int64), ("tet", ctypes.POINTER(ctypes.c_int32))]


class _FemResult(ctypes.Structure):
    _fields_ = [("iters_u1", ctypes.c_int32), ("iters_u2", ctypes.c_int32), ("resid_u1", ctypes.c_double),
                ("resid_u2", ctypes.c_double), ("energy", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("leaf", ctypes.c_int), ("eta", ctypes.c_double),
                ("precision", ctypes.c_int), ("alpha", ctypes.c_double), ("device", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("coupling", ctypes.c_int), ("dense_far_max", ctypes.c_int64),
                ("recompress_eps", ctypes.c_double), ("row_basis", ctypes.c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_tris", ctypes.c_int64),
                ("order", ctypes.c_int32), ("leaf", ctypes.c_int32), ("k", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("n_clusters", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("n_far", ctypes.c_int64), ("n_near", ctypes.c_int64),
                ("coupling_entries", ctypes.c_int64), ("near_entries", ctypes.c_int64),
                ("nearsing_entries", ctypes.c_int64),
                ("bytes_coupling", ctypes.c_int64), ("bytes_near", ctypes.c_int64),
                ("bytes_bases", ctypes.c_int64), ("bytes_transfer", ctypes.c_int64),
                ("bytes_other", ctypes.c_int64), ("bytes_resident", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("compression", ctypes.c_double),
                ("n_far_dense", ctypes.c_int64), ("dense_far_entries", ctypes.c_int64),
                ("rank_sum_row", ctypes.c_int64), ("rank_sum_col", ctypes.c_int64),
                ("rank_max_row", ctypes.c_int32), ("rank_max_col", ctypes.c_int32)]


EXPORTED = ("h2dlp_default_options", "h2dlp_build", "h2dlp_build_ex", "h2dlp_plan", "h2dlp_apply", "h2dlp_apply_ex",
            "h2dlp_bytes", "h2dlp_info", "h2dlp_export_structure", "h2dlp_export_diagonal", "h2dlp_offload",
            "h2dlp_reload", "h2dlp_reload_ex", "h2dlp_free", "h2dlp_apply_noalloc", "h2dlp_save", "h2dlp_load",
            "h2dlp_fem_build", "h2dlp_fem_info", "h2dlp_fem_boundary_nodes", "h2dlp_fem_field", "h2dlp_fem_free",
            "h2dlp_last_error", "h2dlp_profile", "h2dlp_profile_read")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1811_05731_amd._build`")
    try:                                   # share torch's HIP runtime when torch is present
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, V, L = ctypes.POINTER, ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64
    lib.h2dlp_default_options.argtypes = [P(_Options)]
    lib.h2dlp_default_options.restype = None
    lib.h2dlp_build.argtypes = [P(_Mesh), I, I, D]
    lib.h2dlp_build.restype = V
    lib.h2dlp_build_ex.argtypes = [P(_Mesh), P(_Options), P(V)]
    lib.h2dlp_build_ex.restype = I
    lib.h2dlp_plan.argtypes = [P(_Mesh), P(_Options), P(V)]
    lib.h2dlp_plan.restype = I
    lib.h2dlp_apply.argtypes = [V, V, V, I]
    lib.h2dlp_apply.restype = I
    lib.h2dlp_apply_ex.argtypes = [V, V, V, I, I, V, V, ctypes.c_size_t]
    lib.h2dlp_apply_ex.restype = I
    lib.h2dlp_apply_noalloc.argtypes = [V, V, V, I, I, V]
    lib.h2dlp_apply_noalloc.restype = I
    lib.h2dlp_fem_build.argtypes = [P(_Volume), P(_Options), P(V)]
    lib.h2dlp_fem_build.restype = I
    lib.h2dlp_fem_info.argtypes = [V, P(L), P(L), P(ctypes.c_size_t), P(V)]
    lib.h2dlp_fem_info.restype = I
    lib.h2dlp_fem_boundary_nodes.argtypes = [V, P(L)]
    lib.h2dlp_fem_boundary_nodes.restype = I
    lib.h2dlp_fem_field.argtypes = [V, V, V, V, V, D, I, V, P(_FemResult)]
    lib.h2dlp_fem_field.restype = I
    lib.h2dlp_fem_free.argtypes = [V]
    lib.h2dlp_fem_free.restype = None
    lib.h2dlp_save.argtypes = [V, ctypes.c_char_p]
    lib.h2dlp_save.restype = I
    lib.h2dlp_load.argtypes = [ctypes.c_char_p, I, P(V)]
    lib.h2dlp_load.restype = I
    lib.h2dlp_bytes.argtypes = [V, P(ctypes.c_size_t), P(ctypes.c_size_t)]
    lib.h2dlp_bytes.restype = I
    lib.h2dlp_info.argtypes = [V, P(_Stats)]
    lib.h2dlp_info.restype = I
    lib.h2dlp_export_structure.argtypes = [V, P(L), P(L), P(D), P(L), P(L)]
    lib.h2dlp_export_structure.restype = I
    lib.h2dlp_export_diagonal.argtypes = [V, P(D)]
    lib.h2dlp_export_diagonal.restype = I
    lib.h2dlp_offload.argtypes = [V]
    lib.h2dlp_offload.restype = I
    lib.h2dlp_reload.argtypes = [V]
    lib.h2dlp_reload.restype = I
    lib.h2dlp_reload_ex.argtypes = [V, V]
    lib.h2dlp_reload_ex.restype = I
    lib.h2dlp_free.argtypes = [V]
    lib.h2dlp_free.restype = None
    lib.h2dlp_last_error.argtypes = []
    lib.h2dlp_last_error.restype = ctypes.c_char_p
    lib.h2dlp_profile.argtypes = [V, I]
    lib.h2dlp_profile.restype = I
    lib.h2dlp_profile_read.argtypes = [V, P(D), P(L), I, I]
    lib.h2dlp_profile_read.restype = I
    return lib


_lib = _load()


def _check(rc: int):
    if rc != OK:
        raise H2dlpError(rc, _lib.h2dlp_last_error().decode())


def default_options() -> dict:
    o = _Options()
    _lib.h2dlp_default_options(ctypes.byref(o))
    return {f: getattr(o, f) for f, _ in _Options._fields_}


@dataclass
class Stats:
    n_nodes: int
    n_tris: int
    order: int
    leaf: int
    k: int
    precision: int
    depth: int
    n_clusters: int
    n_leaves: int
    n_far: int
    n_near: int
    coupling_entries: int
    near_entries: int
    nearsing_entries: int
    bytes_coupling: int
    bytes_near: int
    bytes_bases: int
    bytes_transfer: int
    bytes_other: int
    bytes_resident: int
    workspace_bytes: int
    compression: float
    n_far_dense: int
    dense_far_entries: int
    rank_sum_row: int
    rank_sum_col: int
    rank_max_row: int
    rank_max_col: int


def _ptr(t) -> int:
    """Device pointer of a torch tensor (CUDA/HIP) after checking contiguity."""
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


class Operator:
    """A built H2 boundary operator resident on one GPU (owns its device memory).

    The options are those of h2dlp_options in include/h2dlp.h: precision
    ("fp64", "fp32", "bf16x3", "bf16x6"), coupling ("stored" or "generated"),
    dense_far_max (admissible blocks kept exact), recompress_eps (algebraic
    recompression to adaptive ranks) and row_basis ("stored" or "generated":
    leaf row bases evaluated in the apply).  plan_only builds the host
    structure and byte counts without a GPU."""

    def __init__(self, xyz, tri, order: int = 4, leaf: int = 32, eta: float = 2.0,
                 precision="fp64", alpha: float = 0.1, device: int = -1, stream=None, plan_only: bool = False,
                 coupling: str = "stored", dense_far_max: int = 0, recompress_eps: float = 0.0,
                 row_basis: str = "stored"):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        if xyz.ndim != 2 or xyz.shape[1] != 3 or tri.ndim != 2 or tri.shape[1] != 3:
            raise ValueError("xyz must be N x 3 and tri T x 3")
        mesh = _Mesh(xyz.shape[0], xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     tri.shape[0], tri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        opt = _Options()
        _lib.h2dlp_default_options(ctypes.byref(opt))
        opt.order, opt.leaf, opt.eta, opt.alpha, opt.device = order, leaf, eta, alpha, device
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        opt.stream = stream
        opt.coupling = COUPLING[coupling]
        opt.dense_far_max = int(dense_far_max)
        opt.recompress_eps = float(recompress_eps)
        opt.row_basis = ROW_BASIS[row_basis] if isinstance(row_basis, str) else int(row_basis)
        h = ctypes.c_void_p()
        entry = _lib.h2dlp_plan if plan_only else _lib.h2dlp_build_ex
        _check(entry(ctypes.byref(mesh), ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self._free = _lib.h2dlp_free          # kept for interpreter shutdown
        self.plan_only = plan_only
        if plan_only:
            self.device = None
        else:
            import torch
            self.device = device if device >= 0 else torch.cuda.current_device()
        self.n_nodes = xyz.shape[0]
        self.stats = self.info()

    @classmethod
    def load(cls, path, device: int = -1):
        """An operator restored from a file written by save() (h2dlp_load): no
        build, the device buffers come from the file."""
        h = ctypes.c_void_p()
        _check(_lib.h2dlp_load(os.fsencode(path), int(device), ctypes.byref(h)))
        op = cls.__new__(cls)
        op._h = h
        op._free = _lib.h2dlp_free
        op.plan_only = False
        if device >= 0:
            op.device = device
        else:
            import torch
            op.device = torch.cuda.current_device()
        op.stats = op.info()
        op.n_nodes = int(op.stats.n_nodes)
        return op

    def save(self, path):
        """Write the built operator to `path` (h2dlp_save), for Operator.load."""
        if self.plan_only:
            raise ValueError("a planned operator has nothing to save")
        _check(_lib.h2dlp_save(self._h, os.fsencode(path)))

    def close(self):
        if getattr(self, "_h", None):
            self._free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def handle(self):
        return self._h

    def info(self) -> Stats:
        s = _Stats()
        _check(_lib.h2dlp_info(self._h, ctypes.byref(s)))
        return Stats(**{f: getattr(s, f) for f, _ in _Stats._fields_})

    def bytes(self):
        r, w = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.h2dlp_bytes(self._h, ctypes.byref(r), ctypes.byref(w)))
        return r.value, w.value

    def _io_args(self, u1, u2, nrhs, stream, workspace):
        """Check the apply operands before any pointer reaches the library:
        (nrhs, io dtype, stream handle)."""
        import torch
        if self.plan_only:
            raise ValueError("a planned operator has nothing on the device")
        if u1.dtype != u2.dtype or u1.dtype not in (torch.float64, torch.float32):
            raise ValueError("u1 and u2 must both be float64 or both float32")
        if u1.dim() not in (1, 2) or u1.shape[-1] != self.n_nodes or u2.shape != u1.shape:
            raise ValueError("u1, u2 must have shape (nrhs, N) or (N,)")
        rows = u1.shape[0] if u1.dim() == 2 else 1
        nrhs = rows if nrhs is None else int(nrhs)
        if not 1 <= nrhs <= rows:
            raise ValueError(f"nrhs must be in [1, {rows}]")
        for name, t in (("u1", u1), ("u2", u2), ("workspace", workspace)):
            if t is not None and (t.device.type != "cuda" or t.device.index != self.device):
                raise ValueError(f"{name} must be on cuda:{self.device}, not {t.device}")
        io = IO_F64 if u1.dtype == torch.float64 else IO_F32
        st = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        return nrhs, io, st

    def apply(self, u1, u2, nrhs: int | None = None, stream=None, workspace=None):
        """u2 = M u1 for device tensors of shape (nrhs, N) or (N,) (float64 or
        float32, same dtype) on the operator's GPU; `nrhs` (default: all rows)
        applies to the first nrhs rows only."""
        nrhs, io, st = self._io_args(u1, u2, nrhs, stream, workspace)
        ws_ptr, ws_bytes = (None, 0) if workspace is None else (_ptr(workspace), workspace.numel() * workspace.element_size())
        _check(_lib.h2dlp_apply_ex(self._h, _ptr(u1), _ptr(u2), nrhs, io, st, ws_ptr, ws_bytes))
        return u2

    def apply_noalloc(self, u1, u2, nrhs: int | None = None, stream=None):
        """As apply(), with the workspace in the library's own device array
        (h2dlp_apply_noalloc): nothing is allocated, and calls on one GPU must
        not overlap."""
        nrhs, io, st = self._io_args(u1, u2, nrhs, stream, None)
        _check(_lib.h2dlp_apply_noalloc(self._h, _ptr(u1), _ptr(u2), nrhs, io, st))
        return u2

    def export_structure(self) -> dict:
        s = self.stats
        perm = np.empty(s.n_nodes, np.int64)
        cl = np.empty((s.n_clusters, 6), np.int64)
        boxes = np.empty((s.n_clusters, 6), np.float64)
        far = np.empty((s.n_far, 2), np.int64)
        near = np.empty((s.n_near, 2), np.int64)
        P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))  # noqa: E731
        _check(_lib.h2dlp_export_structure(self._h, P(perm, ctypes.c_int64), P(cl, ctypes.c_int64),
                                           P(boxes, ctypes.c_double), P(far, ctypes.c_int64),
                                           P(near, ctypes.c_int64)))
        return dict(perm=perm, begin=cl[:, 0], end=cl[:, 1], level=cl[:, 2], parent=cl[:, 3],
                    child0=cl[:, 4], child1=cl[:, 5], box_lo=boxes[:, :3], box_hi=boxes[:, 3:],
                    far=far, near=near)

    def export_diagonal(self) -> np.ndarray:
        d = np.empty(self.n_nodes, np.float64)
        _check(_lib.h2dlp_export_diagonal(self._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return d

    def offload(self):
        """Park the operator in pinned host memory and free its HBM."""
        _check(_lib.h2dlp_offload(self._h))

    def reload(self, stream=None):
        """Bring an offloaded operator back to the device.

        Without a stream this returns when the copies are done; with a torch
        stream the copies are only enqueued there, and every later apply waits
        for them on the device."""
        if stream is None:
            _check(_lib.h2dlp_reload(self._h))
        else:
            _check(_lib.h2dlp_reload_ex(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def profile(self, enable=True):
        """Record per-kernel HIP events: True = every kind, False = off, or an
        iterable of kind names (KIND_NAMES) to record only those."""
        if enable is True or enable is False:
            mask = (1 << NKINDS) - 1 if enable else 0
        else:
            mask = 0
            for name in enable:
                mask |= 1 << KIND_NAMES.index(name)
        _check(_lib.h2dlp_profile(self._h, mask))

    def profile_read(self, reset: bool = True) -> dict:
        ms = (ctypes.c_double * NKINDS)()
        n = (ctypes.c_int64 * NKINDS)()
        _check(_lib.h2dlp_profile_read(self._h, ms, n, NKINDS, int(reset)))
        return {KIND_NAMES[q]: (ms[q], n[q]) for q in range(NKINDS)}


@dataclass
class FemResult:
    iters_u1: int
    iters_u2: int
    resid_u1: float
    resid_u2: float
    energy: float


class FemField:
    """The magnetostatic field of a magnetised body on one GPU (h2dlp_fem_*):
    the P1 finite-element solves either side of the boundary operator."""

    def __init__(self, xyz, tet, order: int = 4, leaf: int = 32, eta: float = 2.0, precision="fp64",
                 alpha: float = 0.1, device: int = -1, coupling: str = "stored", dense_far_max: int = 0,
                 recompress_eps: float = 0.0, row_basis: str = "stored"):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tet = np.ascontiguousarray(tet, dtype=np.int32)
        if xyz.ndim != 2 or xyz.shape[1] != 3 or tet.ndim != 2 or tet.shape[1] != 4:
            raise ValueError("xyz must be N x 3 and tet T x 4")
        vol = _Volume(xyz.shape[0], xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      tet.shape[0], tet.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        opt = _Options()
        _lib.h2dlp_default_options(ctypes.byref(opt))
        opt.order, opt.leaf, opt.eta, opt.alpha, opt.device = order, leaf, eta, alpha, device
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        opt.coupling = COUPLING[coupling]
        opt.dense_far_max = int(dense_far_max)
        opt.recompress_eps = float(recompress_eps)
        opt.row_basis = ROW_BASIS[row_basis] if isinstance(row_basis, str) else int(row_basis)
        h = ctypes.c_void_p()
        _check(_lib.h2dlp_fem_build(ctypes.byref(vol), ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self._free = _lib.h2dlp_fem_free
        import torch
        self.device = device if device >= 0 else torch.cuda.current_device()
        self.n_nodes, self.n_tets = xyz.shape[0], tet.shape[0]
        nb, nnz, nbytes, op = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_void_p()
        _check(_lib.h2dlp_fem_info(h, ctypes.byref(nb), ctypes.byref(nnz), ctypes.byref(nbytes), ctypes.byref(op)))
        self.n_boundary, self.nnz, self.device_bytes = nb.value, nnz.value, nbytes.value
        self.boundary_nodes = np.empty(self.n_boundary, np.int64)
        _check(_lib.h2dlp_fem_boundary_nodes(h, self.boundary_nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        s = _Stats()
        _check(_lib.h2dlp_info(op, ctypes.byref(s)))
        self.boundary_stats = Stats(**{f: getattr(s, f) for f, _ in _Stats._fields_})

    def close(self):
        if getattr(self, "_h", None):
            self._free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def field(self, m, h, u1=None, u2=None, tol: float = 1e-12, max_iter: int = 20000, stream=None) -> FemResult:
        """H (into the device tensor h, n_tets x 3 float64) for the magnetisation m
        (device tensor, n_tets x 3 float64); u1, u2 (device tensors, n_nodes
        float64) receive the two potentials when given."""
        import torch
        for name, t, shape in (("m", m, (self.n_tets, 3)), ("h", h, (self.n_tets, 3)), ("u1", u1, (self.n_nodes,)),
                               ("u2", u2, (self.n_nodes,))):
            if t is None:
                continue
            if t.dtype != torch.float64 or tuple(t.shape) != shape:
                raise ValueError(f"{name} must be float64 of shape {shape}")
            if t.device.type != "cuda" or t.device.index != self.device:
                raise ValueError(f"{name} must be on cuda:{self.device}")
        st = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        r = _FemResult()
        _check(_lib.h2dlp_fem_field(self._h, _ptr(m), _ptr(h), None if u1 is None else _ptr(u1),
                                    None if u2 is None else _ptr(u2), float(tol), int(max_iter), st, ctypes.byref(r)))
        return FemResult(r.iters_u1, r.iters_u2, r.resid_u1, r.resid_u2, r.energy)


def plan(xyz, tri, order: int = 4, leaf: int = 32, eta: float = 2.0, precision="fp64", alpha: float = 0.1,
         coupling: str = "stored", dense_far_max: int = 0, recompress_eps: float = 0.0, row_basis: str = "stored"):
    """Host-only structure and byte counts (no GPU needed)."""
    return Operator(xyz, tri, order, leaf, eta, precision, alpha, plan_only=True, coupling=coupling,
                    dense_far_max=dense_far_max, recompress_eps=recompress_eps, row_basis=row_basis)


def last_error() -> str:
    return _lib.h2dlp_last_error().decode()


def library():
    return _lib
