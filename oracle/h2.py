"""H2 approximation of the double-layer matrix K and its matvec (oracle; test only).

Section 4 of the paper: blocks K|_{t x s} of well-separated index sets are
replaced by low-rank factors from an analytic approximation of the kernel
(interpolation), and the H2 format stores per block only k x k coupling
coefficients between nested cluster bases.  The paper builds its H2 matrix with
H2Lib (HCA followed by algebraic recompression); the method reproduced here is
the direct interpolation construction the paper names as the analytic route:
tensor Chebyshev interpolation of g(x, y) = 1/(4 pi |x - y|) on bounding boxes,

    g(x, y) ~ sum_nu sum_mu L^t_nu(x) g(eta^t_nu, eta^s_mu) L^s_mu(y),

so that for i in t, j in s (block admissible)

    K_ij ~ sum_nu sum_mu V_t(i, nu) S_ts(nu, mu) W_s(j, mu),
    V_t(i, nu)  = L^t_nu(xi_i),
    S_ts(nu,mu) = 1/(4 pi |eta^t_nu - eta^s_mu|),
    W_s(j, mu)  = integral phi_j(y) n(y).grad L^s_mu(y) dS_y,

with the bases nested through the transfer matrices E_c(nu', nu) = L^t_nu(eta^c_nu')
of a child c of t.  Readings of points the paper leaves open (all shared with
the library by specification only, never by code):

* cluster tree: split the bounding box of the cluster's nodes at the midpoint
  (lo + hi) * 0.5 of its longest side (ties: lowest axis), nodes with
  coordinate <= mid to the first child, order kept; a leaf has <= `leaf` nodes;
* cluster box: bounding box of the supports of the cluster's hat functions
  (all vertices of the triangles incident to its nodes), then every side
  widened, about its centre, to at least alpha = 0.1 times the longest side;
* admissibility: max(diam_t^2, diam_s^2) <= eta^2 dist^2 (box diagonal,
  Euclidean box distance; squares summed x, y, z in that order);
* Chebyshev points of the first kind cos((2l + 1) pi/(2m)) on each box axis,
  tensor index nu = l_x + m l_y + m^2 l_z, k = m^3;
* near blocks (inadmissible leaf pairs) hold the exact entries of K;
* optionally (dense_far_max > 0) an admissible block with |t| |s| <=
  dense_far_max entries also holds its exact entries instead of the factors
  (the storage choice of a representation variant: with dense_far_max >= N^2
  every block is exact and the product is the dense matrix's).
"""
from __future__ import annotations

import copy

import numpy as np

from . import geometry, lindholm, quadrature

ALPHA = 0.1


# ----------------------------------------------------------------------------- tree

def build_cluster_tree(xyz: np.ndarray, leaf: int):
    """Preorder cluster tree.  Returns (perm, begin, end, level, parent, child0, child1)."""
    perm: list = []
    rows: list = []

    def rec(idx, level, parent):
        cid = len(rows)
        rows.append(None)
        begin = len(perm)
        if idx.size <= leaf:
            perm.extend(idx.tolist())
            rows[cid] = (begin, len(perm), level, parent, -1, -1)
            return cid
        pts = xyz[idx]
        lo = pts.min(axis=0)
        hi = pts.max(axis=0)
        axis = int(np.argmax(hi - lo))            # first maximum: lowest axis on ties
        mid = (lo[axis] + hi[axis]) * 0.5
        first = pts[:, axis] <= mid
        a, b = idx[first], idx[~first]
        if a.size == 0 or b.size == 0:
            raise ValueError("cluster split produced an empty child (duplicate nodes?)")
        c0 = rec(a, level + 1, cid)
        c1 = rec(b, level + 1, cid)
        rows[cid] = (begin, len(perm), level, parent, c0, c1)
        return cid

    rec(np.arange(xyz.shape[0], dtype=np.int64), 0, -1)
    arr = np.array(rows, dtype=np.int64)
    return (np.array(perm, dtype=np.int64),) + tuple(arr[:, q].copy() for q in range(6))


def support_boxes(xyz, tri, perm, begin, end, alpha=ALPHA):
    """Inflated bounding boxes of the clusters' hat-function supports: (C x 3, C x 3)."""
    t = np.asarray(tri, dtype=np.int64)
    n = xyz.shape[0]
    tlo = np.minimum(np.minimum(xyz[t[:, 0]], xyz[t[:, 1]]), xyz[t[:, 2]])
    thi = np.maximum(np.maximum(xyz[t[:, 0]], xyz[t[:, 1]]), xyz[t[:, 2]])
    nlo = np.full((n, 3), np.inf)
    nhi = np.full((n, 3), -np.inf)
    for a in range(3):
        np.minimum.at(nlo, t[:, a], tlo)
        np.maximum.at(nhi, t[:, a], thi)
    C = begin.size
    lo = np.empty((C, 3))
    hi = np.empty((C, 3))
    for c in range(C):
        nodes = perm[begin[c]:end[c]]
        lo[c] = nlo[nodes].min(axis=0)
        hi[c] = nhi[nodes].max(axis=0)
    for c in range(C):
        ext = hi[c] - lo[c]
        w = alpha * max(ext[0], ext[1], ext[2])
        for a in range(3):
            if ext[a] < w:
                mid = (lo[c, a] + hi[c, a]) * 0.5
                half = w * 0.5
                lo[c, a] = mid - half
                hi[c, a] = mid + half
    return lo, hi


def admissible(lo, hi, t, s, eta) -> bool:
    dt = hi[t] - lo[t]
    ds = hi[s] - lo[s]
    diam_t = (dt[0] * dt[0] + dt[1] * dt[1]) + dt[2] * dt[2]
    diam_s = (ds[0] * ds[0] + ds[1] * ds[1]) + ds[2] * ds[2]
    g = [max(0.0, lo[s, a] - hi[t, a], lo[t, a] - hi[s, a]) for a in range(3)]
    dist = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]
    return max(diam_t, diam_s) <= (eta * eta) * dist


def build_block_tree(lo, hi, child0, child1, eta):
    """Far (admissible) and near (inadmissible leaf x leaf) block lists, sorted by (t, s)."""
    far, near = [], []
    stack = [(0, 0)]
    while stack:
        t, s = stack.pop()
        if admissible(lo, hi, t, s, eta):
            far.append((t, s))
            continue
        tl, sl = child0[t] < 0, child0[s] < 0
        if tl and sl:
            near.append((t, s))
        elif not tl and not sl:
            for ct in (child0[t], child1[t]):
                for cs in (child0[s], child1[s]):
                    stack.append((ct, cs))
        elif tl:
            stack.append((t, child0[s]))
            stack.append((t, child1[s]))
        else:
            stack.append((child0[t], s))
            stack.append((child1[t], s))
    far = np.array(sorted(far), dtype=np.int64).reshape(-1, 2)
    near = np.array(sorted(near), dtype=np.int64).reshape(-1, 2)
    return far, near


# ----------------------------------------------------------------------------- interpolation

def chebyshev_points(lo, hi, m):
    """First-kind Chebyshev points on each axis of each box: (C, 3, m)."""
    ref = np.cos((2.0 * np.arange(m) + 1.0) * np.pi / (2.0 * m))
    c = 0.5 * (lo + hi)
    h = 0.5 * (hi - lo)
    return c[:, :, None] + h[:, :, None] * ref[None, None, :]


def lagrange(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Values L_l(x) of the 1D Lagrange basis on `nodes`: shape (len(x), m)."""
    m = nodes.size
    out = np.ones((x.size, m))
    for l in range(m):
        for p in range(m):
            if p != l:
                out[:, l] *= (x - nodes[p]) / (nodes[l] - nodes[p])
    return out


def lagrange_deriv(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Derivatives L_l'(x): shape (len(x), m) (product rule)."""
    m = nodes.size
    out = np.zeros((x.size, m))
    for l in range(m):
        for p in range(m):
            if p == l:
                continue
            term = np.full(x.size, 1.0 / (nodes[l] - nodes[p]))
            for q in range(m):
                if q != l and q != p:
                    term = term * (x - nodes[q]) / (nodes[l] - nodes[q])
            out[:, l] += term
    return out


def tensor(fx, fy, fz):
    """(P, m) x3 -> (P, m^3) with index nu = lx + m ly + m^2 lz."""
    P, m = fx.shape
    return np.einsum("pc,pb,pa->pcba", fz, fy, fx).reshape(P, m ** 3)


def grid_points(pts_c: np.ndarray) -> np.ndarray:
    """Tensor grid (k, 3) of one cluster's Chebyshev points, nu = lx + m ly + m^2 lz."""
    m = pts_c.shape[1]
    lz, ly, lx = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    return np.stack([pts_c[0][lx.ravel()], pts_c[1][ly.ravel()], pts_c[2][lz.ravel()]], axis=1)


# ----------------------------------------------------------------------------- the H2 matrix

class H2Oracle:
    """Interpolation H2 matrix of M = K + D; lazily built pieces, plain matvec."""

    def __init__(self, xyz, tri, order=4, leaf=32, eta=2.0, alpha=ALPHA, cache_coupling=True, dense_far_max=0):
        geometry.check_mesh(xyz, tri)
        if order < 1 or leaf < 1 or not eta > 0:
            raise ValueError("order >= 1, leaf >= 1 and eta > 0 required")
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.tri = np.asarray(tri, dtype=np.int64)
        self.m, self.k = order, order ** 3
        self.leaf, self.eta = leaf, eta
        (self.perm, self.begin, self.end, self.level, self.parent,
         self.child0, self.child1) = build_cluster_tree(self.xyz, leaf)
        self.lo, self.hi = support_boxes(self.xyz, self.tri, self.perm, self.begin, self.end, alpha)
        self.far_all, self.near = build_block_tree(self.lo, self.hi, self.child0, self.child1, eta)
        self.pts = chebyshev_points(self.lo, self.hi, order)
        self.normals, self.areas = geometry.triangle_normals_areas(self.xyz, self.tri)
        self.inc_off, self.inc_tri, self.inc_loc = geometry.incidence(self.xyz.shape[0], self.tri)
        self.D = geometry.diagonal(self.xyz, self.tri)
        qp, qw = quadrature.triangle_rule(3 * (order - 1))
        self.qp, self.qw = qp, qw
        self.cache_coupling = cache_coupling
        self._W, self._V, self._E, self._K, self._S = {}, {}, {}, {}, {}
        C = self.begin.size
        self._split_far(dense_far_max)
        self.near_of = [[] for _ in range(C)]
        for t, s in self.near:
            self.near_of[t].append(int(s))

    def _split_far(self, dense_far_max):
        """Admissible blocks with |t| |s| <= dense_far_max keep their exact
        entries (Section 3) instead of the interpolation factors."""
        size = self.end - self.begin
        small = size[self.far_all[:, 0]] * size[self.far_all[:, 1]] <= dense_far_max
        self.far, self.far_dense = self.far_all[~small], self.far_all[small]
        self.dense_far_max = dense_far_max
        self.far_of = [[] for _ in range(self.begin.size)]
        for t, s in self.far:
            self.far_of[t].append(int(s))

    def with_dense_far_max(self, dense_far_max):
        """The same matrix with another exact-block threshold.  The tree, the
        boxes and every cached basis, transfer and exact block are shared: none
        of them depends on which admissible blocks are kept exact."""
        other = copy.copy(self)
        other._split_far(dense_far_max)
        return other

    # -- structure -----------------------------------------------------------
    @property
    def n_clusters(self):
        return self.begin.size

    def nodes(self, c):
        return self.perm[self.begin[c]:self.end[c]]

    def is_leaf(self, c):
        return self.child0[c] < 0

    def export_structure(self) -> dict:
        return dict(perm=self.perm, begin=self.begin, end=self.end, level=self.level,
                    parent=self.parent, child0=self.child0, child1=self.child1,
                    box_lo=self.lo, box_hi=self.hi, far=self.far, near=self.near)

    # -- bases -----------------------------------------------------------------
    def V(self, t):
        """Row basis of leaf t: (n_t, k), V(i, nu) = L^t_nu(xi_i)."""
        if t not in self._V:
            p = self.xyz[self.nodes(t)]
            P = self.pts[t]
            self._V[t] = tensor(lagrange(P[0], p[:, 0]), lagrange(P[1], p[:, 1]), lagrange(P[2], p[:, 2]))
        return self._V[t]

    def _incidences(self, nodes):
        """(local node index, triangle, local vertex) for every triangle incident to `nodes`."""
        jl, tris, locs = [], [], []
        for a, j in enumerate(nodes):
            lo, hi = self.inc_off[j], self.inc_off[j + 1]
            jl.append(np.full(hi - lo, a))
            tris.append(self.inc_tri[lo:hi])
            locs.append(self.inc_loc[lo:hi])
        return np.concatenate(jl), np.concatenate(tris), np.concatenate(locs)

    def W(self, s):
        """Column basis of leaf s: (n_s, k), W(j, mu) = sum_{T ni j} int_T phi_j n_T.grad L^s_mu dS."""
        if s not in self._W:
            nodes = self.nodes(s)
            P = self.pts[s]
            jl, T, loc = self._incidences(nodes)
            r1, r2, r3 = (self.xyz[self.tri[T, a]] for a in range(3))
            u, v = self.qp[:, 0], self.qp[:, 1]
            y = (r1[:, None, :] + u[None, :, None] * (r2 - r1)[:, None, :]
                 + v[None, :, None] * (r3 - r1)[:, None, :]).reshape(-1, 3)       # (n_inc*Q, 3)
            bary = np.stack([1.0 - u - v, u, v], 1)                              # (Q, 3)
            phi = bary[:, loc].T                                                 # (n_inc, Q)
            fx, fy, fz = (lagrange(P[a], y[:, a]) for a in range(3))
            dx, dy, dz = (lagrange_deriv(P[a], y[:, a]) for a in range(3))
            n = np.repeat(self.normals[T], self.qw.size, axis=0)
            dn = (n[:, :1] * tensor(dx, fy, fz) + n[:, 1:2] * tensor(fx, dy, fz)
                  + n[:, 2:] * tensor(fx, fy, dz)).reshape(T.size, self.qw.size, self.k)
            wq = (2.0 * self.areas[T])[:, None] * self.qw[None, :] * phi        # (n_inc, Q)
            contrib = np.einsum("iq,iqk->ik", wq, dn)
            out = np.zeros((nodes.size, self.k))
            np.add.at(out, jl, contrib)
            self._W[s] = out
        return self._W[s]

    def E(self, c):
        """Transfer matrix of child c: (k, k), E(nu', nu) = L^{parent}_nu(eta^c_nu')."""
        if c not in self._E:
            t = self.parent[c]
            Pt, Pc = self.pts[t], self.pts[c]
            ex, ey, ez = (lagrange(Pt[a], Pc[a]) for a in range(3))
            self._E[c] = np.kron(ez, np.kron(ey, ex))
        return self._E[c]

    def S(self, t, s):
        """Coupling matrix (k, k): g at the interpolation points of t and s."""
        key = (t, s)
        if key in self._S:
            return self._S[key]
        a = grid_points(self.pts[t])
        b = grid_points(self.pts[s])
        d = np.linalg.norm(a[:, None, :] - b[None, :, :], axis=2)
        out = 1.0 / (4.0 * np.pi * d)
        if self.cache_coupling:
            self._S[key] = out
        return out

    def K_near(self, t, s):
        """Exact double-layer entries K|_{t x s} of a near block (n_t, n_s)."""
        key = (t, s)
        if key not in self._K:
            it, js = self.nodes(t), self.nodes(s)
            jl, T, loc = self._incidences(js)
            vt = self.tri[T]                                                     # (n_inc, 3)
            r1, r2, r3 = (self.xyz[vt[:, a]][None, :, :] for a in range(3))
            with np.errstate(divide="ignore", invalid="ignore"):               # incident pairs: dropped below
                L = lindholm.weights(self.xyz[it][:, None, :], r1, r2, r3)      # (n_t, n_inc, 3)
            Lj = np.take_along_axis(L, np.broadcast_to(loc[None, :, None], L.shape[:2] + (1,)), 2)[..., 0]
            incident = np.any(vt[None, :, :] == it[:, None, None], axis=2)       # by index
            Lj = np.where(incident, 0.0, Lj)
            onehot = (jl[:, None] == np.arange(js.size)[None, :]).astype(np.float64)
            self._K[key] = Lj @ onehot
        return self._K[key]

    # -- matvec ----------------------------------------------------------------
    def forward(self, x):
        """xhat[c] = W_c^T x|_c at leaves, then sum_children E_c^T xhat_c upwards (None = 0)."""
        C = self.n_clusters
        xh = [None] * C
        for c in range(C - 1, -1, -1):               # children have larger preorder ids
            if self.is_leaf(c):
                xs = x[self.nodes(c)]
                if np.any(xs != 0.0):
                    xh[c] = self.W(c).T @ xs
            else:
                acc = None
                for ch in (self.child0[c], self.child1[c]):
                    if xh[ch] is not None:
                        v = self.E(ch).T @ xh[ch]
                        acc = v if acc is None else acc + v
                xh[c] = acc
        return xh

    def coupling(self, xh):
        """yhat[t] = sum over admissible (t, s) of S_ts xhat[s] (None = 0)."""
        yh = [None] * self.n_clusters
        for t in range(self.n_clusters):
            for s in self.far_of[t]:
                if xh[s] is not None:
                    v = self.S(t, s) @ xh[s]
                    yh[t] = v if yh[t] is None else yh[t] + v
        return yh

    def backward(self, yh, r):
        """Downward transfer yhat_c += E_c yhat_parent, then y|_t = V_t yhat_t at leaves."""
        N = self.xyz.shape[0]
        y = np.zeros((N, r))
        yh = list(yh)
        for c in range(1, self.n_clusters):           # parents precede children in preorder
            p = self.parent[c]
            if yh[p] is not None:
                v = self.E(c) @ yh[p]
                yh[c] = v if yh[c] is None else yh[c] + v
        for c in range(self.n_clusters):
            if self.is_leaf(c) and yh[c] is not None:
                y[self.nodes(c)] += self.V(c) @ yh[c]
        return y

    def near_field(self, x, y):
        for t, s in np.concatenate([self.near, self.far_dense]):
            xs = x[self.nodes(s)]
            if np.any(xs != 0.0):
                y[self.nodes(t)] += self.K_near(t, s) @ xs
        return y

    def apply(self, u1: np.ndarray) -> np.ndarray:
        """u2 = (K_H2 + D) u1 for u1 of shape (r, N) (or (N,)); returns the same shape."""
        u = np.asarray(u1, dtype=np.float64)
        squeeze = u.ndim == 1
        x = np.atleast_2d(u).T.copy()
        xh = self.forward(x)
        yh = self.coupling(xh)
        y = self.backward(yh, x.shape[1])
        y = self.near_field(x, y)
        y += self.D[:, None] * x
        out = y.T
        return out[0] if squeeze else out

    def apply_rows(self, u1: np.ndarray, rows, xh=None) -> np.ndarray:
        """Rows `rows` (node indices) of u2 = (K_H2 + D) u1: shape (r, len(rows)).

        The same steps as apply(): the full upward pass (or `xh`, a forward()
        result for the same u1), then the coupling and the downward pass only
        for the clusters on the root paths of the leaves holding the rows, the
        rows of V_t there, and the exact blocks of those clusters.
        """
        u = np.atleast_2d(np.asarray(u1, dtype=np.float64))
        x = u.T.copy()
        rows = np.asarray(rows, dtype=np.int64)
        if xh is None:
            xh = self.forward(x)
        N = self.xyz.shape[0]
        pos = np.empty(N, dtype=np.int64)
        pos[self.perm] = np.arange(N)
        # every cluster whose index range holds a requested row (root paths)
        on_path = np.zeros(self.n_clusters, dtype=bool)
        for p in np.unique(pos[rows]):
            c = 0
            while True:
                on_path[c] = True
                if self.is_leaf(c):
                    break
                c = self.child0[c] if p < self.end[self.child0[c]] else self.child1[c]
        # coupling and downward pass along the paths (parents precede children)
        yt = [None] * self.n_clusters
        for t in np.where(on_path)[0]:
            acc = None
            for s in self.far_of[t]:
                if xh[s] is not None:
                    v = self.S(t, s) @ xh[s]
                    acc = v if acc is None else acc + v
            p = self.parent[t]
            if p >= 0 and yt[p] is not None:
                v = self.E(t) @ yt[p]
                acc = v if acc is None else acc + v
            yt[t] = acc
        exact_of = {}
        for t, s in np.concatenate([self.near, self.far_dense]):
            if on_path[t]:
                exact_of.setdefault(int(t), []).append(int(s))
        out = np.empty((x.shape[1], rows.size))
        for q, i in enumerate(rows):
            acc = self.D[i] * x[i]
            c = 0
            while True:
                li = pos[i] - self.begin[c]                 # local row of i in cluster c
                for s in exact_of.get(c, ()):
                    acc = acc + self.K_near(c, s)[li] @ x[self.nodes(s)]
                if self.is_leaf(c):
                    if yt[c] is not None:
                        acc = acc + self.V(c)[li] @ yt[c]
                    break
                c = self.child0[c] if pos[i] < self.end[self.child0[c]] else self.child1[c]
            out[:, q] = acc
        return out

    # -- sizes -------------------------------------------------------------------
    def counts(self) -> dict:
        size = self.end - self.begin
        n_near = int(sum(size[t] * size[s] for t, s in self.near))
        n_dense = int(sum(size[t] * size[s] for t, s in self.far_dense))
        return dict(N=int(self.xyz.shape[0]), clusters=int(self.n_clusters),
                    leaves=int(np.sum(self.child0 < 0)), far=int(self.far.shape[0]),
                    near=int(self.near.shape[0]), near_entries=n_near,
                    far_dense=int(self.far_dense.shape[0]), dense_far_entries=n_dense,
                    depth=int(self.level.max()))
