"""Write sphere_l8_h2_rows.npz: rows of the oracle's H2 product on the 655362-node sphere.

The level-8 icosphere (radial jitter 0.25 %, seed 0) with order 5, leaf 64,
eta 2, and u1 = 16 N(0,1) columns from seed 0 (the benchmarked input).  The
1000 rows are numpy default_rng(3).choice(N, 1000, replace=False).  For each
exact-block threshold dense_far_max in (0, 7812, 15625) -- the plain
interpolation H2 matrix (Section 4), and admissible blocks with |t||s| <= k^2/2
or <= k^2 kept as exact entries (Section 3) -- the file holds those rows of
u2 = (K_H2 + D) u1, all from oracle.h2.H2Oracle.apply_rows, and the oracle's
diagonal D at the rows.  Worker processes only fill the oracle's own caches
(column bases) and evaluate disjoint row subsets; the arithmetic of every value
is the oracle's.  A few minutes on 8 cores.

    python tests/golden/make_l8_rows.py
"""
from __future__ import annotations

import os
import sys
import time
from multiprocessing import get_context

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import h2  # noqa: E402
from workloads import cases, rhs  # noqa: E402

OUT = os.path.join(HERE, "sphere_l8_h2_rows.npz")
N_ROWS = 1000
THRESHOLDS = (0, 7812, 15625)
_g = {}


def _column_bases(leaves):
    H = _g["H"]
    return [(int(c), H.W(c)) for c in leaves]


def _rows(args):
    d, rows = args
    return _g["H"].with_dense_far_max(d).apply_rows(_g["u"], rows, xh=_g["xh"])


def main(workers: int = 8):
    t0 = time.time()
    c = cases.CASES["sphere_l8"]
    xyz, tri = cases.mesh_of(c.mesh)
    n = xyz.shape[0]
    u = rhs.normal_rhs(n, 16, 0)
    rows = np.random.default_rng(3).choice(n, N_ROWS, replace=False)
    H = h2.H2Oracle(xyz, tri, order=c.order, leaf=c.leaf, eta=c.eta, cache_coupling=False)
    _g["H"] = H
    ctx = get_context("fork")
    leaves = np.where(H.child0 < 0)[0]
    with ctx.Pool(workers) as pool:
        for part in pool.imap_unordered(_column_bases, np.array_split(leaves, 8 * workers)):
            for leaf, w in part:
                H._W[leaf] = w
    print(f"column bases: {time.time() - t0:.0f} s", flush=True)
    xh = H.forward(u.T.copy())
    _g["u"], _g["xh"] = u, xh
    print(f"upward pass: {time.time() - t0:.0f} s", flush=True)
    pos = np.empty(n, dtype=np.int64)
    pos[H.perm] = np.arange(n)
    order = np.argsort(pos[rows], kind="stable")             # neighbouring rows share root paths
    chunks = np.array_split(order, 4 * workers)
    out = {"n_nodes": n, "rows": rows, "diag": H.D[rows], "thresholds": np.array(THRESHOLDS)}
    for d in THRESHOLDS:
        vals = np.empty((u.shape[0], N_ROWS))
        with ctx.Pool(workers) as pool:
            for ch, v in zip(chunks, pool.map(_rows, [(d, rows[ch]) for ch in chunks])):
                vals[:, ch] = v
        out[f"values_{d}"] = vals
        print(f"dense_far_max {d}: {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
