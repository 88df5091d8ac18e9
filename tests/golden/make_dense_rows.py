"""Write sphere_l7_dense_rows.npz: exact rows of M u1 on the 163842-node sphere.

The level-7 icosphere (radial jitter 0.5 %, seed 0), u1 = [z, 8 N(0,1) columns
from seed 0], and the 1000 rows chosen by numpy default_rng(2).choice(N, 1000,
replace=False).  Every value comes from the oracle's dense rows of M = K + D
(Section 3, eqs. matrix_definition and denseMat): the Lindholm weights of
each row's node against all triangles, plus the diagonal.  About a minute on
8 cores.

    python tests/golden/make_dense_rows.py
"""
from __future__ import annotations

import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dense, geometry  # noqa: E402
from workloads import cases, rhs  # noqa: E402

OUT = os.path.join(HERE, "sphere_l7_dense_rows.npz")
N_ROWS = 1000
_ctx = {}


def _setup():
    c = cases.CASES["sphere_l7"]
    xyz, tri = cases.mesh_of(c.mesh)
    u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(xyz.shape[0], 8, 0)])
    rows = np.random.default_rng(2).choice(xyz.shape[0], N_ROWS, replace=False)
    return xyz, tri, u, rows


def _init(diag):
    _ctx["xyz"], _ctx["tri"], _ctx["u"], _ = _setup()
    _ctx["diag"] = diag


def _chunk(rows):
    M = dense.m_rows(_ctx["xyz"], _ctx["tri"], rows, diag=_ctx["diag"])
    return M @ _ctx["u"].T                              # (len(rows), r)


def main():
    xyz, tri, u, rows = _setup()
    diag = geometry.diagonal(xyz, tri)
    chunks = np.array_split(rows, 40)
    with Pool(min(8, os.cpu_count() or 1), initializer=_init, initargs=(diag,)) as pool:
        parts = pool.map(_chunk, chunks)
    values = np.concatenate(parts, axis=0).T            # (r, N_ROWS)
    np.savez_compressed(OUT, rows=rows, values=values, n_nodes=np.int64(xyz.shape[0]))
    print(f"wrote {OUT}: rows {rows.shape}, values {values.shape}")


if __name__ == "__main__":
    main()
