"""Pins for the oracle's H2 construction and matvec (Section 4).

Brute force on small inputs (the dense matrix), exact polynomial identities
(nestedness, quadrature exactness) and a direct, transfer-free evaluation of
every block catch mistakes in the tree, the bases, the transfers and the
up/down passes.
"""
from math import factorial

import numpy as np
import pytest

from oracle import dense, h2, quadrature
from workloads import meshes, rhs


@pytest.fixture(scope="module")
def l4():
    xyz, tri = meshes.icosphere(4, 0.01, 0)
    return xyz, tri, dense.dense_m(xyz, tri)


@pytest.fixture(scope="module")
def l4_h2(l4):
    xyz, tri, _ = l4
    return h2.H2Oracle(xyz, tri, order=4, leaf=32, eta=2.0)


def test_tree_partitions_nodes(l4_h2):
    H = l4_h2
    N = H.xyz.shape[0]
    assert np.array_equal(np.sort(H.perm), np.arange(N))
    leaves = np.where(H.child0 < 0)[0]
    assert np.all(H.end[leaves] - H.begin[leaves] <= 32)
    assert np.sum(H.end[leaves] - H.begin[leaves]) == N
    inner = np.where(H.child0 >= 0)[0]
    assert np.all(H.begin[H.child0[inner]] == H.begin[inner])
    assert np.all(H.end[H.child1[inner]] == H.end[inner])
    assert np.all(H.end[H.child0[inner]] == H.begin[H.child1[inner]])
    assert np.all(H.level[H.child0[inner]] == H.level[inner] + 1)


def test_split_rule(l4_h2):
    H = l4_h2
    for c in np.where(H.child0 >= 0)[0][:40]:
        pts = H.xyz[H.nodes(c)]
        lo, hi = pts.min(0), pts.max(0)
        ax = int(np.argmax(hi - lo))
        mid = (lo[ax] + hi[ax]) * 0.5
        assert np.all(H.xyz[H.nodes(H.child0[c]), ax] <= mid)
        assert np.all(H.xyz[H.nodes(H.child1[c]), ax] > mid)


def test_boxes_contain_supports_and_are_inflated(l4_h2):
    H = l4_h2
    for c in range(H.n_clusters):
        nodes = H.nodes(c)
        tris = H.tri[np.any(np.isin(H.tri, nodes), axis=1)]
        v = H.xyz[np.unique(tris)]
        assert np.all(v >= H.lo[c]) and np.all(v <= H.hi[c])
        ext = H.hi[c] - H.lo[c]
        assert ext.min() >= 0.1 * ext.max() * (1 - 1e-12)


def test_blocks_cover_matrix_once():
    xyz, tri = meshes.icosphere(3, 0.01, 0)
    H = h2.H2Oracle(xyz, tri, order=2, leaf=16, eta=2.0)
    N = xyz.shape[0]
    cover = np.zeros((N, N), dtype=np.int32)
    for t, s in np.vstack([H.far, H.near]):
        cover[np.ix_(H.nodes(t), H.nodes(s))] += 1
    assert np.all(cover == 1)
    for t, s in H.far:
        assert h2.admissible(H.lo, H.hi, t, s, 2.0)
    for t, s in H.near:
        assert not h2.admissible(H.lo, H.hi, t, s, 2.0)
        assert H.is_leaf(t) and H.is_leaf(s)


def test_quadrature_exact_for_monomials():
    for d in (3, 9, 12, 21):
        p, w = quadrature.triangle_rule(d)
        for a in range(d + 1):
            for b in range(d + 1 - a):
                exact = factorial(a) * factorial(b) / factorial(a + b + 2)
                assert abs(np.sum(w * p[:, 0] ** a * p[:, 1] ** b) - exact) < 1e-15


def test_transfer_reproduces_parent_polynomials(l4_h2):
    H = l4_h2
    rng = np.random.default_rng(0)
    for c in rng.choice(np.arange(1, H.n_clusters), 20, replace=False):
        t = H.parent[c]
        p = H.lo[c] + rng.random((30, 3)) * (H.hi[c] - H.lo[c])
        Lt = h2.tensor(*(h2.lagrange(H.pts[t][a], p[:, a]) for a in range(3)))
        Lc = h2.tensor(*(h2.lagrange(H.pts[c][a], p[:, a]) for a in range(3)))
        np.testing.assert_allclose(Lc @ H.E(c), Lt, atol=1e-12)


def test_bases_are_nested(l4_h2):
    H = l4_h2
    for t in np.where(H.child0 >= 0)[0][-6:]:
        c0, c1 = H.child0[t], H.child1[t]
        np.testing.assert_allclose(np.vstack([H.V(c0) @ H.E(c0), H.V(c1) @ H.E(c1)]), H.V(t), atol=1e-12)
        Wt = H.W(t)
        scale = np.abs(Wt).max()
        np.testing.assert_allclose(np.vstack([H.W(c0) @ H.E(c0), H.W(c1) @ H.E(c1)]) / scale, Wt / scale,
                                   atol=1e-12)


def test_column_basis_quadrature_is_exact(l4_h2):
    H = l4_h2
    H2 = h2.H2Oracle(H.xyz, H.tri, order=4, leaf=32, eta=2.0)
    H2.qp, H2.qw = quadrature.triangle_rule(3 * 3 + 6)
    leaf = int(np.where(H.child0 < 0)[0][3])
    np.testing.assert_allclose(H2.W(leaf), H.W(leaf), rtol=0, atol=1e-13 * np.abs(H.W(leaf)).max())


def test_near_blocks_are_exact_entries(l4, l4_h2):
    _, _, M = l4
    H = l4_h2
    K = M - np.diag(np.diag(M))
    for t, s in H.near[::97]:
        np.testing.assert_allclose(H.K_near(t, s), K[np.ix_(H.nodes(t), H.nodes(s))], atol=1e-15)


def test_nested_apply_equals_direct_block_sum():
    # the up/down transfer passes must equal sum_blocks V_t S_ts W_s^T evaluated without transfers
    xyz, tri = meshes.icosphere(3, 0.02, 3)
    H = h2.H2Oracle(xyz, tri, order=3, leaf=12, eta=1.5)
    x = rhs.normal_rhs(xyz.shape[0], 2, 9)
    y = H.D[None, :] * x
    for t, s in H.far:
        y[:, H.nodes(t)] += (H.V(t) @ H.S(t, s) @ H.W(s).T @ x[:, H.nodes(s)].T).T
    for t, s in H.near:
        y[:, H.nodes(t)] += (H.K_near(t, s) @ x[:, H.nodes(s)].T).T
    np.testing.assert_allclose(H.apply(x), y, atol=1e-13)


def test_far_block_approximation_converges(l4):
    xyz, tri, M = l4
    errs = []
    for m in (2, 3, 4, 5):
        H = h2.H2Oracle(xyz, tri, order=m, leaf=32, eta=2.0)
        t, s = H.far[len(H.far) // 2]
        exact = M[np.ix_(H.nodes(t), H.nodes(s))]
        approx = H.V(t) @ H.S(t, s) @ H.W(s).T
        errs.append(np.linalg.norm(approx - exact) / np.linalg.norm(exact))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[2] < 5e-3 and errs[3] < 0.5 * errs[2]


def test_h2_matches_dense_at_order4(l4, l4_h2):
    xyz, tri, M = l4
    u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(xyz.shape[0], 1, 0)])
    u2 = l4_h2.apply(u)
    ref = u @ M.T
    for q in range(2):
        assert np.linalg.norm(u2[q] - ref[q]) / np.linalg.norm(ref[q]) <= 1e-4
    one = l4_h2.apply(np.ones(xyz.shape[0]))
    assert np.max(np.abs(one + 1.0)) < 2e-3


def test_sparse_input_matches_dense_input(l4_h2):
    # skipping all-zero pieces must not change anything (linearity)
    H = l4_h2
    N = H.xyz.shape[0]
    x = np.zeros((3, N))
    x[0, 5] = 1.0
    x[1, 1700] = -2.0
    x[2] = rhs.normal_rhs(N, 1, 4)[0]
    full = H.apply(x)
    cols = np.stack([H.apply(x[q]) for q in range(3)])
    np.testing.assert_allclose(full, cols, atol=1e-14)
    e5 = H.apply(np.eye(N)[5])
    assert np.count_nonzero(e5) > N // 2


def test_order_sweep_smallest_passing_order_is_4(l4):
    # H2 against the dense matrix on the 2562-node sphere for m = 2..5 (u1 = z
    # and one N(0,1) column): geometric convergence, and m = 4 is the smallest
    # order inside 1e-4 (measured: m = 2..7 give 9.0e-3, 9.6e-4, 9.1e-5,
    # 1.2e-5, 2.3e-6, 3.8e-7 for u1 = z)
    xyz, tri, M = l4
    u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(xyz.shape[0], 1, 0)])
    ref = u @ M.T
    errs = []
    for m in (2, 3, 4, 5):
        H = h2.H2Oracle(xyz, tri, order=m, leaf=32, eta=2.0, cache_coupling=False)
        out = H.apply(u)
        errs.append(np.max(np.linalg.norm(out - ref, axis=1) / np.linalg.norm(ref, axis=1)))
    assert all(errs[q + 1] < errs[q] / 3.0 for q in range(3)), errs
    assert errs[1] > 1e-4 >= errs[2], errs


def test_dense_far_blocks():
    # admissible blocks kept as exact entries: the block partition is unchanged,
    # every block exact reproduces the dense matrix, and a partial threshold
    # only removes approximation error
    xyz, tri = meshes.icosphere(3, 0.01, 3)
    M = dense.dense_m(xyz, tri)
    u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(xyz.shape[0], 1, 0)])
    ref = u @ M.T
    plain = h2.H2Oracle(xyz, tri, order=3, leaf=16, eta=2.0)
    part = h2.H2Oracle(xyz, tri, order=3, leaf=16, eta=2.0, dense_far_max=27 * 27)
    full = h2.H2Oracle(xyz, tri, order=3, leaf=16, eta=2.0, dense_far_max=xyz.shape[0] ** 2)
    c0, c1 = plain.counts(), part.counts()
    assert c1["far"] + c1["far_dense"] == c0["far"] and c1["far_dense"] > 0 and c1["far"] > 0
    assert c1["near"] == c0["near"] and c1["near_entries"] == c0["near_entries"]
    size = part.end - part.begin
    assert np.all(size[part.far_dense[:, 0]] * size[part.far_dense[:, 1]] <= 27 * 27)
    assert np.all(size[part.far[:, 0]] * size[part.far[:, 1]] > 27 * 27)
    assert full.far.shape[0] == 0
    np.testing.assert_allclose(full.apply(u), ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    e0 = np.linalg.norm(plain.apply(u) - ref, axis=1) / np.linalg.norm(ref, axis=1)
    e1 = np.linalg.norm(part.apply(u) - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert np.all(e1 < e0), (e0, e1)


def test_dense_far_max_view_equals_fresh_build():
    # re-splitting an existing oracle gives the operator a fresh build with the
    # same threshold gives (shared pieces do not depend on the split)
    xyz, tri = meshes.icosphere(3, 0.01, 3)
    u = rhs.normal_rhs(xyz.shape[0], 2, 4)
    plain = h2.H2Oracle(xyz, tri, order=3, leaf=16, eta=2.0)
    plain.apply(u)                                           # fill the caches first
    for d in (27 * 27, 16 * 16):
        view = plain.with_dense_far_max(d)
        fresh = h2.H2Oracle(xyz, tri, order=3, leaf=16, eta=2.0, dense_far_max=d)
        assert np.array_equal(view.far, fresh.far) and np.array_equal(view.far_dense, fresh.far_dense)
        assert np.array_equal(view.apply(u), fresh.apply(u))
    assert plain.far_dense.shape[0] == 0                    # the original keeps its own split


def test_rows_of_the_product():
    # the row-restricted product against the whole product, and with every
    # block exact against rows of the dense matrix (Section 3)
    xyz, tri = meshes.icosphere(3, 0.02, 6)
    N = xyz.shape[0]
    M = dense.dense_m(xyz, tri)
    u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(N, 2, 12)])
    rows = np.random.default_rng(5).choice(N, 37, replace=False)
    H = h2.H2Oracle(xyz, tri, order=3, leaf=12, eta=2.0)
    for d in (0, 12 * 12, N * N):
        Hd = H.with_dense_far_max(d)
        full = Hd.apply(u)
        got = Hd.apply_rows(u, rows)
        np.testing.assert_allclose(got, full[:, rows], rtol=0, atol=1e-14 * np.abs(full).max())
    exact = (u @ M.T)[:, rows]
    np.testing.assert_allclose(H.with_dense_far_max(N * N).apply_rows(u, rows), exact, rtol=0,
                               atol=1e-13 * np.abs(exact).max())
    # a precomputed upward pass gives the same rows
    x = u.T.copy()
    np.testing.assert_array_equal(H.apply_rows(u, rows, xh=H.forward(x)), H.apply_rows(u, rows))
