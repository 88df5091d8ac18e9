"""Pins for the oracle's algebraic recompression (Section 4: the purely
algebraic conversion to an H2 matrix with adaptive ranks).

Exactness at eps = 0, orthonormal nested bases, the weights against their
direct definition (a sum over every block the basis serves), the error
against the interpolation H2 matrix bounded by eps, ranks that fall as eps
grows, and the dense matrix within the H2 tolerance."""
import numpy as np
import pytest

from oracle import dense, h2, recompress
from workloads import meshes, rhs


@pytest.fixture(scope="module")
def l3():
    xyz, tri = meshes.icosphere(3, 0.01, 2)
    H = h2.H2Oracle(xyz, tri, order=4, leaf=16, eta=2.0)
    u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(xyz.shape[0], 2, 3)])
    return H, u, H.apply(u)


def rel(a, b):
    return np.max(np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1))


def test_eps_zero_is_the_interpolation_matrix(l3):
    H, u, ref = l3
    R = recompress.Recompressed(H, 0.0)
    assert rel(R.apply(u), ref) < 1e-13
    # ranks never exceed the rows of a leaf or the interpolation rank k
    size = H.end - H.begin
    for side in (R.row, R.col):
        assert np.all(side["rank"] <= np.minimum(size, H.k))


def test_bases_are_orthonormal_and_nested(l3):
    H, _, _ = l3
    R = recompress.Recompressed(H, 1e-6)
    for side in ("row", "col"):
        d = R.row if side == "row" else R.col
        for c in list(range(0, H.n_clusters, 7)) + [0]:
            B = R.basis(side, c)
            assert B.shape == (H.end[c] - H.begin[c], d["rank"][c])
            np.testing.assert_allclose(B.T @ B, np.eye(B.shape[1]), atol=1e-12)
            if not H.is_leaf(c):
                c0, c1 = H.child0[c], H.child1[c]
                Fs = np.vstack([d["F"][c0], d["F"][c1]])
                np.testing.assert_allclose(Fs.T @ Fs, np.eye(Fs.shape[1]), atol=1e-12)
        # the old basis in the new one: V_t ~ B_t P_t, within eps of the weighted part
        old = H.V if side == "row" else H.W
        for c in np.where(H.child0 < 0)[0][::5]:
            B = R.basis(side, c)
            np.testing.assert_allclose(B @ d["P"][c], B @ (B.T @ old(c)), atol=1e-12 * np.abs(old(c)).max())


def test_weights_against_every_served_block():
    # L_t L_t^T must equal the sum, over t and its ancestors a and the
    # admissible blocks (a, s), of (E_t ... E_a') S_as W_s^T W_s S_as^T (...)^T
    xyz, tri = meshes.icosphere(2, 0.02, 4)
    H = h2.H2Oracle(xyz, tri, order=3, leaf=8, eta=2.0)
    R = recompress.Recompressed(H, 1e-8)
    Rw = R._orth_factors(H.W)
    L = R._weights(Rw, transpose=False)
    for t in range(H.n_clusters):
        total = np.zeros((H.k, H.k))
        chain, a = np.eye(H.k), t
        while a >= 0:
            for b, s in H.far:
                if b == a:
                    # W_s over the rows of s: the leaf bases times the transfers up to s
                    Ws = np.vstack([H.W(l) @ _up(H, l, s) for l in _leaves_of(H, s)])
                    M = chain @ H.S(a, s) @ Ws.T
                    total += M @ M.T
            if H.parent[a] >= 0:
                chain = chain @ H.E(a)
            a = H.parent[a]
        np.testing.assert_allclose(L[t] @ L[t].T, total, atol=1e-12 * max(1.0, np.abs(total).max()))


def _leaves_of(H, c):
    if H.is_leaf(c):
        return [c]
    return _leaves_of(H, H.child0[c]) + _leaves_of(H, H.child1[c])


def _up(H, leaf, s):
    """E_leaf E_parent ... up to (excluding) s: the leaf basis in s's interpolation basis."""
    M, c = np.eye(H.k), leaf
    while c != s:
        M = M @ H.E(c)
        c = H.parent[c]
    return M


def test_error_within_eps_and_ranks_fall(l3):
    H, u, ref = l3
    k_ref = ref - H.D[None, :] * u
    prev = None
    for eps in (1e-8, 1e-6, 1e-4, 1e-2):
        R = recompress.Recompressed(H, eps)
        out = R.apply(u)
        err_k = rel(out - H.D[None, :] * u, k_ref)
        assert err_k <= 10 * eps, (eps, err_k)
        c = R.counts()
        if prev is not None:
            leaves = H.child0 < 0
            assert np.all(R.row["rank"][leaves] <= prev.row["rank"][leaves])
            assert np.all(R.col["rank"][leaves] <= prev.col["rank"][leaves])
            assert c["coupling_entries"] <= prev.counts()["coupling_entries"]
        prev = R
    assert prev.counts()["coupling_entries"] < 0.05 * H.far.shape[0] * H.k ** 2


def test_recompressed_matches_dense_like_the_interpolation_matrix():
    xyz, tri = meshes.icosphere(4, 0.01, 0)
    M = dense.dense_m(xyz, tri)
    u = np.vstack([rhs.z_rhs(xyz), rhs.normal_rhs(xyz.shape[0], 1, 0)])
    H = h2.H2Oracle(xyz, tri, order=4, leaf=32, eta=2.0)
    R = recompress.Recompressed(H, 1e-5)
    assert rel(R.apply(u), u @ M.T) <= 1e-4
    assert R.counts()["coupling_entries"] < 0.15 * H.far.shape[0] * H.k ** 2
