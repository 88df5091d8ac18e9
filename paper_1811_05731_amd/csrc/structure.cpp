// Host-side H2 block structure (see structure.h).
#include "structure.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>
#include <utility>

namespace h2dlp {

namespace {

std::string check_mesh(const double* xyz, int64_t n, const int32_t* tri, int64_t t) {
    if (n < 4 || t < 4) return "mesh needs at least 4 nodes and 4 triangles";
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(xyz[i])) return "non-finite node coordinate";
    for (int64_t e = 0; e < t; ++e) {
        const int32_t a = tri[3 * e], b = tri[3 * e + 1], c = tri[3 * e + 2];
        if (a < 0 || b < 0 || c < 0 || a >= n || b >= n || c >= n) return "triangle index out of range";
        if (a == b || b == c || a == c) return "degenerate triangle (repeated vertex)";
        const double* p = xyz + 3 * a; const double* q = xyz + 3 * b; const double* r = xyz + 3 * c;
        const double u[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
        const double v[3] = {r[0] - p[0], r[1] - p[1], r[2] - p[2]};
        const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
        if (!(cx * cx + cy * cy + cz * cz > 0.0)) return "degenerate triangle (zero area)";
    }
    // every directed edge exactly once, and its reverse present
    std::vector<int64_t> key(3 * t);
    for (int64_t e = 0; e < t; ++e)
        for (int a = 0; a < 3; ++a)
            key[3 * e + a] = int64_t(tri[3 * e + a]) * n + tri[3 * e + (a + 1) % 3];
    std::sort(key.begin(), key.end());
    for (size_t q = 1; q < key.size(); ++q)
        if (key[q] == key[q - 1]) return "directed edge used twice (inconsistent orientation or non-manifold)";
    for (int64_t k : key) {
        const int64_t r = (k % n) * n + k / n;
        if (!std::binary_search(key.begin(), key.end(), r)) return "open or non-manifold edge";
    }
    double vol = 0.0;
    for (int64_t e = 0; e < t; ++e) {
        const double* p = xyz + 3 * tri[3 * e]; const double* q = xyz + 3 * tri[3 * e + 1];
        const double* r = xyz + 3 * tri[3 * e + 2];
        vol += p[0] * (q[1] * r[2] - q[2] * r[1]) + p[1] * (q[2] * r[0] - q[0] * r[2]) + p[2] * (q[0] * r[1] - q[1] * r[0]);
    }
    if (!(vol > 0.0)) return "signed volume is not positive (inward orientation)";
    // coincident nodes make the double-layer kernel singular between different nodes
    std::vector<int64_t> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
        for (int d = 0; d < 3; ++d)
            if (xyz[3 * a + d] != xyz[3 * b + d]) return xyz[3 * a + d] < xyz[3 * b + d];
        return a < b;
    });
    for (int64_t q = 1; q < n; ++q) {
        const double* a = xyz + 3 * ord[q - 1]; const double* b = xyz + 3 * ord[q];
        if (a[0] == b[0] && a[1] == b[1] && a[2] == b[2]) return "coincident nodes";
    }
    return "";
}

}  // namespace

bool admissible(const Cluster& t, const Cluster& s, double eta) {
    const double tx = t.hi[0] - t.lo[0], ty = t.hi[1] - t.lo[1], tz = t.hi[2] - t.lo[2];
    const double sx = s.hi[0] - s.lo[0], sy = s.hi[1] - s.lo[1], sz = s.hi[2] - s.lo[2];
    const double diam_t = (tx * tx + ty * ty) + tz * tz;
    const double diam_s = (sx * sx + sy * sy) + sz * sz;
    double g[3];
    for (int a = 0; a < 3; ++a)
        g[a] = std::max(0.0, std::max(s.lo[a] - t.hi[a], t.lo[a] - s.hi[a]));
    const double dist = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
    return std::max(diam_t, diam_s) <= (eta * eta) * dist;
}

std::string build_structure(Structure& s, const double* xyz, int64_t n, const int32_t* tri, int64_t t,
                            int leaf, double eta, double alpha, bool want_rings) {
    std::string err = check_mesh(xyz, n, tri, t);
    if (!err.empty()) return err;
    s.n_nodes = n;
    s.n_tris = t;
    s.xyz.assign(xyz, xyz + 3 * n);
    s.tri.assign(tri, tri + 3 * t);

    // node -> incident triangles
    s.inc_off.assign(n + 1, 0);
    for (int64_t e = 0; e < 3 * t; ++e) s.inc_off[tri[e] + 1]++;
    for (int64_t i = 0; i < n; ++i) s.inc_off[i + 1] += s.inc_off[i];
    s.inc_tri.resize(3 * t);
    s.inc_loc.resize(3 * t);
    {
        std::vector<int64_t> fill(s.inc_off.begin(), s.inc_off.end() - 1);
        for (int64_t e = 0; e < t; ++e)
            for (int a = 0; a < 3; ++a) {
                const int64_t q = fill[tri[3 * e + a]]++;
                s.inc_tri[q] = int32_t(e);
                s.inc_loc[q] = a;
            }
    }

    // cluster tree: bisect the nodes' bounding box at the midpoint of its longest side
    s.perm.resize(n);
    std::iota(s.perm.begin(), s.perm.end(), 0);
    s.cl.clear();
    std::function<int(int64_t, int64_t, int, int)> rec = [&](int64_t b, int64_t e, int level, int parent) -> int {
        const int cid = int(s.cl.size());
        s.cl.push_back(Cluster{});
        s.cl[cid].begin = b;
        s.cl[cid].end = e;
        s.cl[cid].level = level;
        s.cl[cid].parent = parent;
        s.depth = std::max(s.depth, int32_t(level));
        if (e - b <= leaf) return cid;
        double lo[3], hi[3];
        for (int a = 0; a < 3; ++a) lo[a] = hi[a] = xyz[3 * int64_t(s.perm[b]) + a];
        for (int64_t q = b + 1; q < e; ++q)
            for (int a = 0; a < 3; ++a) {
                const double v = xyz[3 * int64_t(s.perm[q]) + a];
                lo[a] = std::min(lo[a], v);
                hi[a] = std::max(hi[a], v);
            }
        int axis = 0;
        if (hi[1] - lo[1] > hi[axis] - lo[axis]) axis = 1;
        if (hi[2] - lo[2] > hi[axis] - lo[axis]) axis = 2;
        const double mid = (lo[axis] + hi[axis]) * 0.5;
        auto it = std::stable_partition(s.perm.begin() + b, s.perm.begin() + e,
                                        [&](int32_t node) { return xyz[3 * int64_t(node) + axis] <= mid; });
        const int64_t p = it - s.perm.begin();
        if (p == b || p == e) {
            err = "cluster split produced an empty child (coincident nodes)";
            return cid;
        }
        const int c0 = rec(b, p, level + 1, cid);
        if (!err.empty()) return cid;
        const int c1 = rec(p, e, level + 1, cid);
        s.cl[cid].child0 = c0;
        s.cl[cid].child1 = c1;
        return cid;
    };
    s.depth = 0;
    rec(0, n, 0, -1);
    if (!err.empty()) return err;
    s.iperm.resize(n);
    for (int64_t q = 0; q < n; ++q) s.iperm[s.perm[q]] = q;

    // boxes of the hat-function supports, then inflation
    std::vector<double> nlo(3 * n), nhi(3 * n);
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) nlo[3 * i + a] = nhi[3 * i + a] = xyz[3 * i + a];
    for (int64_t e = 0; e < t; ++e) {
        double lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = hi[a] = xyz[3 * int64_t(tri[3 * e]) + a];
            for (int v = 1; v < 3; ++v) {
                const double x = xyz[3 * int64_t(tri[3 * e + v]) + a];
                lo[a] = std::min(lo[a], x);
                hi[a] = std::max(hi[a], x);
            }
        }
        for (int v = 0; v < 3; ++v) {
            const int64_t i = tri[3 * e + v];
            for (int a = 0; a < 3; ++a) {
                nlo[3 * i + a] = std::min(nlo[3 * i + a], lo[a]);
                nhi[3 * i + a] = std::max(nhi[3 * i + a], hi[a]);
            }
        }
    }
    for (int c = int(s.cl.size()) - 1; c >= 0; --c) {   // children have larger preorder ids
        Cluster& C = s.cl[c];
        if (C.leaf()) {
            for (int a = 0; a < 3; ++a) {
                C.lo[a] = nlo[3 * int64_t(s.perm[C.begin]) + a];
                C.hi[a] = nhi[3 * int64_t(s.perm[C.begin]) + a];
            }
            for (int64_t q = C.begin + 1; q < C.end; ++q)
                for (int a = 0; a < 3; ++a) {
                    C.lo[a] = std::min(C.lo[a], nlo[3 * int64_t(s.perm[q]) + a]);
                    C.hi[a] = std::max(C.hi[a], nhi[3 * int64_t(s.perm[q]) + a]);
                }
        } else {
            const Cluster& A = s.cl[C.child0];
            const Cluster& B = s.cl[C.child1];
            for (int a = 0; a < 3; ++a) {
                C.lo[a] = std::min(A.lo[a], B.lo[a]);
                C.hi[a] = std::max(A.hi[a], B.hi[a]);
            }
        }
    }
    // inflation is applied after all raw boxes exist (parents use the children's raw boxes)
    for (Cluster& C : s.cl) {
        const double ext[3] = {C.hi[0] - C.lo[0], C.hi[1] - C.lo[1], C.hi[2] - C.lo[2]};
        const double w = alpha * std::max(std::max(ext[0], ext[1]), ext[2]);
        for (int a = 0; a < 3; ++a)
            if (ext[a] < w) {
                const double mid = (C.lo[a] + C.hi[a]) * 0.5;
                const double half = w * 0.5;
                C.lo[a] = mid - half;
                C.hi[a] = mid + half;
            }
    }

    // block tree
    s.far.clear();
    s.near.clear();
    std::vector<std::pair<int32_t, int32_t>> stack{{0, 0}};
    while (!stack.empty()) {
        const auto [tt, ss] = stack.back();
        stack.pop_back();
        const Cluster& T = s.cl[tt];
        const Cluster& S = s.cl[ss];
        if (admissible(T, S, eta)) {
            s.far.push_back({tt, ss});
        } else if (T.leaf() && S.leaf()) {
            s.near.push_back({tt, ss});
        } else if (!T.leaf() && !S.leaf()) {
            stack.push_back({T.child0, S.child0});
            stack.push_back({T.child0, S.child1});
            stack.push_back({T.child1, S.child0});
            stack.push_back({T.child1, S.child1});
        } else if (T.leaf()) {
            stack.push_back({tt, S.child0});
            stack.push_back({tt, S.child1});
        } else {
            stack.push_back({T.child0, ss});
            stack.push_back({T.child1, ss});
        }
    }
    std::sort(s.far.begin(), s.far.end());
    std::sort(s.near.begin(), s.near.end());

    // 2-ring of every node (graph distance 1 or 2), stored by cluster position
    s.ring_off.assign(n + 1, 0);
    s.ring_pos.clear();
    if (want_rings) {
        std::vector<std::vector<int32_t>> nb(n);
        for (int64_t e = 0; e < t; ++e)
            for (int a = 0; a < 3; ++a) {
                nb[tri[3 * e + a]].push_back(tri[3 * e + (a + 1) % 3]);
                nb[tri[3 * e + (a + 1) % 3]].push_back(tri[3 * e + a]);
            }
        for (auto& v : nb) {
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
        }
        std::vector<int32_t> acc;
        for (int64_t p = 0; p < n; ++p) {
            const int32_t i = s.perm[p];
            acc.clear();
            for (int32_t j : nb[i]) {
                acc.push_back(int32_t(s.iperm[j]));
                for (int32_t k : nb[j])
                    if (k != i) acc.push_back(int32_t(s.iperm[k]));
            }
            std::sort(acc.begin(), acc.end());
            acc.erase(std::unique(acc.begin(), acc.end()), acc.end());
            s.ring_pos.insert(s.ring_pos.end(), acc.begin(), acc.end());
            s.ring_off[p + 1] = int64_t(s.ring_pos.size());
        }
    }
    return "";
}

}  // namespace h2dlp
