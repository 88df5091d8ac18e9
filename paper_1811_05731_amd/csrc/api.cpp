// C ABI of the library (include/h2dlp.h): build, apply, sizes, export, errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/h2dlp.h"
#include "entry.h"
#include "kernels.h"
#include "recompress.h"
#include "structure.h"

using namespace h2dlp;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

struct HipError {
    hipError_t err;
    std::string where;
};

void check(hipError_t e, const char* where) {
    if (e != hipSuccess) throw HipError{e, where};
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Gauss-Legendre nodes/weights on [-1, 1] by Newton's method on the
// three-term recurrence of the Legendre polynomials.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int j = 2; j <= n; ++j) {
            const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Collapsed-square rule on the reference triangle {u, v >= 0, u + v <= 1},
// exact for total degree `degree`: v = (1 - u) t, Jacobian (1 - u).
std::vector<double> triangle_rule(int degree) {
    const int n = (degree + 3) / 2;
    std::vector<double> x, w;
    gauss_legendre(n, x, w);
    std::vector<double> out;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            const double u = 0.5 * (x[a] + 1.0), t = 0.5 * (x[b] + 1.0);
            out.push_back(u);
            out.push_back((1.0 - u) * t);
            out.push_back(0.25 * w[a] * w[b] * (1.0 - u));
        }
    return out;
}

}  // namespace

struct h2dlp_ctx {
    h2dlp_options opt{};
    int device = -1;                 // -1 until device memory exists
    int m = 0, k = 0, prec = 0;
    size_t elem = 8;                 // bytes per stored value of the operator
    size_t elem_s = 8;               // bytes per coupling entry (6 for BF16X6)
    Structure S;
    int32_t n_clusters = 0, n_leaves = 0;
    std::vector<int32_t> gid_of_pre;
    std::vector<int32_t> level_off;  // clusters of level l: gids [level_off[l], level_off[l+1])
    // device
    std::vector<DevBuf> bufs;
    int32_t* d_perm = nullptr;
    int32_t* d_iperm = nullptr;
    double* d_diag = nullptr;
    int32_t* d_child0 = nullptr;
    int32_t* d_child1 = nullptr;
    int32_t* d_parent = nullptr;
    int32_t* d_front = nullptr;
    void* d_e = nullptr;
    void* d_pool_wt = nullptr;
    void* d_pool_s = nullptr;
    double* d_cgeo = nullptr;        // generated coupling: per cluster centre xyz, half extent xyz
    void* d_pool_leaf = nullptr;
    ItemDesc* d_items_fwd = nullptr;
    BlkDesc* d_blks_fwd = nullptr;
    ItemDesc* d_items_cpl = nullptr;
    BlkDesc* d_blks_cpl = nullptr;
    ItemDesc* d_items_leaf = nullptr;
    BlkDesc* d_blks_leaf = nullptr;
    ItemDesc* d_items_near = nullptr;   // the leaf items without their V_t block
    ItemDesc* d_items_v = nullptr;      // the leaf items' V_t block alone
    // row basis regenerated in the apply: the leaves and the node coordinates
    // (cluster order, N x 3)
    bool regen_v = false;
    std::vector<VLeaf> vgen;
    VLeaf* d_vgen = nullptr;
    double* d_vxyz = nullptr;
    int64_t* d_ns_off = nullptr;
    int32_t* d_ns_pos = nullptr;
    double* d_ns_val = nullptr;
    void* d_ws = nullptr;
    size_t ws_bytes = 0, ws_x = 0, ws_x64 = 0, ws_y64 = 0, ws_xh = 0;
    int32_t n_items_fwd = 0, n_items_cpl = 0, n_items_leaf = 0;
    // near-field items launched at the fork; the rest wait for the first
    // coupling launch (stored or recompressed coupling)
    int32_t n_near_head = 0;
    int32_t rt_leaf = 1;
    // LDS each FP32 generated-coupling workgroup reserves beyond its own
    // arrays: a quarter of a CU's, so that at most three share a CU (their
    // registers would allow six) and the near field running beside them keeps
    // its share.  The FP64 kernel's registers already allow only four.
    size_t cpl_lds = 0;
    int kp = 0;                      // stored columns of a coupling block
    bool materialized = false;
    // offload: device buffers parked in pinned host memory
    bool offloaded = false;
    struct Parked { void** field; void* host; size_t bytes; bool scratch; };
    std::vector<bool> empty_field;   // fields() entries that hold no bytes (NULL after the build)
    // the near field runs on this stream while the far-field chain runs on the caller's;
    // fork and join order it against the caller's stream (created once: an apply
    // creates no event)
    hipStream_t side = nullptr, side2 = nullptr;
    hipEvent_t fork_ev = nullptr, mid_ev = nullptr, join_ev = nullptr, cut_ev = nullptr, upper_ev = nullptr;
    // a reload enqueued on a stream: every later use of the device buffers waits for it
    hipEvent_t ready = nullptr;
    bool ready_pending = false;
    std::vector<Parked> parked;
    // host-side plan
    std::vector<int32_t> child0, child1, parent;
    // downward pass: the clusters of level down_l0 and the leaves above it get
    // their yhat in one launch, each from its path to the root; the levels
    // below follow one launch per level
    std::vector<int32_t> down_front;
    int32_t down_l0 = 0;
    std::vector<double> boxes;
    std::vector<double> cgeo;
    std::vector<char> far_dense;     // per block-tree admissible block: stored as exact entries
    std::vector<LeafDesc> leaves, vleaves;
    std::vector<FarDesc> fars;
    std::vector<NearDesc> nears;
    std::vector<ItemDesc> items_fwd, items_cpl, items_leaf, items_near, items_v;
    std::vector<BlkDesc> blks_fwd, blks_cpl, blks_leaf;
    int64_t off_wt = 0, off_s = 0, off_l = 0, off_v = 0;
    // algebraic recompression (recompress_eps > 0): adaptive ranks of the row
    // and column bases; x^ rows of cluster g start at xo[g] (column ranks),
    // y^ rows at yo[g] (row ranks); the transfers have their own pools and
    // per-level item ranges
    bool rec = false;
    std::vector<int32_t> far_t, far_s;
    std::vector<int32_t> rank_row, rank_col;
    void* d_pool_up = nullptr;
    void* d_pool_down = nullptr;
    void* d_pool_q = nullptr;
    ItemDesc* d_items_up = nullptr;
    BlkDesc* d_blks_up = nullptr;
    ItemDesc* d_items_down = nullptr;
    BlkDesc* d_blks_down = nullptr;
    BlkDesc* d_blks_v = nullptr;
    std::vector<int32_t> up_off, up_end, down_off;   // item ranges by level: [up_off[l], up_end[l]),
                                                     // [down_off[l], down_off[l + 1])
    // the coupling in two launches: blocks whose source cluster is at level
    // up_cut or deeper (d_items_cpl, storing y^) run while the upward pass
    // finishes levels above up_cut on side2; the rest (d_items_cpl_b) add
    ItemDesc* d_items_cpl_b = nullptr;
    int32_t n_items_cpl_b = 0;
    int32_t up_cut = 0;
    int32_t n_items_v = 0;           // recompressed: leaf output items (Q_t y^_t)
    int32_t rt_fwd = 1, rt_up = 1, rt_cpl = 1, rt_down = 1;
    h2dlp_stats st{};
    // profiling
    int prof = 0;                    // bit q: record launches of kind q
    struct Rec { int kind; hipEvent_t a, b; };
    std::vector<Rec> recs;
    double prof_ms[H2DLP_NKINDS] = {0};
    int64_t prof_n[H2DLP_NKINDS] = {0};

    ~h2dlp_ctx() {
        if (device < 0) return;   // plan only: nothing on a device
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        for (auto& r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        if (ready) { (void)hipEventSynchronize(ready); (void)hipEventDestroy(ready); }
        if (side) { (void)hipStreamSynchronize(side); (void)hipStreamDestroy(side); }
        if (side2) { (void)hipStreamSynchronize(side2); (void)hipStreamDestroy(side2); }
        if (cut_ev) (void)hipEventDestroy(cut_ev);
        if (upper_ev) (void)hipEventDestroy(upper_ev);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        if (mid_ev) (void)hipEventDestroy(mid_ev);
        if (join_ev) (void)hipEventDestroy(join_ev);
        for (auto& b : bufs) if (b.p) (void)hipFree(b.p);
        for (auto& p : parked) if (p.host) (void)hipHostFree(p.host);
        (void)hipSetDevice(cur);
    }

    // every device pointer the apply reads, with the field that holds it
    std::vector<std::pair<void**, bool>> fields() {
        return {{(void**)&d_perm, false}, {(void**)&d_iperm, false}, {(void**)&d_diag, false},
                {(void**)&d_child0, false}, {(void**)&d_child1, false}, {(void**)&d_parent, false},
                {(void**)&d_front, false},
                {(void**)&d_e, false}, {(void**)&d_pool_wt, false}, {(void**)&d_pool_s, false},
                {(void**)&d_cgeo, false},
                {(void**)&d_pool_leaf, false}, {(void**)&d_items_fwd, false}, {(void**)&d_blks_fwd, false},
                {(void**)&d_items_cpl, false}, {(void**)&d_blks_cpl, false}, {(void**)&d_items_leaf, false},
                {(void**)&d_blks_leaf, false}, {(void**)&d_items_near, false}, {(void**)&d_items_v, false},
                {(void**)&d_ns_off, false}, {(void**)&d_ns_pos, false},
                {(void**)&d_ns_val, false}, {(void**)&d_pool_up, false}, {(void**)&d_pool_down, false},
                {(void**)&d_pool_q, false}, {(void**)&d_items_up, false}, {(void**)&d_blks_up, false},
                {(void**)&d_items_down, false}, {(void**)&d_blks_down, false}, {(void**)&d_blks_v, false},
                {(void**)&d_items_cpl_b, false}, {(void**)&d_vgen, false}, {(void**)&d_vxyz, false},
                {(void**)&d_ws, true}};
    }
    size_t bytes_of(void* p) const {
        for (const auto& b : bufs) if (b.p == p) return b.bytes;
        return 0;
    }

    template <typename P>
    P* alloc(size_t bytes, int64_t* account) {
        DevBuf b;
        b.bytes = bytes;
        if (bytes > 0) {
            const hipError_t e = hipMalloc(&b.p, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw std::bad_alloc();
            }
        }
        bufs.push_back(b);
        if (account) *account += int64_t(bytes);
        return static_cast<P*>(b.p);
    }

    template <typename V>
    typename V::value_type* upload(const V& v, int64_t* account, hipStream_t s) {
        typedef typename V::value_type E;
        E* p = alloc<E>(v.size() * sizeof(E), account);
        if (!v.empty()) check(hipMemcpyAsync(p, v.data(), v.size() * sizeof(E), hipMemcpyHostToDevice, s), "upload");
        return p;
    }

    void release(void* p) {
        for (auto& b : bufs)
            if (b.p == p) {
                hipFree(b.p);
                b.p = nullptr;
                b.bytes = 0;
            }
    }
};

namespace {

// Share of the near-field entries (stored or recompressed coupling) launched
// after the first coupling launch instead of at the fork: they keep HBM busy
// during the second coupling launch and the downward pass, which move little.
constexpr double kNearTail = 0.3;

// Host part of a build: block structure, level-order numbering, pool layouts
// and block descriptors, byte counts.  No HIP call.
int plan_impl(h2dlp_ctx* h, const h2dlp_mesh* mesh, const h2dlp_options* o) {
    h->opt = *o;
    h->m = o->order;
    h->k = o->order * o->order * o->order;
    h->prec = o->precision;
    h->elem = h->prec == H2DLP_FP64 ? 8 : 4;
    h->elem_s = h->prec == H2DLP_BF16X6 ? 6 : h->elem;
    const bool fp64 = h->prec == H2DLP_FP64;
    const bool rec = o->recompress_eps > 0.0;
    h->rec = rec;
    const bool regen = o->row_basis == H2DLP_ROW_BASIS_GENERATED;
    h->regen_v = regen;
    const bool has_v = !rec && !regen;     // a leaf item's first block is V_t

    std::string err = build_structure(h->S, mesh->xyz, mesh->n_nodes, mesh->tri, mesh->n_tris, o->leaf, o->eta,
                                      o->alpha, !fp64);
    if (!err.empty()) return fail(H2DLP_EINVAL, err);
    Structure& S = h->S;
    const int64_t N = S.n_nodes, T = S.n_tris;
    const int m = h->m, k = h->k;
    const int32_t C = int32_t(S.cl.size());
    h->n_clusters = C;

    // level-major cluster numbering (clusters of one level contiguous, left to right)
    std::vector<int32_t> order(C);
    for (int32_t c = 0; c < C; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return S.cl[a].level < S.cl[b].level; });
    h->gid_of_pre.assign(C, 0);
    for (int32_t g = 0; g < C; ++g) h->gid_of_pre[order[g]] = g;
    h->level_off.assign(S.depth + 2, 0);
    for (int32_t c = 0; c < C; ++c) h->level_off[S.cl[c].level + 1]++;
    for (int l = 0; l <= S.depth; ++l) h->level_off[l + 1] += h->level_off[l];
    h->child0.assign(C, -1);
    h->child1.assign(C, -1);
    h->parent.assign(C, -1);
    h->boxes.assign(6 * size_t(C), 0.0);
    for (int32_t c = 0; c < C; ++c) {
        const int32_t g = h->gid_of_pre[c];
        const Cluster& X = S.cl[c];
        if (!X.leaf()) { h->child0[g] = h->gid_of_pre[X.child0]; h->child1[g] = h->gid_of_pre[X.child1]; }
        if (X.parent >= 0) h->parent[g] = h->gid_of_pre[X.parent];
        for (int a = 0; a < 3; ++a) { h->boxes[6 * size_t(g) + a] = X.lo[a]; h->boxes[6 * size_t(g) + 3 + a] = X.hi[a]; }
    }
    // the deepest level down to which no level holds more than kPathFront
    // clusters (paths of at most kMaxPath clusters), and the leaves above it
    h->down_l0 = 0;
    for (int l = 1; l <= S.depth && l < kMaxPath; ++l) {
        if (h->level_off[l + 1] - h->level_off[l] > kPathFront) break;
        h->down_l0 = l;
    }
    h->down_front.clear();
    for (int32_t g = 0; g < h->level_off[h->down_l0 + 1]; ++g)
        if (g >= h->level_off[h->down_l0] || h->child0[g] < 0) h->down_front.push_back(g);
    std::vector<int32_t> leaf_pre;
    for (int32_t g = 0; g < C; ++g)
        if (S.cl[order[g]].leaf()) leaf_pre.push_back(order[g]);
    h->n_leaves = int32_t(leaf_pre.size());

    // leaf forward: one item and one block (W_s^T, k x n_s) per leaf
    h->leaves.resize(leaf_pre.size());
    int64_t off_wt = 0;
    for (size_t q = 0; q < leaf_pre.size(); ++q) {
        const Cluster& X = S.cl[leaf_pre[q]];
        const int32_t g = h->gid_of_pre[leaf_pre[q]];
        off_wt = align_block(off_wt);
        h->leaves[q] = LeafDesc{int32_t(X.begin), int32_t(X.size()), g, 0, off_wt};
        h->items_fwd.push_back(ItemDesc{g * k, k, int32_t(h->blks_fwd.size()), int32_t(h->blks_fwd.size() + 1)});
        h->blks_fwd.push_back(BlkDesc{off_wt, int32_t(X.size()), int32_t(X.begin)});
        off_wt += int64_t(k) * X.size();
    }
    // admissible blocks small enough to keep as exact entries (|t| |s| <= dense_far_max)
    h->far_dense.assign(S.far.size(), 0);
    int64_t n_far_dense = 0, dense_entries = 0;
    for (size_t b = 0; b < S.far.size(); ++b) {
        const int64_t e = S.cl[S.far[b].first].size() * S.cl[S.far[b].second].size();
        if (e <= o->dense_far_max) {
            h->far_dense[b] = 1;
            ++n_far_dense;
            dense_entries += e;
        }
    }
    // coupling: one item per cluster (level order), its low-rank blocks sorted by source
    std::vector<std::vector<int32_t>> far_by_t(C);
    for (size_t b = 0; b < S.far.size(); ++b)
        if (!h->far_dense[b]) far_by_t[h->gid_of_pre[S.far[b].first]].push_back(h->gid_of_pre[S.far[b].second]);
    int64_t off_s = 0;
    const bool gen = o->coupling == H2DLP_COUPLING_GENERATED;
    const int kp = bf16_parts(h->prec) > 0 ? bf16s_cols(k) : coupling_cols(k);
    h->kp = kp;
    for (int32_t g = 0; g < C; ++g) {
        auto& lst = far_by_t[g];
        std::sort(lst.begin(), lst.end());
        h->items_cpl.push_back(ItemDesc{g * k, k, int32_t(h->blks_cpl.size()), int32_t(h->blks_cpl.size() + lst.size())});
        for (int32_t s : lst) {
            if (rec) {                   // low-rank pairs, in this order; layouts follow the ranks
                h->far_t.push_back(g);
                h->far_s.push_back(s);
            }
            if (gen) {                   // nothing stored: a_off names the source cluster
                h->blks_cpl.push_back(BlkDesc{int64_t(s), k, s * k});
                continue;
            }
            off_s = align_block(off_s);
            h->fars.push_back(FarDesc{g, s, off_s});
            h->blks_cpl.push_back(BlkDesc{off_s, kp, s * k});
            off_s += int64_t(k) * kp;
        }
    }
    // leaf output: V_t (n_t x k) then the near blocks of t (sorted by source position)
    // (an exact admissible block (t, s) enters every leaf of t, restricted to that leaf's rows)
    std::vector<std::vector<int32_t>> near_by_t(C);
    for (size_t b = 0; b < S.near.size(); ++b) near_by_t[S.near[b].first].push_back(S.near[b].second);
    for (size_t b = 0; b < S.far.size(); ++b) {
        if (!h->far_dense[b]) continue;
        std::vector<int32_t> stack{S.far[b].first};
        while (!stack.empty()) {
            const int32_t c = stack.back();
            stack.pop_back();
            if (S.cl[c].leaf()) near_by_t[c].push_back(S.far[b].second);
            else { stack.push_back(S.cl[c].child0); stack.push_back(S.cl[c].child1); }
        }
    }
    h->vleaves.resize(leaf_pre.size());
    int64_t off_l = 0, off_v = 0, near_entries = 0;
    for (size_t q = 0; q < leaf_pre.size(); ++q) {
        const int32_t t = leaf_pre[q];
        const Cluster& X = S.cl[t];
        auto& lst = near_by_t[t];
        std::sort(lst.begin(), lst.end(), [&](int32_t a, int32_t b) { return S.cl[a].begin < S.cl[b].begin; });
        const int32_t b0 = int32_t(h->blks_leaf.size());
        h->items_leaf.push_back(ItemDesc{int32_t(X.begin), int32_t(X.size()), b0,
                                         int32_t(b0 + (has_v ? 1 : 0) + lst.size())});
        if (rec) {           // V_t in FP64 for the recompression only, in a pool of the build
            off_v = align_block(off_v);
            h->vleaves[q] = LeafDesc{int32_t(X.begin), int32_t(X.size()), h->gid_of_pre[t], 0, off_v};
            off_v += int64_t(X.size()) * k;
        } else if (regen) {  // V_t evaluated in the apply from the leaf's box
            const int32_t g = h->gid_of_pre[t];
            VLeaf v{int32_t(X.begin), int32_t(X.size()), g * k, 0, {}};
            for (int a = 0; a < 6; ++a) v.box[a] = h->boxes[6 * size_t(g) + a];
            h->vgen.push_back(v);
        } else {
            off_l = align_block(off_l);
            h->vleaves[q] = LeafDesc{int32_t(X.begin), int32_t(X.size()), h->gid_of_pre[t], 0, off_l};
            h->blks_leaf.push_back(BlkDesc{off_l, k, SRC1 | (h->gid_of_pre[t] * k)});
            off_l += int64_t(X.size()) * k;
        }
        for (int32_t s : lst) {
            const Cluster& Y = S.cl[s];
            off_l = align_block(off_l);
            h->nears.push_back(NearDesc{int32_t(X.begin), int32_t(X.size()), int32_t(Y.begin), int32_t(Y.size()), off_l});
            h->blks_leaf.push_back(BlkDesc{off_l, int32_t(Y.size()), int32_t(Y.begin)});
            off_l += int64_t(X.size()) * Y.size();
            near_entries += int64_t(X.size()) * Y.size();
        }
    }
    h->n_items_fwd = int32_t(h->items_fwd.size());
    h->n_items_cpl = int32_t(h->items_cpl.size());
    h->n_items_leaf = int32_t(h->items_leaf.size());
    for (const ItemDesc& d : h->items_leaf) {     // block 0 of a leaf item is V_t, the rest near blocks
        h->items_near.push_back(ItemDesc{d.out_row, d.m, d.blk_begin + (has_v ? 1 : 0), d.blk_end});
        if (has_v) h->items_v.push_back(ItemDesc{d.out_row, d.m, d.blk_begin, d.blk_begin + 1});
    }
    // near-field items in node (depth-first) order rather than level order:
    // neighbouring items, dealt to one XCD in chunks, are then neighbouring
    // leaves whatever their level, and share source rows of x in that L2
    std::stable_sort(h->items_near.begin(), h->items_near.end(),
                     [](const ItemDesc& a, const ItemDesc& b) { return a.out_row < b.out_row; });
    {
        // the last kNearTail of the near-field entries run after the first
        // coupling launch, beside the latency-bound passes that follow it
        std::vector<int64_t> cum(h->items_near.size() + 1, 0);
        for (size_t q = 0; q < h->items_near.size(); ++q) {
            const ItemDesc& d = h->items_near[q];
            int64_t e = 0;
            for (int32_t b = d.blk_begin; b < d.blk_end; ++b) e += int64_t(d.m) * h->blks_leaf[b].k;
            cum[q + 1] = cum[q] + e;
        }
        size_t head = 0;
        while (head < h->items_near.size() && double(cum[head]) < (1.0 - kNearTail) * double(cum.back())) ++head;
        h->n_near_head = int32_t(head);
    }
    h->rt_leaf = (o->leaf + 15) / 16;
    h->off_v = off_v;
    h->off_wt = off_wt;
    h->off_s = off_s;
    h->off_l = off_l;

    const size_t e = h->elem;
    // workspace of one 16-column pass: x (operator precision), x64 (FP32 path),
    // y64, xhat and yhat
    h->ws_x = align_up(e * size_t(N) * RHS_TILE);
    h->ws_x64 = fp64 ? 0 : align_up(8 * size_t(N) * RHS_TILE);
    h->ws_y64 = align_up(8 * size_t(N) * RHS_TILE);
    h->ws_xh = align_up(e * size_t(C) * k * RHS_TILE);
    h->ws_bytes = h->ws_x + h->ws_x64 + h->ws_y64 + 2 * h->ws_xh;

    h2dlp_stats& st = h->st;
    st = h2dlp_stats{};
    st.n_nodes = N;
    st.n_tris = T;
    st.order = m;
    st.leaf = o->leaf;
    st.k = k;
    st.precision = h->prec;
    st.depth = S.depth;
    st.n_clusters = C;
    st.n_leaves = h->n_leaves;
    st.n_far = int64_t(S.far.size()) - n_far_dense;
    st.n_far_dense = n_far_dense;
    st.dense_far_entries = dense_entries;
    st.n_near = int64_t(S.near.size());
    st.coupling_entries = st.n_far * k * k;
    st.near_entries = near_entries - dense_entries;
    st.nearsing_entries = fp64 ? 0 : int64_t(S.ring_pos.size());
    st.bytes_coupling = gen ? 0 : int64_t(h->elem_s * size_t(st.coupling_entries));
    if (gen) {
        h->cgeo.resize(size_t(6) * C);
        for (int32_t g = 0; g < C; ++g)
            for (int a = 0; a < 3; ++a) {
                const double lo = h->boxes[6 * size_t(g) + a], hi = h->boxes[6 * size_t(g) + 3 + a];
                h->cgeo[6 * size_t(g) + a] = 0.5 * (lo + hi);
                h->cgeo[6 * size_t(g) + 3 + a] = 0.5 * (hi - lo);
            }
    }
    st.bytes_near = int64_t(e * size_t(near_entries));
    if (!fp64) st.bytes_near += int64_t((N + 1) * 8 + S.ring_pos.size() * (4 + 8));
    // a regenerated row basis keeps the node coordinates and the leaf boxes
    const int64_t regen_bytes = regen ? int64_t(24 * N + int64_t(sizeof(VLeaf)) * h->n_leaves) : 0;
    st.bytes_bases = int64_t(e * size_t((regen ? 1 : 2) * N * int64_t(k))) + regen_bytes;
    st.bytes_transfer = int64_t(e * size_t(C) * 3 * m * m);
    st.bytes_other = int64_t(N * 8 + 3 * int64_t(C) * 4 + N * 8 + int64_t(h->cgeo.size()) * 8 +
                             (h->items_fwd.size() + h->items_cpl.size() + h->items_leaf.size()) * sizeof(ItemDesc) +
                             (h->blks_fwd.size() + h->blks_cpl.size() + h->blks_leaf.size()) * sizeof(BlkDesc));
    st.workspace_bytes = int64_t(h->ws_bytes);
    st.bytes_resident = int64_t(e * size_t(off_wt + off_l) + h->elem_s * size_t(off_s)) + st.bytes_transfer +
                        st.bytes_other + regen_bytes +
                        st.workspace_bytes + (fp64 ? 0 : int64_t((N + 1) * 8 + S.ring_pos.size() * (4 + 8)));
    const double h2_bytes = double(st.bytes_coupling + st.bytes_near + st.bytes_bases + st.bytes_transfer);
    st.compression = 1.0 - h2_bytes / (8.0 * double(N) * double(N));
    st.rank_sum_row = st.rank_sum_col = int64_t(C) * k;     // the interpolation ranks (an upper bound
    st.rank_max_row = st.rank_max_col = k;                  //   when recompressed: set by the build)
    return H2DLP_OK;
}

int32_t row_tiles(const std::vector<int32_t>& r) {
    int32_t mx = 1;
    for (int32_t v : r) mx = std::max(mx, v);
    return (mx + 15) / 16;
}

// The recompressed operator: ranks from the GPU recompression of the FP64
// interpolation bases (wt64: W_s^T blocks at h->leaves, v64: V_t blocks at
// h->vleaves), then every apply descriptor and pool laid out by those ranks.
void recompress_impl(h2dlp_ctx* h, const double* d_boxes, const double* wt64, const double* v64, int64_t* kept,
                     hipStream_t stream) {
    const Structure& S = h->S;
    const int k = h->k, m = h->m;
    const int32_t C = h->n_clusters;
    const size_t e = h->elem;
    RecompressPlan P;
    P.m = m;
    P.k = k;
    P.n_clusters = C;
    P.depth = S.depth;
    P.level_off = h->level_off;
    P.child0 = h->child0;
    P.child1 = h->child1;
    P.parent = h->parent;
    P.leaf_n.assign(C, 0);
    int maxleaf = 1;
    for (const LeafDesc& L : h->leaves) { P.leaf_n[L.gid] = L.n; maxleaf = std::max(maxleaf, int(L.n)); }
    P.rows = std::max(2 * k, maxleaf);
    P.far_t = h->far_t;
    P.far_s = h->far_s;
    P.eps = h->opt.recompress_eps;
    const int64_t rk = int64_t(P.rows) * k;

    // leaf bases into per-cluster column-major slots
    double* vslot = h->alloc<double>(sizeof(double) * size_t(C) * rk, nullptr);
    double* wslot = h->alloc<double>(sizeof(double) * size_t(C) * rk, nullptr);
    check(hipMemsetAsync(vslot, 0, sizeof(double) * size_t(C) * rk, stream), "clear");
    check(hipMemsetAsync(wslot, 0, sizeof(double) * size_t(C) * rk, stream), "clear");
    {
        std::vector<GatherDesc> gv, gw;
        for (const LeafDesc& L : h->vleaves) gv.push_back(GatherDesc{L.a_off, L.gid, L.n});
        for (const LeafDesc& L : h->leaves) gw.push_back(GatherDesc{L.a_off, L.gid, L.n});
        GatherDesc* dgv = h->upload(gv, nullptr, stream);
        GatherDesc* dgw = h->upload(gw, nullptr, stream);
        check(launch_gather_leaf_basis(dgv, int64_t(gv.size()), v64, k, P.rows, false, vslot, stream), "gather");
        check(launch_gather_leaf_basis(dgw, int64_t(gw.size()), wt64, k, P.rows, true, wslot, stream), "gather");
        check(hipStreamSynchronize(stream), "gather");
        h->release(dgv);
        h->release(dgw);
    }
    RecompressResult R;
    std::string err = recompress(P, d_boxes, vslot, wslot, stream, &R);
    h->release(vslot);
    h->release(wslot);
    if (!err.empty()) throw HipError{hipErrorUnknown, "recompression: " + err};
    const std::vector<int32_t>& rr = R.rank_row;
    const std::vector<int32_t>& rc = R.rank_col;
    h->rank_row = rr;
    h->rank_col = rc;
    std::vector<int32_t> xo(C + 1, 0), yo(C + 1, 0);
    for (int32_t g = 0; g < C; ++g) { xo[g + 1] = xo[g] + rc[g]; yo[g + 1] = yo[g] + rr[g]; }

    // descriptors, pool offsets and the stores from the FP64 slots
    std::vector<StoreDesc> st_wt, st_up, st_down, st_q;
    std::vector<BlkDesc> blks_up, blks_down, blks_v;
    std::vector<ItemDesc> items_up, items_down;
    h->items_fwd.clear(); h->blks_fwd.clear(); h->items_cpl.clear(); h->blks_cpl.clear(); h->items_v.clear();
    int64_t o_wt = 0, o_up = 0, o_s = 0, o_down = 0, o_q = 0;
    double* Uc = R.u_col;
    double* Ur = R.u_row;
    for (const LeafDesc& L : h->leaves) {              // x^_s = Q'_s^T x|_s
        const int32_t r = rc[L.gid];
        if (r == 0) continue;
        o_wt = align_block(o_wt);
        h->items_fwd.push_back(ItemDesc{xo[L.gid], r, int32_t(h->blks_fwd.size()), int32_t(h->blks_fwd.size() + 1)});
        h->blks_fwd.push_back(BlkDesc{o_wt, L.n, L.pos});
        st_wt.push_back(StoreDesc{Uc + int64_t(L.gid) * rk, P.rows, r, L.n, 1, o_wt});
        o_wt += int64_t(r) * L.n;
    }
    h->up_off.assign(S.depth + 2, 0);
    h->up_end.assign(S.depth + 2, 0);
    for (int l = S.depth; l >= 0; --l) {               // x^_t = sum_c F'_c^T x^_c (levels deepest first)
        h->up_off[l] = int32_t(items_up.size());
        for (int32_t g = h->level_off[l]; g < h->level_off[l + 1]; ++g) {
            if (h->child0[g] < 0 || rc[g] == 0) continue;
            const int32_t b0 = int32_t(blks_up.size());
            for (int side = 0; side < 2; ++side) {
                const int32_t c = side == 0 ? h->child0[g] : h->child1[g];
                if (rc[c] == 0) continue;
                o_up = align_block(o_up);
                blks_up.push_back(BlkDesc{o_up, rc[c], xo[c]});
                st_up.push_back(StoreDesc{Uc + int64_t(g) * rk + side * k, P.rows, rc[g], rc[c], 1, o_up});
                o_up += int64_t(rc[g]) * rc[c];
            }
            items_up.push_back(ItemDesc{xo[g], rc[g], b0, int32_t(blks_up.size())});
        }
        h->up_end[l] = int32_t(items_up.size());
    }
    // y^_t = sum_s S'_ts x^_s in two launches split at level up_cut of the
    // source: the deepest cut that leaves at most 1/32 of the coupling
    // entries to the second launch, so that the latency-bound top of the
    // upward pass runs beside the first (at 655362 nodes, FP32: 2.09 ms
    // against 2.11 ms with 1/8)
    std::vector<int32_t> lvl(C, 0);
    for (int l = 0; l <= S.depth; ++l)
        for (int32_t g = h->level_off[l]; g < h->level_off[l + 1]; ++g) lvl[g] = l;
    {
        std::vector<int64_t> by_level(S.depth + 2, 0);
        int64_t total = 0;
        for (size_t b = 0; b < h->far_t.size(); ++b) {
            const int64_t n = int64_t(rr[h->far_t[b]]) * rc[h->far_s[b]];
            by_level[lvl[h->far_s[b]]] += n;
            total += n;
        }
        constexpr int64_t share = 32;
        h->up_cut = 0;
        int64_t above = 0;                             // entries with sources above level l
        for (int l = 0; l <= S.depth; ++l) {
            if (share * (above + by_level[l]) > total) break;
            above += by_level[l];
            h->up_cut = l + 1;
        }
        h->up_cut = std::min(h->up_cut, S.depth);
    }
    std::vector<int64_t> a_s(h->far_t.size(), 0);
    std::vector<ItemDesc> items_cpl_b;
    for (size_t b = 0, g = 0; g < size_t(C); ++g) {
        const int32_t b0 = int32_t(h->blks_cpl.size());
        const size_t bb = b;
        for (; b < h->far_t.size() && h->far_t[b] == int32_t(g); ++b) {}
        int32_t nb_a = 0;
        for (int pass = 0; pass < 2; ++pass)           // sources at up_cut or deeper first
            for (size_t q = bb; q < b; ++q) {
                const int32_t s = h->far_s[q];
                if (rr[g] == 0 || rc[s] == 0 || (lvl[s] >= h->up_cut) != (pass == 0)) continue;
                o_s = align_block(o_s);
                a_s[q] = o_s;
                h->blks_cpl.push_back(BlkDesc{o_s, rc[s], xo[s]});
                o_s += int64_t(rr[g]) * rc[s];
                nb_a += pass == 0;
            }
        if (rr[g] == 0) continue;
        const int32_t b1 = int32_t(h->blks_cpl.size());
        h->items_cpl.push_back(ItemDesc{yo[g], rr[g], b0, b0 + nb_a});
        if (b0 + nb_a < b1) items_cpl_b.push_back(ItemDesc{yo[g], rr[g], b0 + nb_a, b1});
    }
    h->down_off.assign(S.depth + 2, 0);
    for (int l = 0; l <= S.depth; ++l) {               // y^_c += F_c y^_parent
        h->down_off[l] = int32_t(items_down.size());
        for (int32_t c = h->level_off[l]; c < h->level_off[l + 1]; ++c) {
            const int32_t p = h->parent[c];
            if (p < 0 || rr[c] == 0 || rr[p] == 0) continue;
            o_down = align_block(o_down);
            items_down.push_back(ItemDesc{yo[c], rr[c], int32_t(blks_down.size()), int32_t(blks_down.size() + 1)});
            blks_down.push_back(BlkDesc{o_down, rr[p], yo[p]});
            st_down.push_back(StoreDesc{Ur + int64_t(p) * rk + (c == h->child1[p] ? k : 0), P.rows, rr[c], rr[p], 0,
                                        o_down});
            o_down += int64_t(rr[c]) * rr[p];
        }
        h->down_off[l + 1] = int32_t(items_down.size());
    }
    for (const LeafDesc& L : h->vleaves) {             // y|_t += Q_t y^_t
        const int32_t r = rr[L.gid];
        if (r == 0) continue;
        o_q = align_block(o_q);
        h->items_v.push_back(ItemDesc{L.pos, L.n, int32_t(blks_v.size()), int32_t(blks_v.size() + 1)});
        blks_v.push_back(BlkDesc{o_q, r, SRC1 | yo[L.gid]});
        st_q.push_back(StoreDesc{Ur + int64_t(L.gid) * rk, P.rows, L.n, r, 0, o_q});
        o_q += int64_t(L.n) * r;
    }
    h->d_pool_wt = h->alloc<void>(e * size_t(std::max<int64_t>(o_wt, 1)), kept);
    h->d_pool_up = h->alloc<void>(e * size_t(std::max<int64_t>(o_up, 1)), kept);
    h->d_pool_s = h->alloc<void>(e * size_t(std::max<int64_t>(o_s, 1)), kept);
    h->d_pool_down = h->alloc<void>(e * size_t(std::max<int64_t>(o_down, 1)), kept);
    h->d_pool_q = h->alloc<void>(e * size_t(std::max<int64_t>(o_q, 1)), kept);
    for (auto* list : {&st_wt, &st_up, &st_down, &st_q}) {
        void* pool = list == &st_wt ? h->d_pool_wt : list == &st_up ? h->d_pool_up
                   : list == &st_down ? h->d_pool_down : h->d_pool_q;
        if (list->empty()) continue;
        StoreDesc* d = h->upload(*list, nullptr, stream);
        check(launch_store_layout(d, int64_t(list->size()), h->prec, pool, stream), "store bases");
        check(hipStreamSynchronize(stream), "store bases");
        h->release(d);
    }
    err = recompress_couplings(P, d_boxes, R, a_s, h->prec, h->d_pool_s, stream);
    R.release();
    if (!err.empty()) throw HipError{hipErrorUnknown, "recompression: " + err};
    h->d_items_fwd = h->upload(h->items_fwd, kept, stream);
    h->d_blks_fwd = h->upload(h->blks_fwd, kept, stream);
    h->d_items_up = h->upload(items_up, kept, stream);
    h->d_blks_up = h->upload(blks_up, kept, stream);
    h->d_items_cpl = h->upload(h->items_cpl, kept, stream);
    h->d_blks_cpl = h->upload(h->blks_cpl, kept, stream);
    h->d_items_cpl_b = items_cpl_b.empty() ? nullptr : h->upload(items_cpl_b, kept, stream);
    h->n_items_cpl_b = int32_t(items_cpl_b.size());
    h->d_items_down = h->upload(items_down, kept, stream);
    h->d_blks_down = h->upload(blks_down, kept, stream);
    h->d_items_v = h->upload(h->items_v, kept, stream);
    h->n_items_v = int32_t(h->items_v.size());
    h->d_blks_v = h->upload(blks_v, kept, stream);
    h->n_items_fwd = int32_t(h->items_fwd.size());
    h->n_items_cpl = int32_t(h->items_cpl.size());
    h->rt_fwd = row_tiles(rc);
    h->rt_up = row_tiles(rc);
    h->rt_cpl = row_tiles(rr);
    h->rt_down = row_tiles(rr);
    // workspace and sizes with the ranks found
    h->ws_xh = align_up(e * size_t(std::max({xo[C], yo[C], 1})) * RHS_TILE);
    h->ws_bytes = h->ws_x + h->ws_x64 + h->ws_y64 + 2 * h->ws_xh;
    h2dlp_stats& st = h->st;
    st.coupling_entries = 0;
    for (size_t b = 0; b < h->far_t.size(); ++b) st.coupling_entries += int64_t(rr[h->far_t[b]]) * rc[h->far_s[b]];
    st.bytes_coupling = int64_t(e) * st.coupling_entries;
    st.bytes_bases = int64_t(e) * (o_wt + o_q);
    st.bytes_transfer = int64_t(e) * (o_up + o_down);
    st.workspace_bytes = int64_t(h->ws_bytes);
    st.rank_sum_row = yo[C];
    st.rank_sum_col = xo[C];
    st.rank_max_row = *std::max_element(rr.begin(), rr.end());
    st.rank_max_col = *std::max_element(rc.begin(), rc.end());
    const double h2_bytes = double(st.bytes_coupling + st.bytes_near + st.bytes_bases + st.bytes_transfer);
    st.compression = 1.0 - h2_bytes / (8.0 * double(S.n_nodes) * double(S.n_nodes));
}

// The handle's own streams and events (created once: an apply creates none) and
// the device's LDS figures for the generated coupling's occupancy shaping.
void make_streams(h2dlp_ctx* h) {
    check(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking), "side stream");
    check(hipStreamCreateWithFlags(&h->side2, hipStreamNonBlocking), "side stream");
    check(hipEventCreateWithFlags(&h->cut_ev, hipEventDisableTiming), "event");
    check(hipEventCreateWithFlags(&h->upper_ev, hipEventDisableTiming), "event");
    check(hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming), "event");
    check(hipEventCreateWithFlags(&h->mid_ev, hipEventDisableTiming), "event");
    check(hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming), "event");
    int dev = 0, lds_cu = 0, lds_wg = 0;
    check(hipGetDevice(&dev), "device");
    check(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev), "attribute");
    check(hipDeviceGetAttribute(&lds_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "attribute");
    h->cpl_lds = size_t(std::max(0, std::min(lds_cu / 4, lds_wg)));
}

// The end of a build or a load: which buffers are empty, host descriptors dropped.
void finish_materialize(h2dlp_ctx* h) {
    h->empty_field.clear();
    for (auto& f : h->fields()) h->empty_field.push_back(*f.first == nullptr);
    h->leaves.clear(); h->leaves.shrink_to_fit();
    h->vleaves.clear(); h->vleaves.shrink_to_fit();
    h->fars.clear(); h->fars.shrink_to_fit();
    h->nears.clear(); h->nears.shrink_to_fit();
    h->materialized = true;
}

// Device part of a build: upload, generate every block in FP64 arithmetic, free the build-only arrays.
int materialize_impl(h2dlp_ctx* h, hipStream_t stream) {
    Structure& S = h->S;
    const int64_t N = S.n_nodes, T = S.n_tris;
    const int m = h->m;
    const int32_t C = h->n_clusters;
    const bool fp64 = h->prec == H2DLP_FP64;
    const size_t e = h->elem;
    int64_t kept = 0, scratch = 0;
    std::vector<int32_t> perm32(S.perm.begin(), S.perm.end());
    std::vector<int32_t> iperm32(S.iperm.begin(), S.iperm.end());
    h->d_perm = h->upload(perm32, &kept, stream);
    h->d_iperm = h->upload(iperm32, &kept, stream);
    h->d_child0 = h->upload(h->child0, &kept, stream);
    h->d_child1 = h->upload(h->child1, &kept, stream);
    h->d_parent = h->upload(h->parent, &kept, stream);
    h->d_front = h->upload(h->down_front, &kept, stream);
    h->d_diag = h->alloc<double>(sizeof(double) * N, &kept);
    const bool rec = h->rec;
    // recompression: the interpolation bases are built in FP64 for it alone;
    // transfers, couplings and the new bases follow the ranks it finds
    if (!rec) {
        h->d_e = h->alloc<void>(e * size_t(C) * 3 * m * m, &kept);
        h->d_pool_wt = h->alloc<void>(e * size_t(h->off_wt), &kept);
        h->d_pool_s = h->alloc<void>(h->elem_s * size_t(h->off_s), &kept);
        h->d_items_fwd = h->upload(h->items_fwd, &kept, stream);
        h->d_blks_fwd = h->upload(h->blks_fwd, &kept, stream);
        h->d_items_cpl = h->upload(h->items_cpl, &kept, stream);
        h->d_blks_cpl = h->upload(h->blks_cpl, &kept, stream);
        h->d_items_v = h->upload(h->items_v, &kept, stream);
    }
    h->d_pool_leaf = h->alloc<void>(e * size_t(h->off_l), &kept);
    if (!h->cgeo.empty()) h->d_cgeo = h->upload(h->cgeo, &kept, stream);
    if (h->regen_v) {
        std::vector<double> pxyz(3 * size_t(N));
        for (int64_t p = 0; p < N; ++p)
            for (int a = 0; a < 3; ++a) pxyz[3 * size_t(p) + a] = S.xyz[3 * size_t(S.perm[p]) + a];
        h->d_vgen = h->upload(h->vgen, &kept, stream);
        h->d_vxyz = h->upload(pxyz, &kept, stream);
    }
    h->d_items_leaf = h->upload(h->items_leaf, &kept, stream);
    h->d_blks_leaf = h->upload(h->blks_leaf, &kept, stream);
    h->d_items_near = h->upload(h->items_near, &kept, stream);
    make_streams(h);
    if (!fp64) {
        h->d_ns_off = h->upload(S.ring_off, &kept, stream);
        h->d_ns_pos = h->upload(S.ring_pos, &kept, stream);
        const size_t nb = sizeof(double) * std::max<size_t>(1, S.ring_pos.size());
        h->d_ns_val = h->alloc<double>(nb, &kept);
        check(hipMemsetAsync(h->d_ns_val, 0, nb, stream), "clear near-singular values");
    }
    std::vector<double> quad = triangle_rule(3 * (m - 1));
    std::vector<void*> temp;
    auto tmp = [&](auto* p) { temp.push_back(static_cast<void*>(p)); return p; };
    double* d_xyz = tmp(h->upload(S.xyz, &scratch, stream));
    int32_t* d_tri = tmp(h->upload(S.tri, &scratch, stream));
    int64_t* d_inc_off = tmp(h->upload(S.inc_off, &scratch, stream));
    int32_t* d_inc_tri = tmp(h->upload(S.inc_tri, &scratch, stream));
    int32_t* d_inc_loc = tmp(h->upload(S.inc_loc, &scratch, stream));
    double* d_tgeo = tmp(h->alloc<double>(sizeof(double) * 4 * T, &scratch));
    double* d_boxes = tmp(h->upload(h->boxes, &scratch, stream));
    double* d_quad = tmp(h->upload(quad, &scratch, stream));
    LeafDesc* d_leaves = tmp(h->upload(h->leaves, &scratch, stream));
    LeafDesc* d_vleaves = tmp(h->upload(h->vleaves, &scratch, stream));
    FarDesc* d_far = tmp(h->upload(h->fars, &scratch, stream));
    NearDesc* d_near = tmp(h->upload(h->nears, &scratch, stream));

    DevMesh dm{d_xyz, d_tri, d_inc_off, d_inc_tri, d_inc_loc, d_tgeo, h->d_perm};
    int max_leaf = 1;
    for (const LeafDesc& L : h->leaves) max_leaf = std::max(max_leaf, int(L.n));
    check(launch_tri_geometry(d_xyz, d_tri, T, d_tgeo, stream), "triangle geometry");
    check(launch_diagonal(dm, N, h->d_diag, stream), "diagonal");
    if (rec) {
        double* wt64 = tmp(h->alloc<double>(sizeof(double) * size_t(h->off_wt), &scratch));
        double* v64 = tmp(h->alloc<double>(sizeof(double) * size_t(h->off_v), &scratch));
        check(launch_build_wt(dm, d_boxes, m, d_quad, int(quad.size() / 3), d_leaves, int64_t(h->leaves.size()),
                              max_leaf, P_FP64, wt64, stream), "column basis");
        check(launch_build_v(dm, d_boxes, m, d_vleaves, int64_t(h->vleaves.size()), P_FP64, v64, stream),
              "row basis");
        recompress_impl(h, d_boxes, wt64, v64, &kept, stream);
    } else {
        check(launch_build_wt(dm, d_boxes, m, d_quad, int(quad.size() / 3), d_leaves, int64_t(h->leaves.size()),
                              max_leaf, h->prec, h->d_pool_wt, stream), "column basis");
        if (!h->regen_v)
            check(launch_build_v(dm, d_boxes, m, d_vleaves, int64_t(h->vleaves.size()), h->prec, h->d_pool_leaf,
                                 stream),
                  "row basis");
        check(launch_build_transfer(d_boxes, h->d_parent, C, m, h->prec, h->d_e, stream), "transfer");
    }
    if (h->d_cgeo == nullptr && !rec)
        check(launch_build_coupling(d_boxes, m, h->kp, d_far, int64_t(h->fars.size()), h->prec, h->d_pool_s, stream),
              "coupling");
    check(launch_build_near(dm, d_near, int64_t(h->nears.size()), h->prec, h->d_pool_leaf,
                            fp64 ? nullptr : h->d_ns_off, fp64 ? nullptr : h->d_ns_pos, fp64 ? nullptr : h->d_ns_val,
                            stream),
          "near field");
    check(hipStreamSynchronize(stream), "build synchronize");
    for (void* p : temp) h->release(p);
    h->d_ws = h->alloc<void>(h->ws_bytes, &kept);
    if (rec) h->st.bytes_resident = kept;
    finish_materialize(h);
    return H2DLP_OK;
}

h2dlp_ctx* as_ctx(h2dlp_handle h) { return reinterpret_cast<h2dlp_ctx*>(h); }

// *dev: a HIP ordinal, or -1 for the current device; it must be a gfx950
int pick_device(int* dev) {
    if (*dev < 0 && hipGetDevice(dev) != hipSuccess) return fail(H2DLP_ENOTSUP, "no HIP device");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || *dev >= ndev) return fail(H2DLP_ENOTSUP, "no such HIP device");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, *dev) != hipSuccess) return fail(H2DLP_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(H2DLP_ENOTSUP, std::string("device is ") + prop.gcnArchName + ", library built for gfx950");
    return H2DLP_OK;
}

// ---------------------------------------------------------------- persistence
// An operator file (host byte order): magic, format, the library's count of
// device buffers and size of h2dlp_stats; the build options; the mesh; the
// host state that a recompressed build derives from its ranks; the stats;
// then every buffer of fields() in order as (scratch flag, bytes, contents),
// a scratch buffer by its size only.  Loading plans the mesh again (the host
// structure is deterministic) and takes the device buffers from the file.
constexpr char kFileMagic[8] = {'H', '2', 'D', 'L', 'P', 'O', 'P', 'S'};
constexpr uint32_t kFileFormat = 2;
constexpr size_t kStage = size_t(64) << 20;     // bytes per copy through pinned host memory

struct FileOut {
    FILE* f = nullptr;
    bool ok = true;
    ~FileOut() { if (f) std::fclose(f); }
    void raw(const void* p, size_t n) { if (ok && n && std::fwrite(p, 1, n, f) != n) ok = false; }
    template <typename T> void pod(const T& v) { raw(&v, sizeof v); }
    template <typename T> void vec(const std::vector<T>& v) {
        pod(uint64_t(v.size()));
        raw(v.data(), v.size() * sizeof(T));
    }
};

struct FileIn {
    FILE* f = nullptr;
    bool ok = true;
    uint64_t left = 0;                          // bytes of the file not read yet
    ~FileIn() { if (f) std::fclose(f); }
    void raw(void* p, size_t n) {
        if (!ok || n == 0) return;
        if (n > left || std::fread(p, 1, n, f) != n) { ok = false; return; }
        left -= n;
    }
    template <typename T> T pod() { T v{}; raw(&v, sizeof v); return v; }
    template <typename T> void vec(std::vector<T>& v) {
        const uint64_t n = pod<uint64_t>();
        if (!ok || n > left / sizeof(T)) { ok = false; return; }
        v.resize(size_t(n));
        raw(v.data(), size_t(n) * sizeof(T));
    }
};

struct PinnedStage {
    void* p = nullptr;
    ~PinnedStage() { if (p) (void)hipHostFree(p); }
};

// state a recompressed build derives from its ranks (plan values otherwise)
template <bool READ, typename IO>
void derived_state(IO& io, h2dlp_ctx* h) {
    for (std::vector<int32_t>* v : {&h->rank_row, &h->rank_col, &h->up_off, &h->up_end, &h->down_off}) io.vec(*v);
    for (int32_t* x : {&h->up_cut, &h->n_items_cpl_b, &h->rt_fwd, &h->rt_up, &h->rt_cpl, &h->rt_down,
                       &h->n_items_fwd, &h->n_items_cpl, &h->n_items_v}) {
        if constexpr (READ) *x = io.template pod<int32_t>();
        else io.pod(*x);
    }
}

// The kernels dereference u1, u2 and the workspace.  Refuse a pointer that is
// not device memory of the handle's GPU, or whose allocation ends before
// `bytes` from it, so that a wrong argument is an error and not a fault.
bool device_range_ok(const void* p, size_t bytes, int dev, const char* name, std::string* why) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        *why = std::string(name) + " is not HIP device memory";
        return false;
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged) {
        *why = std::string(name) + " is host memory, not device memory";
        return false;
    }
    if (a.device != dev) {
        *why = std::string(name) + " is on device " + std::to_string(a.device) + ", the operator on device " +
               std::to_string(dev);
        return false;
    }
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
        (void)hipGetLastError();       // no range for this kind of allocation: nothing more to check
        return true;
    }
    if (static_cast<const char*>(p) + bytes > static_cast<const char*>(base) + size) {
        *why = std::string(name) + ": its allocation ends before the " + std::to_string(bytes) + " bytes the call needs";
        return false;
    }
    return true;
}

void rec_begin(h2dlp_ctx* h, hipStream_t s, int kind, hipEvent_t* a) {
    if (!(h->prof >> kind & 1)) return;
    check(hipEventCreate(a), "event");
    check(hipEventRecord(*a, s), "event record");
}
void rec_end(h2dlp_ctx* h, hipStream_t s, int kind, hipEvent_t a) {
    if (!(h->prof >> kind & 1)) return;
    hipEvent_t b;
    check(hipEventCreate(&b), "event");
    check(hipEventRecord(b, s), "event record");
    h->recs.push_back({kind, a, b});
}

int apply_impl(h2dlp_ctx* h, const void* u1, void* u2, int nrhs, int io, hipStream_t s, void* ws) {
    // every buffer the kernels read must exist (an offloaded operator has none);
    // buffers that were empty at the build (no far blocks, FP64 near-singular
    // arrays) stay NULL
    {
        const auto fs = h->fields();
        for (size_t q = 0; q < fs.size(); ++q)
            if (*fs[q].first == nullptr && !h->empty_field[q])
                return fail(H2DLP_EINVAL, "operator buffers are not on the device");
    }
    if (ws == nullptr) return fail(H2DLP_EINVAL, "no workspace");
    if (h->ready_pending) {        // copies of an asynchronous reload may still be in flight
        const hipError_t q = hipEventQuery(h->ready);
        if (q == hipSuccess) {
            h->ready_pending = false;
        } else {
            if (q == hipErrorNotReady) (void)hipGetLastError();   // not an error: do not leave it behind
            check(hipStreamWaitEvent(s, h->ready, 0), "waiting for the reload");
        }
    }
    const int64_t N = h->S.n_nodes;
    const int m = h->m, k = h->k, prec = h->prec;
    char* base = static_cast<char*>(ws);
    void* x = base;
    double* x64 = h->ws_x64 ? reinterpret_cast<double*>(base + h->ws_x) : static_cast<double*>(x);
    double* y64 = reinterpret_cast<double*>(base + h->ws_x + h->ws_x64);
    void* xh = base + h->ws_x + h->ws_x64 + h->ws_y64;
    void* yh = static_cast<char*>(xh) + h->ws_xh;
    const size_t io_elem = io == H2DLP_IO_F32 ? 4 : 8;
    for (int c0 = 0; c0 < nrhs; c0 += RHS_TILE) {
        const int nr = std::min(RHS_TILE, nrhs - c0);
        const void* u1p = static_cast<const char*>(u1) + io_elem * size_t(c0) * N;
        void* u2p = static_cast<char*>(u2) + io_elem * size_t(c0) * N;
        hipEvent_t ev = nullptr;
        rec_begin(h, s, 0, &ev);
        check(launch_permute(u1p, io, N, nr, h->d_iperm, x, h->ws_x64 ? x64 : nullptr, prec, s), "permute");
        rec_end(h, s, 0, ev);

        // on the side stream from here on: y64 = D x64 + the FP64 near-singular
        // part, then y64 += the near-field blocks (they read only x and x64),
        // beside the far-field chain on the caller's stream.  With stored
        // coupling the near field starts at once (both HBM-bound; it fills the
        // latency-bound upward pass); with generated coupling (MFMA-bound) it
        // waits for the upward pass, which it would otherwise slow more than
        // it gains.
        const bool near_early = h->d_cgeo == nullptr;
        const int32_t near_head = near_early ? h->n_near_head : h->n_items_leaf;
        ProductArgs nearp{h->d_items_near, near_head, h->rt_leaf, h->d_blks_leaf, h->d_pool_leaf, x, nullptr, nullptr};
        check(hipEventRecord(h->fork_ev, s), "event record");
        check(hipStreamWaitEvent(h->side, h->fork_ev, 0), "fork");
        rec_begin(h, h->side, 6, &ev);
        {
            LeafEpilogue epi{h->d_diag, x64, y64, h->d_ns_off, h->d_ns_pos, h->d_ns_val};
            check(launch_diag_nearsing(epi, N, h->side), "diagonal");
            if (near_early) check(launch_product_near(nearp, y64, prec, h->side), "near field");
        }
        rec_end(h, h->side, 6, ev);

        ProductArgs fwd{h->d_items_fwd, h->n_items_fwd, h->rec ? h->rt_fwd : (k + 15) / 16, h->d_blks_fwd,
                        h->d_pool_wt, x, nullptr, xh};
        rec_begin(h, s, 1, &ev);
        check(launch_product_store(fwd, prec, true, s), "leaf forward");
        rec_end(h, s, 1, ev);

        // levels above up_cut (recompressed, split coupling) go to side2, beside
        // the first coupling launch
        const int cut = h->n_items_cpl_b > 0 ? h->up_cut : 0;
        for (int l = h->S.depth - 1; l >= 0; --l) {
            hipStream_t su = s;
            if (l == cut - 1) {
                check(hipEventRecord(h->cut_ev, s), "event record");
                check(hipStreamWaitEvent(h->side2, h->cut_ev, 0), "fork");
            }
            if (l < cut) su = h->side2;
            rec_begin(h, su, 2, &ev);
            if (h->rec) {      // x^_t = sum_c F'_c^T x^_c, a grouped product per level
                ProductArgs up{h->d_items_up + h->up_off[l], h->up_end[l] - h->up_off[l], h->rt_up, h->d_blks_up,
                               h->d_pool_up, xh, nullptr, xh};
                check(launch_product_store(up, prec, true, su), "upward");
            } else {
                check(launch_upward(h->level_off[l], h->level_off[l + 1], h->d_child0, h->d_child1, h->d_e, xh, m,
                                    prec, su),
                      "upward");
            }
            rec_end(h, su, 2, ev);
        }
        if (cut > 0) check(hipEventRecord(h->upper_ev, h->side2), "event record");

        if (!near_early) {
            check(hipEventRecord(h->mid_ev, s), "event record");
            check(hipStreamWaitEvent(h->side, h->mid_ev, 0), "fork");
            rec_begin(h, h->side, 6, &ev);
            check(launch_product_near(nearp, y64, prec, h->side), "near field");
            rec_end(h, h->side, 6, ev);
        }
        // the near-field tail, on the side stream once the first coupling launch is enqueued
        auto near_tail = [&]() {
            if (!near_early || h->n_near_head >= h->n_items_leaf) return;
            check(hipEventRecord(h->mid_ev, s), "event record");
            check(hipStreamWaitEvent(h->side, h->mid_ev, 0), "fork");
            ProductArgs tail{h->d_items_near + h->n_near_head, h->n_items_leaf - h->n_near_head, h->rt_leaf,
                             h->d_blks_leaf, h->d_pool_leaf, x, nullptr, nullptr};
            hipEvent_t ev6 = nullptr;
            rec_begin(h, h->side, 6, &ev6);
            check(launch_product_near(tail, y64, prec, h->side), "near field");
            rec_end(h, h->side, 6, ev6);
        };

        rec_begin(h, s, 3, &ev);
        if (h->rec) {
            ProductArgs cpl{h->d_items_cpl, h->n_items_cpl, h->rt_cpl, h->d_blks_cpl, h->d_pool_s, xh, nullptr, yh};
            check(launch_product_store(cpl, prec, false, s), "coupling");
            near_tail();
            if (cut > 0) {
                check(hipStreamWaitEvent(s, h->upper_ev, 0), "join");
                ProductArgs cpl_b{h->d_items_cpl_b, h->n_items_cpl_b, h->rt_cpl, h->d_blks_cpl, h->d_pool_s, xh,
                                  nullptr, yh};
                check(launch_product_add(cpl_b, prec, false, s), "coupling");
            }
        } else if (h->d_cgeo) {
            ProductArgs cpl{h->d_items_cpl, h->n_items_cpl, (k + 15) / 16, h->d_blks_cpl, h->d_cgeo, xh, nullptr, yh};
            check(launch_coupling_generated(cpl, m, prec, prec == P_FP32 && h->n_items_leaf > 0 ? h->cpl_lds : 0, s),
                  "coupling");
        } else {
            ProductArgs cpl{h->d_items_cpl, h->n_items_cpl, (k + 15) / 16, h->d_blks_cpl, h->d_pool_s, xh, nullptr, yh};
            check(launch_coupling(cpl, k, prec, s), "coupling");
            near_tail();
        }
        rec_end(h, s, 3, ev);
        check(hipEventRecord(h->join_ev, h->side), "event record");

        if (h->rec) {          // y^_c += F_c y^_parent, a grouped product per level
            for (int l = 1; l <= h->S.depth; ++l) {
                rec_begin(h, s, 4, &ev);
                ProductArgs dn{h->d_items_down + h->down_off[l], h->down_off[l + 1] - h->down_off[l], h->rt_down,
                               h->d_blks_down, h->d_pool_down, yh, nullptr, yh};
                check(launch_product_add(dn, prec, true, s), "downward");
                rec_end(h, s, 4, ev);
            }
        } else {
            rec_begin(h, s, 4, &ev);
            check(launch_downward_paths(int32_t(h->down_front.size()), h->d_front, h->d_parent, h->d_e, yh, m, prec,
                                        s),
                  "downward");
            rec_end(h, s, 4, ev);
            for (int l = h->down_l0 + 1; l <= h->S.depth; ++l) {
                rec_begin(h, s, 4, &ev);
                check(launch_downward(h->level_off[l], h->level_off[l + 1], h->d_parent, h->d_e, yh, m, prec, s),
                      "downward");
                rec_end(h, s, 4, ev);
            }
        }

        // join, then y64 += V_t yhat_t and back to the caller's node order
        check(hipStreamWaitEvent(s, h->join_ev, 0), "join");
        ProductArgs leafv = h->rec ? ProductArgs{h->d_items_v, h->n_items_v, h->rt_leaf, h->d_blks_v,
                                                 h->d_pool_q, x, yh, nullptr}
                                   : ProductArgs{h->d_items_v, h->n_items_leaf, h->rt_leaf, h->d_blks_leaf,
                                                 h->d_pool_leaf, x, yh, nullptr};
        rec_begin(h, s, 5, &ev);
        if (h->regen_v)
            check(launch_leaf_regen(h->d_vgen, h->n_leaves, h->d_vxyz, m, yh, y64, prec, s), "leaf output");
        else
            check(launch_product_add64(leafv, y64, prec, s), "leaf output");
        check(launch_unpermute(y64, io, N, nr, h->d_iperm, u2p, s), "unpermute");
        rec_end(h, s, 5, ev);
    }
    return H2DLP_OK;
}

}  // namespace

extern "C" {

void h2dlp_default_options(h2dlp_options* o) {
    if (!o) return;
    o->order = 4;
    o->leaf = 32;
    o->eta = 2.0;
    o->precision = H2DLP_FP64;
    o->alpha = 0.1;
    o->device = -1;
    o->stream = nullptr;
    o->coupling = H2DLP_COUPLING_STORED;
    o->dense_far_max = 0;
    o->recompress_eps = 0.0;
    o->row_basis = H2DLP_ROW_BASIS_STORED;
}

static int check_args(const h2dlp_mesh* mesh, const h2dlp_options* o, h2dlp_handle* out) {
    if (!out) return fail(H2DLP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mesh || !o) return fail(H2DLP_EINVAL, "mesh or options is NULL");
    if (!mesh->xyz || !mesh->tri) return fail(H2DLP_EINVAL, "mesh arrays are NULL");
    if (mesh->n_nodes < 4 || mesh->n_tris < 4) return fail(H2DLP_EINVAL, "mesh needs at least 4 nodes and 4 triangles");
    if (mesh->n_nodes > (int64_t(1) << 30) || mesh->n_tris > (int64_t(1) << 30))
        return fail(H2DLP_ENOTSUP, "mesh larger than 2^30 nodes or triangles");
    if (o->order < 1 || o->order > 8) return fail(H2DLP_EINVAL, "order must be in [1, 8]");
    if (o->leaf < 1 || o->leaf > 64) return fail(H2DLP_EINVAL, "leaf must be in [1, 64]");
    if (!(o->eta > 0.0) || !std::isfinite(o->eta)) return fail(H2DLP_EINVAL, "eta must be positive");
    if (!(o->alpha >= 0.0 && o->alpha <= 1.0)) return fail(H2DLP_EINVAL, "alpha must be in [0, 1]");
    if (o->precision < H2DLP_FP64 || o->precision > H2DLP_BF16X6)
        return fail(H2DLP_EINVAL, "unknown precision");
    if ((o->precision == H2DLP_BF16X3 || o->precision == H2DLP_BF16X6) && o->order > 5)
        return fail(H2DLP_ENOTSUP, "BF16X3 and BF16X6 need order <= 5 (k <= 128)");
    if (o->coupling != H2DLP_COUPLING_STORED && o->coupling != H2DLP_COUPLING_GENERATED)
        return fail(H2DLP_EINVAL, "unknown coupling mode");
    if (o->dense_far_max < 0) return fail(H2DLP_EINVAL, "dense_far_max must be >= 0");
    if (o->coupling == H2DLP_COUPLING_GENERATED &&
        (o->order > 5 || (o->precision != H2DLP_FP64 && o->precision != H2DLP_FP32)))
        return fail(H2DLP_ENOTSUP, "generated coupling needs FP64 or FP32 and order <= 5");
    if (!(o->recompress_eps >= 0.0 && o->recompress_eps < 1.0))
        return fail(H2DLP_EINVAL, "recompress_eps must be in [0, 1)");
    if (o->recompress_eps > 0.0 && (o->order > 5 || o->coupling != H2DLP_COUPLING_STORED ||
                                    (o->precision != H2DLP_FP64 && o->precision != H2DLP_FP32)))
        return fail(H2DLP_ENOTSUP, "recompression needs FP64 or FP32, stored coupling and order <= 5");
    if (o->row_basis != H2DLP_ROW_BASIS_STORED && o->row_basis != H2DLP_ROW_BASIS_GENERATED)
        return fail(H2DLP_EINVAL, "unknown row basis mode");
    if (o->row_basis == H2DLP_ROW_BASIS_GENERATED && o->recompress_eps > 0.0)
        return fail(H2DLP_ENOTSUP, "a generated row basis needs the interpolation bases (recompress_eps 0)");
    return H2DLP_OK;
}

int h2dlp_plan(const h2dlp_mesh* mesh, const h2dlp_options* o, h2dlp_handle* out) {
    int rc = check_args(mesh, o, out);
    if (rc != H2DLP_OK) return rc;
    std::unique_ptr<h2dlp_ctx> h(new (std::nothrow) h2dlp_ctx);
    if (!h) return fail(H2DLP_ENOMEM, "host allocation failed");
    try {
        rc = plan_impl(h.get(), mesh, o);
    } catch (const std::bad_alloc&) {
        rc = fail(H2DLP_ENOMEM, "host allocation failed");
    }
    if (rc != H2DLP_OK) return rc;
    *out = reinterpret_cast<h2dlp_handle>(h.release());
    return H2DLP_OK;
}

int h2dlp_build_ex(const h2dlp_mesh* mesh, const h2dlp_options* o, h2dlp_handle* out) {
    int rc = h2dlp_plan(mesh, o, out);
    if (rc != H2DLP_OK) return rc;
    std::unique_ptr<h2dlp_ctx> h(as_ctx(*out));
    *out = nullptr;
    int dev = o->device;
    rc = pick_device(&dev);
    if (rc != H2DLP_OK) return rc;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(dev) != hipSuccess) return fail(H2DLP_EDEVICE, "hipSetDevice failed");
    h->device = dev;
    try {
        rc = materialize_impl(h.get(), static_cast<hipStream_t>(o->stream));
    } catch (const HipError& e) {
        rc = fail(H2DLP_EDEVICE, e.where + ": " + hipGetErrorString(e.err));
    } catch (const std::bad_alloc&) {
        rc = fail(H2DLP_ENOMEM, "device or host allocation failed");
    }
    if (rc != H2DLP_OK) {
        h.reset();          // frees what was allocated on `dev`
        hipSetDevice(cur);
        return rc;
    }
    hipSetDevice(cur);
    *out = reinterpret_cast<h2dlp_handle>(h.release());
    return H2DLP_OK;
}

h2dlp_handle h2dlp_build(const h2dlp_mesh* mesh, int order, int leaf, double eta) {
    h2dlp_options o;
    h2dlp_default_options(&o);
    o.order = order;
    o.leaf = leaf;
    o.eta = eta;
    h2dlp_handle h = nullptr;
    return h2dlp_build_ex(mesh, &o, &h) == H2DLP_OK ? h : nullptr;
}

}  // extern "C"

namespace h2dlp {

int set_error(int code, const std::string& msg) { return fail(code, msg); }

bool device_memory_ok(const void* p, size_t bytes, int dev, const char* name, std::string* why) {
    return device_range_ok(p, bytes, dev, name, why);
}

int gfx950_device(int* dev) { return pick_device(dev); }

int handle_device(h2dlp_handle hh) {
    const h2dlp_ctx* h = as_ctx(hh);
    return h && h->materialized ? h->device : -1;
}

// h2dlp_apply_ex; `workspace_is_library`: the workspace is the library's own
// device array (its address is not checked against the caller's allocations)
int apply_entry(h2dlp_handle hh, const void* u1, void* u2, int nrhs, int io_dtype, void* stream, void* workspace,
                size_t workspace_bytes, bool workspace_is_library) {
    h2dlp_ctx* h = as_ctx(hh);
    if (!h) return fail(H2DLP_EINVAL, "handle is NULL");
    if (!u1 || !u2) return fail(H2DLP_EINVAL, "u1 or u2 is NULL");
    if (nrhs < 1) return fail(H2DLP_EINVAL, "nrhs must be >= 1");
    if (!h->materialized) return fail(H2DLP_EINVAL, "handle comes from h2dlp_plan: nothing on the device");
    if (h->offloaded) return fail(H2DLP_EINVAL, "operator is offloaded: call h2dlp_reload first");
    if (io_dtype != H2DLP_IO_F64 && io_dtype != H2DLP_IO_F32) return fail(H2DLP_EINVAL, "unknown io dtype");
    const size_t bytes = (io_dtype == H2DLP_IO_F32 ? 4 : 8) * size_t(nrhs) * size_t(h->S.n_nodes);
    const char* a = static_cast<const char*>(u1);
    const char* b = static_cast<const char*>(u2);
    if (a < b + bytes && b < a + bytes) return fail(H2DLP_EINVAL, "u1 and u2 overlap");
    void* ws = workspace;
    if (ws == nullptr) ws = h->d_ws;
    else if (workspace_bytes < h->ws_bytes) return fail(H2DLP_ENOMEM, "workspace smaller than h2dlp_stats.workspace_bytes");
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != h->device && hipSetDevice(h->device) != hipSuccess) return fail(H2DLP_EDEVICE, "hipSetDevice failed");
    std::string why;
    if (!device_range_ok(u1, bytes, h->device, "u1", &why) || !device_range_ok(u2, bytes, h->device, "u2", &why) ||
        (workspace && !workspace_is_library && !device_range_ok(workspace, h->ws_bytes, h->device, "workspace", &why))) {
        if (cur != h->device) hipSetDevice(cur);
        return fail(H2DLP_EINVAL, why);
    }
    int rc;
    try {
        rc = apply_impl(h, u1, u2, nrhs, io_dtype, static_cast<hipStream_t>(stream), ws);
    } catch (const HipError& e) {
        rc = fail(H2DLP_EDEVICE, e.where + ": " + hipGetErrorString(e.err));
    }
    if (cur != h->device) hipSetDevice(cur);
    return rc;
}

}  // namespace h2dlp

extern "C" {

int h2dlp_apply_ex(h2dlp_handle h, const void* u1, void* u2, int nrhs, int io_dtype, void* stream, void* workspace,
                   size_t workspace_bytes) {
    return h2dlp::apply_entry(h, u1, u2, nrhs, io_dtype, stream, workspace, workspace_bytes, false);
}

int h2dlp_apply(h2dlp_handle h, const double* u1, double* u2, int nrhs) {
    return h2dlp_apply_ex(h, u1, u2, nrhs, H2DLP_IO_F64, nullptr, nullptr, 0);
}

int h2dlp_bytes(h2dlp_handle hh, size_t* resident, size_t* workspace) {
    h2dlp_ctx* h = as_ctx(hh);
    if (!h) return fail(H2DLP_EINVAL, "handle is NULL");
    if (resident) *resident = size_t(h->st.bytes_resident);
    if (workspace) *workspace = h->ws_bytes;
    return H2DLP_OK;
}

int h2dlp_info(h2dlp_handle hh, h2dlp_stats* st) {
    h2dlp_ctx* h = as_ctx(hh);
    if (!h || !st) return fail(H2DLP_EINVAL, "handle or stats is NULL");
    *st = h->st;
    return H2DLP_OK;
}

int h2dlp_export_structure(h2dlp_handle hh, int64_t* perm, int64_t* clusters, double* boxes, int64_t* far,
                           int64_t* near) {
    h2dlp_ctx* h = as_ctx(hh);
    if (!h) return fail(H2DLP_EINVAL, "handle is NULL");
    const Structure& S = h->S;
    if (perm)
        for (int64_t q = 0; q < S.n_nodes; ++q) perm[q] = S.perm[q];
    for (size_t c = 0; c < S.cl.size(); ++c) {
        const Cluster& X = S.cl[c];
        if (clusters) {
            int64_t* r = clusters + 6 * c;
            r[0] = X.begin; r[1] = X.end; r[2] = X.level; r[3] = X.parent; r[4] = X.child0; r[5] = X.child1;
        }
        if (boxes)
            for (int a = 0; a < 3; ++a) { boxes[6 * c + a] = X.lo[a]; boxes[6 * c + 3 + a] = X.hi[a]; }
    }
    if (far)
        for (size_t b = 0, q = 0; b < S.far.size(); ++b)
            if (h->far_dense.empty() || !h->far_dense[b]) {
                far[2 * q] = S.far[b].first;
                far[2 * q + 1] = S.far[b].second;
                ++q;
            }
    if (near)
        for (size_t b = 0; b < S.near.size(); ++b) { near[2 * b] = S.near[b].first; near[2 * b + 1] = S.near[b].second; }
    return H2DLP_OK;
}

int h2dlp_export_diagonal(h2dlp_handle hh, double* diag) {
    h2dlp_ctx* h = as_ctx(hh);
    if (!h || !diag) return fail(H2DLP_EINVAL, "handle or output is NULL");
    if (!h->materialized) return fail(H2DLP_EINVAL, "handle comes from h2dlp_plan: nothing on the device");
    if (h->offloaded) return fail(H2DLP_EINVAL, "operator is offloaded: call h2dlp_reload first");
    std::vector<double> d(h->S.n_nodes);
    if (hipSetDevice(h->device) != hipSuccess ||
        (h->ready_pending && hipEventSynchronize(h->ready) != hipSuccess) ||
        hipMemcpy(d.data(), h->d_diag, sizeof(double) * d.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(H2DLP_EDEVICE, "copying the diagonal failed");
    for (int64_t p = 0; p < h->S.n_nodes; ++p) diag[h->S.perm[p]] = d[p];
    return H2DLP_OK;
}

int h2dlp_offload(h2dlp_handle hh) {
    h2dlp_ctx* h = as_ctx(hh);
    if (!h) return fail(H2DLP_EINVAL, "handle is NULL");
    if (!h->materialized) return fail(H2DLP_EINVAL, "handle comes from h2dlp_plan: nothing on the device");
    if (h->offloaded) return H2DLP_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (hipSetDevice(h->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return fail(H2DLP_EDEVICE, "synchronising the device before offload failed");
    h->ready_pending = false;
    // the operator never changes after the build: the first offload keeps a
    // pinned host copy for good, later offloads only free the device memory
    if (h->parked.empty()) {
        std::vector<h2dlp_ctx::Parked> parked;
        int rc = H2DLP_OK;
        for (auto& f : h->fields()) {
            void* p = *f.first;
            if (!p) continue;
            const size_t bytes = h->bytes_of(p);
            void* host = nullptr;
            if (!f.second) {
                if (hipHostMalloc(&host, bytes, hipHostMallocDefault) != hipSuccess) {
                    rc = fail(H2DLP_ENOMEM, "pinned host allocation failed");
                    break;
                }
                if (hipMemcpy(host, p, bytes, hipMemcpyDeviceToHost) != hipSuccess) {
                    (void)hipHostFree(host);
                    rc = fail(H2DLP_EDEVICE, "copy to host failed");
                    break;
                }
            }
            parked.push_back({f.first, host, bytes, f.second});
        }
        if (rc != H2DLP_OK) {
            for (auto& p : parked) if (p.host) (void)hipHostFree(p.host);
            (void)hipSetDevice(cur);
            return rc;
        }
        h->parked = std::move(parked);
    }
    for (auto& p : h->parked) {
        h->release(*p.field);
        *p.field = nullptr;
    }
    h->offloaded = true;
    (void)hipSetDevice(cur);
    return H2DLP_OK;
}

int h2dlp_reload_ex(h2dlp_handle hh, void* stream) {
    h2dlp_ctx* h = as_ctx(hh);
    if (!h) return fail(H2DLP_EINVAL, "handle is NULL");
    if (!h->offloaded) return H2DLP_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (hipSetDevice(h->device) != hipSuccess) return fail(H2DLP_EDEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!h->ready && hipEventCreateWithFlags(&h->ready, hipEventDisableTiming) != hipSuccess) {
        h->ready = nullptr;
        (void)hipSetDevice(cur);
        return fail(H2DLP_EDEVICE, "creating the reload event failed");
    }
    int rc = H2DLP_OK;
    size_t done = 0;
    try {
        for (; done < h->parked.size(); ++done) {
            auto& p = h->parked[done];
            void* d = h->alloc<void>(p.bytes, nullptr);
            *p.field = d;
            if (!p.scratch && hipMemcpyAsync(d, p.host, p.bytes, hipMemcpyHostToDevice, s) != hipSuccess) {
                ++done;
                rc = fail(H2DLP_EDEVICE, "copy to device failed");
                break;
            }
        }
    } catch (const std::bad_alloc&) {
        rc = fail(H2DLP_ENOMEM, "device allocation failed during reload");
    }
    if (rc == H2DLP_OK && hipEventRecord(h->ready, s) != hipSuccess)
        rc = fail(H2DLP_EDEVICE, "recording the reload event failed");
    if (rc != H2DLP_OK) {           // back to the offloaded state once enqueued copies are done
        (void)hipStreamSynchronize(s);
        for (size_t q = 0; q < done && q < h->parked.size(); ++q) {
            h->release(*h->parked[q].field);
            *h->parked[q].field = nullptr;
        }
        (void)hipSetDevice(cur);
        return rc;
    }
    h->ready_pending = true;
    h->offloaded = false;
    (void)hipSetDevice(cur);
    return H2DLP_OK;
}

int h2dlp_reload(h2dlp_handle hh) {
    h2dlp_ctx* h = as_ctx(hh);
    if (!h) return fail(H2DLP_EINVAL, "handle is NULL");
    if (!h->offloaded) return H2DLP_OK;
    int rc = h2dlp_reload_ex(hh, nullptr);
    if (rc != H2DLP_OK) return rc;
    if (hipEventSynchronize(h->ready) != hipSuccess) return fail(H2DLP_EDEVICE, "waiting for the reload failed");
    h->ready_pending = false;
    return H2DLP_OK;
}

int h2dlp_save(h2dlp_handle hh, const char* path) {
    h2dlp_ctx* h = as_ctx(hh);
    if (!h) return fail(H2DLP_EINVAL, "handle is NULL");
    if (!path) return fail(H2DLP_EINVAL, "path is NULL");
    if (!h->materialized) return fail(H2DLP_EINVAL, "handle comes from h2dlp_plan: nothing to save");
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (hipSetDevice(h->device) != hipSuccess) return fail(H2DLP_EDEVICE, "hipSetDevice failed");
    auto done = [&](int rc) { (void)hipSetDevice(cur); return rc; };
    if (h->ready_pending && hipEventSynchronize(h->ready) != hipSuccess)
        return done(fail(H2DLP_EDEVICE, "waiting for the reload failed"));
    FileOut o;
    o.f = std::fopen(path, "wb");
    if (!o.f) return done(fail(H2DLP_EINVAL, std::string("cannot open ") + path + " for writing"));
    auto fs = h->fields();
    o.raw(kFileMagic, sizeof kFileMagic);
    o.pod(kFileFormat);
    o.pod(uint32_t(fs.size()));
    o.pod(uint32_t(sizeof(h2dlp_stats)));
    const h2dlp_options& op = h->opt;
    o.pod(int32_t(op.order)); o.pod(int32_t(op.leaf)); o.pod(op.eta); o.pod(int32_t(op.precision));
    o.pod(op.alpha); o.pod(int32_t(op.coupling)); o.pod(op.dense_far_max); o.pod(op.recompress_eps);
    o.pod(int32_t(op.row_basis));
    o.vec(h->S.xyz);
    o.vec(h->S.tri);
    derived_state<false>(o, h);
    o.pod(uint64_t(h->ws_xh));
    o.pod(uint64_t(h->ws_bytes));
    o.pod(h->st);
    PinnedStage stage;
    if (!h->offloaded && hipHostMalloc(&stage.p, kStage, hipHostMallocDefault) != hipSuccess) {
        stage.p = nullptr;
        return done(fail(H2DLP_ENOMEM, "pinned host allocation failed"));
    }
    for (auto& f : fs) {
        const void* dev = *f.first;
        const void* host = nullptr;
        size_t bytes = 0;
        if (h->offloaded) {        // the parked host copy is the operator
            for (const auto& pk : h->parked)
                if (pk.field == f.first) { bytes = pk.bytes; host = pk.host; }
        } else if (dev) {
            bytes = h->bytes_of(const_cast<void*>(dev));
        }
        o.pod(uint8_t(f.second));
        o.pod(uint64_t(bytes));
        if (f.second) continue;
        for (size_t off = 0; off < bytes && o.ok; off += kStage) {
            const size_t n = std::min(kStage, bytes - off);
            if (host) {
                o.raw(static_cast<const char*>(host) + off, n);
            } else {
                if (hipMemcpy(stage.p, static_cast<const char*>(dev) + off, n, hipMemcpyDeviceToHost) != hipSuccess)
                    return done(fail(H2DLP_EDEVICE, "copy to host failed"));
                o.raw(stage.p, n);
            }
        }
    }
    if (!o.ok || std::fflush(o.f) != 0) return done(fail(H2DLP_EINVAL, std::string("writing ") + path + " failed"));
    return done(H2DLP_OK);
}

int h2dlp_load(const char* path, int device, h2dlp_handle* out) {
    if (!out) return fail(H2DLP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!path) return fail(H2DLP_EINVAL, "path is NULL");
    FileIn in;
    in.f = std::fopen(path, "rb");
    if (!in.f) return fail(H2DLP_EINVAL, std::string("cannot open ") + path);
    if (std::fseek(in.f, 0, SEEK_END) != 0) return fail(H2DLP_EINVAL, "cannot size the file");
    const long size = std::ftell(in.f);
    if (size < 0 || std::fseek(in.f, 0, SEEK_SET) != 0) return fail(H2DLP_EINVAL, "cannot size the file");
    in.left = uint64_t(size);
    char magic[sizeof kFileMagic] = {};
    in.raw(magic, sizeof magic);
    if (!in.ok || std::memcmp(magic, kFileMagic, sizeof magic) != 0)
        return fail(H2DLP_EINVAL, std::string(path) + " is not an h2dlp operator file");
    const uint32_t format = in.pod<uint32_t>(), n_fields = in.pod<uint32_t>(), stats_size = in.pod<uint32_t>();
    if (format != kFileFormat || stats_size != sizeof(h2dlp_stats))
        return fail(H2DLP_ENOTSUP, "operator file written by another version of the library");
    h2dlp_options o;
    h2dlp_default_options(&o);
    o.order = in.pod<int32_t>(); o.leaf = in.pod<int32_t>(); o.eta = in.pod<double>();
    o.precision = in.pod<int32_t>(); o.alpha = in.pod<double>(); o.coupling = in.pod<int32_t>();
    o.dense_far_max = in.pod<int64_t>(); o.recompress_eps = in.pod<double>();
    o.row_basis = in.pod<int32_t>();
    o.device = device;
    std::vector<double> xyz;
    std::vector<int32_t> tri;
    in.vec(xyz);
    in.vec(tri);
    if (!in.ok || xyz.size() % 3 != 0 || tri.size() % 3 != 0) return fail(H2DLP_EINVAL, "truncated operator file");
    const h2dlp_mesh mesh{int64_t(xyz.size() / 3), xyz.data(), int64_t(tri.size() / 3), tri.data()};
    h2dlp_handle planned = nullptr;
    int rc = h2dlp_plan(&mesh, &o, &planned);       // the host structure, exactly as the build had it
    if (rc != H2DLP_OK) return rc;
    std::unique_ptr<h2dlp_ctx> h(as_ctx(planned));
    const size_t ws_xh_plan = h->ws_xh, ws_plan = h->ws_bytes;
    derived_state<true>(in, h.get());
    const size_t ws_xh = size_t(in.pod<uint64_t>()), ws_bytes = size_t(in.pod<uint64_t>());
    const h2dlp_stats st = in.pod<h2dlp_stats>();
    auto fs = h->fields();
    if (!in.ok) return fail(H2DLP_EINVAL, "truncated operator file");
    if (n_fields != fs.size()) return fail(H2DLP_ENOTSUP, "operator file written by another version of the library");
    if (!h->rec && (ws_xh != ws_xh_plan || ws_bytes != ws_plan))
        return fail(H2DLP_EINVAL, "operator file does not match the plan of its own mesh and options");
    int dev = device;
    rc = pick_device(&dev);
    if (rc != H2DLP_OK) return rc;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(dev) != hipSuccess)
        return fail(H2DLP_EDEVICE, "hipSetDevice failed");
    h->device = dev;
    auto done = [&](int r) { (void)hipSetDevice(cur); return r; };
    try {
        h->ws_xh = ws_xh;
        h->ws_bytes = ws_bytes;
        PinnedStage stage;
        if (hipHostMalloc(&stage.p, kStage, hipHostMallocDefault) != hipSuccess) {
            stage.p = nullptr;
            throw std::bad_alloc();
        }
        int64_t kept = 0;
        for (auto& f : fs) {
            const bool scratch = in.pod<uint8_t>() != 0;
            const uint64_t bytes = in.pod<uint64_t>();
            if (!in.ok || scratch != f.second || (!scratch && bytes > in.left))
                return done(fail(H2DLP_EINVAL, "truncated or corrupt operator file"));
            if (scratch || bytes == 0) continue;
            void* d = h->alloc<void>(size_t(bytes), &kept);
            *f.first = d;
            for (size_t off = 0; off < bytes; off += kStage) {
                const size_t n = std::min<size_t>(kStage, size_t(bytes) - off);
                in.raw(stage.p, n);
                if (!in.ok) return done(fail(H2DLP_EINVAL, "truncated operator file"));
                check(hipMemcpy(static_cast<char*>(d) + off, stage.p, n, hipMemcpyHostToDevice), "copy to device");
            }
        }
        h->d_ws = h->alloc<void>(h->ws_bytes, &kept);
        make_streams(h.get());
        h->st = st;                                 // the built operator's figures, ranks included
        finish_materialize(h.get());
    } catch (const HipError& e) {
        return done(fail(H2DLP_EDEVICE, e.where + ": " + hipGetErrorString(e.err)));
    } catch (const std::bad_alloc&) {
        return done(fail(H2DLP_ENOMEM, "device or host allocation failed"));
    }
    *out = reinterpret_cast<h2dlp_handle>(h.release());
    return done(H2DLP_OK);
}

void h2dlp_free(h2dlp_handle hh) { delete as_ctx(hh); }

const char* h2dlp_last_error(void) { return g_last_error.c_str(); }

int h2dlp_profile(h2dlp_handle hh, int enable) {
    h2dlp_ctx* h = as_ctx(hh);
    if (!h) return fail(H2DLP_EINVAL, "handle is NULL");
    h->prof = enable & ((1 << H2DLP_NKINDS) - 1);
    return H2DLP_OK;
}

int h2dlp_profile_read(h2dlp_handle hh, double* ms, int64_t* launches, int n_kinds, int reset) {
    h2dlp_ctx* h = as_ctx(hh);
    if (!h) return fail(H2DLP_EINVAL, "handle is NULL");
    if (n_kinds < 0 || n_kinds > H2DLP_NKINDS) return fail(H2DLP_EINVAL, "n_kinds out of range");
    for (auto& r : h->recs) {
        float t = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
            return fail(H2DLP_EDEVICE, "reading profile events failed");
        h->prof_ms[r.kind] += t;
        h->prof_n[r.kind] += 1;
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    h->recs.clear();
    for (int q = 0; q < n_kinds; ++q) {
        if (ms) ms[q] = h->prof_ms[q];
        if (launches) launches[q] = h->prof_n[q];
    }
    if (reset)
        for (int q = 0; q < H2DLP_NKINDS; ++q) { h->prof_ms[q] = 0; h->prof_n[q] = 0; }
    return H2DLP_OK;
}

}  // extern "C"
