// Internal launch interface between the C ABI (api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.h"

namespace h2dlp {

enum Prec { P_FP64 = 0, P_FP32 = 1, P_BF16X3 = 2, P_BF16X6 = 3 };
// bfloat16 terms per coupling entry: 2 (BF16X3), 3 (BF16X6), 0 otherwise
H2DLP_HD inline int bf16_parts(int prec) { return prec == P_BF16X3 ? 2 : (prec == P_BF16X6 ? 3 : 0); }

// ---------------------------------------------------------------- build (FP64 arithmetic)

struct DevMesh {
    const double* xyz;       // N x 3, node order
    const int32_t* tri;      // T x 3
    const int64_t* inc_off;  // node -> incident triangles (CSR)
    const int32_t* inc_tri;
    const int32_t* inc_loc;
    const double* tgeo;      // T x 4: unit normal, area
    const int32_t* perm;     // cluster position -> node
};

struct LeafDesc {   // one leaf cluster
    int32_t pos;    // first cluster position
    int32_t n;      // number of nodes
    int32_t gid;    // cluster id in level order
    int32_t pad;
    int64_t a_off;  // offset of its block in the pool
};

struct FarDesc {    // one admissible block
    int32_t t, s;   // cluster ids in level order
    int64_t a_off;
};

struct NearDesc {   // one inadmissible leaf block
    int32_t tpos, nt, spos, ns;
    int64_t a_off;
};

hipError_t launch_tri_geometry(const double* xyz, const int32_t* tri, int64_t n_tris, double* tgeo, hipStream_t st);
hipError_t launch_diagonal(DevMesh mesh, int64_t n_nodes, double* diag, hipStream_t st);
hipError_t launch_build_v(DevMesh mesh, const double* boxes, int m, const LeafDesc* leaves, int64_t n_leaves,
                          int prec, void* pool, hipStream_t st);
// max_leaf: the most nodes of any leaf (at most 64)
hipError_t launch_build_wt(DevMesh mesh, const double* boxes, int m, const double* quad, int n_quad,
                           const LeafDesc* leaves, int64_t n_leaves, int max_leaf, int prec, void* pool,
                           hipStream_t st);
hipError_t launch_build_transfer(const double* boxes, const int32_t* parent, int64_t n_clusters, int m, int prec,
                                 void* e, hipStream_t st);
hipError_t launch_build_coupling(const double* boxes, int m, int kp, const FarDesc* far, int64_t n_far, int prec,
                                 void* pool, hipStream_t st);
hipError_t launch_build_near(DevMesh mesh, const NearDesc* near, int64_t n_near, int prec, void* pool,
                             const int64_t* ring_off, const int32_t* ring_pos, double* ns_val, hipStream_t st);

// ---------------------------------------------------------------- apply

struct LeafEpilogue {           // y64 = D x64 (+ near-singular FP64 part), cluster order
    const double* diag;         // by cluster position
    const double* x64;          // FP64 input rows (cluster order, 16 columns)
    double* y64;                // FP64 output rows (cluster order, 16 columns)
    const int64_t* ns_off;      // by cluster position; NULL when there is no FP64 subset
    const int32_t* ns_pos;      // column as a cluster position
    const double* ns_val;
};

struct ProductArgs {
    const ItemDesc* items;
    int32_t n_items;
    int32_t rt;                 // row tiles of the largest item, ceil(m/16)
    const BlkDesc* blks;
    const void* pool;
    const void* x0;
    const void* x1;
    void* y;
};

hipError_t launch_permute(const void* u1, int io, int64_t n_nodes, int nr, const int32_t* iperm, void* x,
                          double* x64, int prec, hipStream_t st);
hipError_t launch_unpermute(const double* y64, int io, int64_t n_nodes, int nr, const int32_t* iperm, void* u2,
                            hipStream_t st);
// prefer_rows: split the rows of one item over the 4 waves (else split its blocks)
hipError_t launch_product_store(const ProductArgs& a, int prec, bool prefer_rows, hipStream_t st);
// y64 = D x64 + the FP64 near-singular part, over n_pos cluster positions (all 16 columns)
hipError_t launch_diag_nearsing(const LeafEpilogue& e, int64_t n_pos, hipStream_t st);
// near field: y64 += sum_b A_b X_b of each leaf item, the waves splitting its blocks
hipError_t launch_product_near(const ProductArgs& a, double* y64, int prec, hipStream_t st);
// Coupling products; for k <= 128 with ceil(k/16) a power of two the blocks are
// stored k x coupling_cols(k) (zero columns beyond k) and a pipelined kernel runs.
hipError_t launch_coupling(const ProductArgs& a, int k, int prec, hipStream_t st);
// y += sum_b A_b X_b of each item, in the operator precision (prefer_rows as
// for launch_product_store; y may be the source array, at rows other than the
// item's)
hipError_t launch_product_add(const ProductArgs& a, int prec, bool prefer_rows, hipStream_t st);
// y64 += sum_b A_b X_b of each item (FP64 accumulation target in cluster order)
hipError_t launch_product_add64(const ProductArgs& a, double* y64, int prec, hipStream_t st);
// Generated coupling (orders 1..5, FP32 or FP64): a.pool holds the per-cluster
// centre and half extent (6 doubles, level-order ids), blks[b].a_off the source cluster.
// lds_floor: LDS bytes each workgroup reserves at least (occupancy shaping
// while the near field shares the device).
hipError_t launch_coupling_generated(const ProductArgs& a, int m, int prec, size_t lds_floor, hipStream_t st);
inline int coupling_cols(int k) {
    const int rt = (k + 15) / 16;
    return (rt <= 8 && (rt & (rt - 1)) == 0) ? 16 * rt : k;
}
// A leaf whose row basis the apply regenerates (interpolation bases only).
struct VLeaf {
    int32_t pos;        // first cluster position
    int32_t n;          // nodes, at most 64
    int32_t yrow;       // its first yhat row (level-order id times k)
    int32_t pad;
    double box[6];      // interpolation box: lo xyz, hi xyz
};
// y64 += V_t yhat_t for every leaf, V_t evaluated from xyz (node coordinates
// in cluster order, N x 3) and the leaf's box; orders 1..8; yh in the operator
// precision (FP64, else FP32)
hipError_t launch_leaf_regen(const VLeaf* leaves, int64_t n_leaves, const double* xyz, int m, const void* yh,
                             double* y64, int prec, hipStream_t st);
hipError_t launch_upward(int32_t c_begin, int32_t c_end, const int32_t* child0, const int32_t* child1, const void* e,
                         void* xh, int m, int prec, hipStream_t st);
hipError_t launch_downward(int32_t c_begin, int32_t c_end, const int32_t* parent, const void* e, void* yh, int m,
                           int prec, hipStream_t st);
// Downward pass over the top of the tree in one launch: for each cluster d of
// front, yhat_d = yhat_d + E_d (yhat_parent + E_parent (... yhat_root)), along
// its path to the root (at most kMaxPath clusters).  Only the front clusters
// are written; the clusters above them are read (their coupling part).
constexpr int kMaxPath = 32;
constexpr int kPathFront = 1024;
hipError_t launch_downward_paths(int32_t n_front, const int32_t* front, const int32_t* parent, const void* e, void* yh,
                                 int m, int prec, hipStream_t st);

}  // namespace h2dlp
