// Algebraic recompression of the interpolation H2 matrix on the GPU (build
// time, FP64): orthonormal nested cluster bases of adaptive rank from
// truncated SVDs weighted by every low-rank block a basis serves, and the
// coupling matrices projected onto them (Section 4: the algebraic conversion
// to an H2 matrix whose ranks follow the accuracy, not the interpolation
// order).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace h2dlp {

// The tree and blocks of an interpolation H2 matrix, in level-order cluster
// ids (gid): the clusters of level l are [level_off[l], level_off[l + 1]).
struct RecompressPlan {
    int m = 0, k = 0;                  // interpolation order, k = m^3 <= 128
    int rows = 0;                      // rows of every per-cluster work matrix: max(2k, largest leaf)
    int32_t n_clusters = 0, depth = 0;
    std::vector<int32_t> level_off, child0, child1, parent;
    std::vector<int32_t> leaf_n;       // by gid: rows of a leaf, 0 for an inner cluster
    std::vector<int32_t> far_t, far_s; // the low-rank admissible blocks (t, s)
    double eps = 0.0;                  // relative truncation tolerance
};

// Device results, FP64 column-major, one slot per gid:
//   u_row / u_col: rows x k (ld rows) left singular vectors of the cluster's
//     weighted basis; a leaf's new basis is its first n_t rows and r_t columns,
//     an inner cluster's new transfers are rows [0, r_c0) (first child) and
//     [k, k + r_c1) (second child) of its first r_t columns;
//   p_row / p_col: k x k (ld k), rows >= rank zero: the interpolation basis in
//     the new one (V_t ~ new basis times P_t).
struct RecompressResult {
    std::vector<int32_t> rank_row, rank_col;
    double* u_row = nullptr;
    double* u_col = nullptr;
    double* p_row = nullptr;
    double* p_col = nullptr;
    size_t bytes = 0;                  // device bytes of the four arrays
    void release();
};

// d_boxes: 6 doubles per gid (lo xyz, hi xyz); d_vleaf / d_wleaf: the leaf row
// and column bases V_t (n_t x k) and W_s (n_s x k), rows x k column-major per
// gid slot (inner clusters' slots unused, rows past n_t zero).  Returns "" or
// an error message.
std::string recompress(const RecompressPlan& plan, const double* d_boxes, const double* d_vleaf,
                       const double* d_wleaf, hipStream_t stream, RecompressResult* out);

// The projected coupling matrices S'_b = P_t S_tb P'_s^T (r_t x r'_s) of the
// low-rank blocks b, stored at a_off[b] in the A-operand layout (layout.h)
// in precision prec (P_FP64 / P_FP32).
std::string recompress_couplings(const RecompressPlan& plan, const double* d_boxes, const RecompressResult& res,
                                 const std::vector<int64_t>& a_off, int prec, void* pool, hipStream_t stream);

// One matrix copied from FP64 column-major device memory into the A-operand
// layout: A(i, j) = src[i + ld j] (or src[j + ld i] when transposed), M x K.
struct StoreDesc {
    const double* src;
    int32_t ld;
    int32_t M, K;
    int32_t transpose;
    int64_t a_off;
};
hipError_t launch_store_layout(const StoreDesc* d_desc, int64_t n, int prec, void* pool, hipStream_t st);

// Leaf bases gathered from their A-operand layout blocks (FP64 pools of the
// build) into rows x k column-major slots by gid: V_t is stored as A = V_t
// (n_t x k), W_s as A = W_s^T (k x n_s).
struct GatherDesc {
    int64_t a_off;
    int32_t gid, n;
};
hipError_t launch_gather_leaf_basis(const GatherDesc* d_desc, int64_t n_leaves, const double* pool, int k, int rows,
                                    bool transposed, double* out, hipStream_t st);

}  // namespace h2dlp
