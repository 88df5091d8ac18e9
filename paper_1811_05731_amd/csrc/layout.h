// Device data layout shared by the build kernels (writers) and the apply
// kernels (readers).  Internal to the library.
//
// Every dense block the apply multiplies -- a leaf's transposed column basis
// W_s^T (k x n_s), a coupling matrix S_ts (k x k), a leaf's row basis V_t
// (n_t x k) and a near-field block K|_{t x s} (n_t x n_s) -- is stored in the
// order in which a wave64 feeds it to the 16x16x4 MFMA as the A operand, with
// no padding: the M x K block is cut into 16 x 4 chunks (row tile rt, k-step
// ks), chunks ordered ks-major, and inside a chunk of rv x kv valid entries the
// entry (row 16 rt + i, col 4 ks + kk) sits at kk * rv + i.  Lane l of the wave
// reads the entry with i = l % 16, kk = l / 16, so every chunk is one
// contiguous run of at most 64 elements.  Only the last row tile and the last
// k-step can be partial.
#pragma once

#include <cstdint>

#ifndef H2DLP_HD
#if defined(__HIPCC__)
#define H2DLP_HD __host__ __device__
#else
#define H2DLP_HD
#endif
#endif

namespace h2dlp {

constexpr int RHS_TILE = 16;   // right-hand sides per pass (the MFMA N dimension)

H2DLP_HD inline int64_t a_offset(int M, int K, int row, int col) {
    const int rt = row >> 4, i = row & 15, ks = col >> 2, kk = col & 3;
    const int rv = (M - 16 * rt) < 16 ? (M - 16 * rt) : 16;
    const int kv = (K - 4 * ks) < 4 ? (K - 4 * ks) : 4;
    return int64_t(4) * M * ks + int64_t(16) * rt * kv + kk * rv + i;
}

// One output tile of a grouped block product: rows [out_row, out_row + m) of
// the output array receive sum over blocks b in [blk_begin, blk_end) of A_b X_b.
struct ItemDesc {
    int32_t out_row;
    int32_t m;
    int32_t blk_begin;
    int32_t blk_end;
};

// A block: A at pool + a_off, shape m x k; its operand X_b is rows
// [src, src + k) of source array (src >> 31) (0 or 1).
struct BlkDesc {
    int64_t a_off;
    int32_t k;
    int32_t src;
};
constexpr int32_t SRC1 = int32_t(0x80000000u);

}  // namespace h2dlp
