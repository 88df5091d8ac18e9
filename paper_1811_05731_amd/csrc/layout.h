// Device data layout shared by the build kernels (writers) and the apply
// kernels (readers).  Internal to the library.
//
// Every dense block the apply multiplies -- a leaf's transposed column basis
// W_s^T (k x n_s), a coupling matrix S_ts (k x k), a leaf's row basis V_t
// (n_t x k) and a near-field block K|_{t x s} (n_t x n_s) -- is stored in the
// order in which a wave64 feeds it to the 16x16x4 MFMA as the A operand (lane
// l holds row l % 16, column l / 16 of a 16 x 4 tile), with no padding:
//
//  * columns come in G = K / 16 full groups of 16 and a tail of K - 16 G;
//  * group g, row tile rt (rv = min(16, M - 16 rt) valid rows) is one
//    contiguous chunk of 16 rv entries at 16 M g + 256 rt; entry
//    (16 rt + i, 16 g + 4 u + kk) sits at (kk rv + i) 4 + u, so a lane reads
//    the four k-steps u of its (i, kk) with one 4-element load;
//  * the tail follows at 16 M G, cut into k-steps of kv <= 4 columns; chunk
//    (ks, rt) of rv kv entries at 4 M ks + 16 rt kv, entry at kk rv + i.
//
// Only the last row tile and the last tail k-step can be partial.  Blocks
// start on 16-element boundaries (BLOCK_ALIGN) so the 4-element loads align.
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

constexpr int64_t BLOCK_ALIGN = 16;

H2DLP_HD inline int64_t align_block(int64_t off) { return (off + BLOCK_ALIGN - 1) / BLOCK_ALIGN * BLOCK_ALIGN; }

H2DLP_HD inline int64_t a_offset(int M, int K, int row, int col) {
    const int rt = row >> 4, i = row & 15;
    const int rv = (M - 16 * rt) < 16 ? (M - 16 * rt) : 16;
    const int G = K >> 4;
    if (col < 16 * G) {
        const int g = col >> 4, u = (col & 15) >> 2, kk = col & 3;
        return int64_t(16) * M * g + 256 * rt + (kk * rv + i) * 4 + u;
    }
    const int c = col - 16 * G, ks = c >> 2, kk = c & 3, kt = K - 16 * G;
    const int kv = (kt - 4 * ks) < 4 ? (kt - 4 * ks) : 4;
    return int64_t(16) * M * G + int64_t(4) * M * ks + 16 * rt * kv + kk * rv + i;
}

// Split-bfloat16 coupling blocks (k <= 128): M x KP entries, KP = 32 ceil(k / 32)
// (zero columns past k), each entry a sum of P bfloat16 terms (P = 2: hi, lo;
// P = 3: hi, mid, lo).  Columns come in k-steps of 32; chunk (ks, rt) of row
// tile rt starts at bf16 index 32 P M ks + 512 P rt and lane (i, g) of the
// 16x16x32 MFMA owns 8 P contiguous values at (g rv + i) 8 P: term 0 of
// columns 32 ks + 8 g + j (j < 8), then term 1, ...
H2DLP_HD inline int64_t bf16s_offset(int M, int row, int col, int part, int P) {
    const int rt = row >> 4, i = row & 15;
    const int rv = (M - 16 * rt) < 16 ? (M - 16 * rt) : 16;
    const int ks = col >> 5, g = (col & 31) >> 3, j = col & 7;
    return int64_t(32 * P) * M * ks + 512 * P * rt + (g * rv + i) * 8 * P + 8 * part + j;
}
H2DLP_HD inline int bf16s_cols(int k) { return 32 * ((k + 31) / 32); }

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
