// Apply kernels: u2 = (K_H2 + D) u1, 16 right-hand sides per pass.
//
//   permute      x = P u1 (node order -> cluster order) in the operator
//                precision, plus an FP64 copy x64 on the FP32 path
//   diagonal     y64 = D x64 + the FP64 near-singular part (cluster order)
//   product      grouped block products Y_item = sum_b A_b X_b on MFMA 16x16x4
//                (FP32 or FP64), used for:
//                  leaf forward   xhat_s = W_s^T x|_s                     (one block per leaf)
//                  coupling       yhat_t = sum_{s admissible} S_ts xhat_s  (one item per cluster)
//                  near field     y64|_t += sum_{s near} K_ts x|_s
//                  leaf output    y64|_t += V_t yhat_t
//   upward       xhat_t = sum_c E_c^T xhat_c     (Kronecker mode products, per level)
//   downward     yhat_c += E_c yhat_parent        (top levels along paths, then per level)
//   unpermute    u2 = P^T y64
//
// The product kernel owns every output row it writes (no atomics): a
// workgroup of 4 waves takes one item, the waves split its blocks (or its row
// tiles), and partial sums meet in LDS in a fixed order, so results are
// bitwise reproducible.  A blocks stream from HBM straight into MFMA operand
// registers, four k-steps per lane load (layout.h); X rows come through L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "interp.h"
#include "kernels.h"

namespace h2dlp {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// A operand: lane l holds A[l % 16][l / 16]; B operand: B[l / 16][l % 16].
// The 16 x 16 result comes back as 4 values per lane, column l % 16; the row
// of value v in lane group g = l / 16 differs by type: 4 g + v for f32, g + 4 v
// for f64 (measured on gfx950, pinned by the GPU parity tests).
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    typedef f32x4 acc;
    typedef f32x4 vec4;
    static constexpr int kGroupUnroll = 2;
    static __device__ inline acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Mfma<double> {
    typedef f64x4 acc;
    typedef f64x4 vec4;
    static constexpr int kGroupUnroll = 1;
    static __device__ inline acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int g, int v) { return g + 4 * v; }
};

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8).  Items are grouped in chunks of kChunk neighbouring clusters, and
// XCD x takes chunks x, x + 8, x + 16, ...: neighbours share sources in one
// L2, while every XCD gets a slice of every level (the levels' costs differ
// widely, and a contiguous range per XCD left some with several times the
// work of others).  The grid is xcd_grid(n); items past n return at once.
constexpr int kChunk = 16;

__host__ __device__ inline unsigned xcd_grid(int n_items) {
    return unsigned(8 * kChunk * ((n_items + 8 * kChunk - 1) / (8 * kChunk)));
}

__device__ inline int xcd_item_of(int v, int n_items) {     // v: index in the grid xcd_grid(n)
    const int x = v & 7, j = v >> 3;
    const int item = ((j / kChunk) * 8 + x) * kChunk + j % kChunk;
    return item < n_items ? item : -1;
}

__device__ inline int xcd_item(int n_items) { return xcd_item_of(int(blockIdx.x), n_items); }

enum { EPI_STORE = 0, EPI_ADD64 = 2, EPI_ADD = 3 };

template <typename V>
__device__ inline V ld(const unsigned char* base, unsigned byte_off) {
    return *reinterpret_cast<const V*>(base + byte_off);   // SGPR base + 32-bit VGPR offset
}

// Accumulate sum_b A_b X_b of one item into acc[RTW] (row tiles t0 ... t0 + RTW - 1,
// all of them holding rows of the item).
//
// The item's blocks form a flat sequence of units -- each 16-column group of a
// block, then one unit for the block's tail of K - 16 G columns (up to 4
// k-steps loaded together); a wave walks every nbg-th unit with the next
// unit's loads in flight while the current unit's MFMAs run.  A unit is RTW vectors of
// 4 A entries (one per k-step u) and 4 B entries.  Each lane keeps, per row
// tile, the byte offset of its group vector; lanes past the rows of a partial
// tile read the group's first entries (finite values) and so only fill
// result rows past the item, which are never stored.
template <typename T, int RTW>
__device__ inline void accumulate(const ItemDesc& it, const BlkDesc* __restrict__ blks, const T* __restrict__ pool,
                                  const T* __restrict__ x0, const T* __restrict__ x1, int t0, int bg, int nbg,
                                  typename Mfma<T>::acc* acc) {
    typedef typename Mfma<T>::vec4 vec4;
    constexpr unsigned E = sizeof(T);
    const unsigned lane = threadIdx.x & 63;
    const unsigned i = lane & 15, kk = lane >> 4;
    const int M = it.m;
    unsigned goff[RTW], rvs[RTW];
    bool ok[RTW];
#pragma unroll
    for (int r = 0; r < RTW; ++r) {
        const int rt = t0 + r;
        rvs[r] = unsigned(M - 16 * rt < 16 ? M - 16 * rt : 16);
        ok[r] = i < rvs[r];
        goff[r] = ok[r] ? E * (256u * rt + 4u * (kk * rvs[r] + i)) : 0u;
    }
    const unsigned xoff = E * lane;
    const unsigned gstep = E * 16u * unsigned(M);
    const unsigned char* P = reinterpret_cast<const unsigned char*>(pool);

    auto load_unit = [&](const BlkDesc& d, int g, vec4* av, T* bv) {
        const unsigned char* Ab = P + int64_t(d.a_off) * E;
        const unsigned char* Xb = reinterpret_cast<const unsigned char*>(
            ((d.src & SRC1) ? x1 : x0) + int64_t(d.src & 0x7fffffff) * RHS_TILE);
        const int G = d.k >> 4;
        if (g < G) {
#pragma unroll
            for (int u = 0; u < 4; ++u) bv[u] = ld<T>(Xb + E * (256u * g + 64u * u), xoff);
#pragma unroll
            for (int r = 0; r < RTW; ++r) av[r] = ld<vec4>(Ab + gstep * g, goff[r]);
        } else {
            const int kt = d.k - 16 * G;
            const unsigned char* At = Ab + gstep * G;
            const unsigned char* Xt = Xb + E * 256u * G;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int kvi = kt - 4 * u;
                const unsigned kv = unsigned(kvi < 0 ? 0 : (kvi < 4 ? kvi : 4));
                const T bl = ld<T>(Xt, kk < kv ? E * 64u * u + xoff : 0u);
                bv[u] = kk < kv ? bl : T(0);
#pragma unroll
                for (int r = 0; r < RTW; ++r) {
                    const unsigned rt = unsigned(t0 + r);
                    const bool valid = ok[r] && kk < kv;
                    const T al = ld<T>(At, valid ? E * (4u * M * u + 16u * rt * kv + kk * rvs[r] + i) : 0u);
                    av[r][u] = valid ? al : T(0);
                }
            }
        }
    };
    auto compute = [&](const vec4* av, const T* bv) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < RTW; ++r) acc[r] = Mfma<T>::mma(av[r][u], bv[u], acc[r]);
    };

    // the item's units (every 16-column group of every block, then the block's
    // tail) form one sequence; the wave takes units bg, bg + nbg, bg + 2 nbg, ...
    // so blocks of very different widths still split evenly
    int b = it.blk_begin, g = bg;
    BlkDesc d{};
    int units = 0;
    auto settle = [&]() {                          // move (b, g) onto an existing unit
        while (b < it.blk_end) {
            d = blks[b];
            units = (d.k >> 4) + ((d.k & 15) != 0);
            if (g < units) return;
            g -= units;
            ++b;
        }
    };
    auto advance = [&]() {
        g += nbg;
        if (g >= units) settle();
    };
    settle();
    if (b >= it.blk_end) return;
    vec4 a0[RTW], a1[RTW];
    T b0[4], b1[4];
    load_unit(d, g, a0, b0);
    advance();
    while (true) {
        const bool more1 = b < it.blk_end;
        if (more1) {
            load_unit(d, g, a1, b1);
            advance();
        }
        compute(a0, b0);
        if (!more1) break;
        const bool more0 = b < it.blk_end;
        if (more0) {
            load_unit(d, g, a0, b0);
            advance();
        }
        compute(a1, b1);
        if (!more0) break;
    }
}

// accumulate over the wave's row tiles that hold rows of the item (live of
// RTW; uniform per wave): a leaf of 40 rows takes 3 tiles, not 4, and the
// dead tiles cost neither loads nor MFMAs.
template <typename T, int NR>
__device__ inline void accumulate_live(int live, const ItemDesc& it, const BlkDesc* __restrict__ blks,
                                       const T* __restrict__ pool, const T* __restrict__ x0, const T* __restrict__ x1,
                                       int t0, int bg, int nbg, typename Mfma<T>::acc* acc) {
    if constexpr (NR > 0) {
        if (live >= NR) {
            accumulate<T, NR>(it, blks, pool, x0, x1, t0, bg, nbg, acc);
            return;
        }
        accumulate_live<T, NR - 1>(live, it, blks, pool, x0, x1, t0, bg, nbg, acc);
    }
}

// One item of a grouped product.  Every wave of the workgroup runs it; the
// barriers inside are reached by all waves (waves with nothing left to store
// leave only after the last one).
template <typename T, int RTW, int NRG, int EPI>
__device__ inline void product_item(const ProductArgs& a, double* y64, int item, T* red) {
    typedef typename Mfma<T>::acc acc_t;
    constexpr int NBG = kWaves / NRG;
    const ItemDesc it = a.items[item];
    // the wave index is uniform per wave: keep block descriptors and base pointers in SGPRs
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int rg = w % NRG, bg = w / NRG;

    acc_t acc[RTW];
#pragma unroll
    for (int r = 0; r < RTW; ++r) acc[r] = acc_t{0, 0, 0, 0};
    const int live = __builtin_amdgcn_readfirstlane(((it.m + 15) >> 4) - rg * RTW);
    accumulate_live<T, RTW>(live, it, a.blks, static_cast<const T*>(a.pool), static_cast<const T*>(a.x0),
                            static_cast<const T*>(a.x1), rg * RTW, bg, NBG, acc);

    if (NBG > 1) {   // fixed-order reduction of the block groups
        if (bg > 0) {
            T* slot = red + ((bg - 1) * NRG + rg) * RTW * 256;
#pragma unroll
            for (int r = 0; r < RTW; ++r)
#pragma unroll
                for (int v = 0; v < 4; ++v) slot[(r * 4 + v) * 64 + lane] = acc[r][v];
        }
        __syncthreads();
        if (bg == 0)
            for (int g = 1; g < NBG; ++g) {
                const T* slot = red + ((g - 1) * NRG + rg) * RTW * 256;
#pragma unroll
                for (int r = 0; r < RTW; ++r)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[r][v] += slot[(r * 4 + v) * 64 + lane];
            }
        if (bg > 0) return;
    }

    const int M = it.m;
    const int q = lane & 15;
    if (EPI == EPI_ADD64) {          // y64 += the item's rows (cluster order)
#pragma unroll
        for (int r = 0; r < RTW; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * (rg * RTW + r) + Mfma<T>::row(lane >> 4, v);
                if (row < M) y64[(int64_t(it.out_row) + row) * RHS_TILE + q] += double(acc[r][v]);
            }
        return;
    }
    // y = acc, or y += acc in the operator precision
#pragma unroll
    for (int r = 0; r < RTW; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * (rg * RTW + r) + Mfma<T>::row(lane >> 4, v);
            if (row < M) {
                T* o = static_cast<T*>(a.y) + (int64_t(it.out_row) + row) * RHS_TILE + q;
                *o = EPI == EPI_ADD ? *o + acc[r][v] : acc[r][v];
            }
        }
}

// One item per workgroup, grid xcd_grid(n).
template <typename T, int RTW, int NRG, int EPI>
__global__ void __launch_bounds__(kThreads) k_product(ProductArgs a, double* y64) {
    extern __shared__ unsigned char smem_raw[];
    T* red = reinterpret_cast<T*>(smem_raw);
    const int item = xcd_item(a.n_items);
    if (item >= 0) product_item<T, RTW, NRG, EPI>(a, y64, item, red);
}

// y64 = D x64 + sum over the node's near-singular pairs of w x64 (FP64), for
// every cluster position and all 16 columns: the part of the near field that
// stays in FP64 when the blocks are stored in lower precision (ns_off NULL:
// D x64 alone).  One thread per (position, 4 columns): each pair's position
// and weight are loaded once per 4 columns, the x64 rows as two 16-byte loads,
// four pairs in flight.
__global__ void __launch_bounds__(256) k_diag_nearsing(int64_t n, LeafEpilogue e) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t pos = t >> 2;
    const int c0 = int(t & 3) * 4;
    if (pos >= n) return;
    const double d = e.diag[pos];
    const d2* xr = reinterpret_cast<const d2*>(e.x64 + pos * RHS_TILE + c0);
    const d2 xa = xr[0], xb = xr[1];
    d2 ya = d * xa, yb = d * xb;
    if (e.ns_off != nullptr) {
        const int64_t e1 = e.ns_off[pos + 1];
        d2 sa = {0.0, 0.0}, sb = {0.0, 0.0};
        int64_t q = e.ns_off[pos];
        for (; q + 4 <= e1; q += 4) {
            int32_t p[4];
            double w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                p[j] = e.ns_pos[q + j];
                w[j] = e.ns_val[q + j];
            }
            d2 ua[4], ub[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const d2* xs = reinterpret_cast<const d2*>(e.x64 + int64_t(p[j]) * RHS_TILE + c0);
                ua[j] = xs[0];
                ub[j] = xs[1];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                sa += w[j] * ua[j];
                sb += w[j] * ub[j];
            }
        }
        for (; q < e1; ++q) {
            const double w = e.ns_val[q];
            const d2* xs = reinterpret_cast<const d2*>(e.x64 + int64_t(e.ns_pos[q]) * RHS_TILE + c0);
            sa += w * xs[0];
            sb += w * xs[1];
        }
        ya += sa;
        yb += sb;
    }
    d2* yr = reinterpret_cast<d2*>(e.y64 + pos * RHS_TILE + c0);
    yr[0] = ya;
    yr[1] = yb;
}

// Coupling products yhat_t = sum_s S_ts xhat_s for orders with k <= 128.  Every
// S_ts is stored k x kp, kp = 16 RT (columns k..kp-1 zero), so a block is RT
// uniform 16-column groups.  A wave takes every 4th block of its item and walks
// the flattened (block, group) sequence with the next group's loads in flight
// while the current group's MFMAs run; B rows >= k are read as zero.
template <typename T, int RT>
__global__ void __launch_bounds__(kThreads) k_coupling(ProductArgs a, int kvalid) {
    typedef typename Mfma<T>::acc acc_t;
    typedef typename Mfma<T>::vec4 vec4;
    constexpr unsigned E = sizeof(T);
    constexpr int G = RT;
    extern __shared__ unsigned char smem_raw[];
    T* red = reinterpret_cast<T*>(smem_raw);

    const int item = xcd_item(a.n_items);
    if (item < 0) return;
    const ItemDesc it = a.items[item];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned lane = threadIdx.x & 63;
    const unsigned i = lane & 15, kk = lane >> 4;
    const int M = it.m;
    unsigned goff[RT];
    bool ok[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const unsigned rv = unsigned(M - 16 * r < 16 ? M - 16 * r : 16);
        ok[r] = i < rv;
        goff[r] = ok[r] ? E * (256u * r + 4u * (kk * rv + i)) : 0u;
    }
    const unsigned gstep = E * 16u * unsigned(M);
    const unsigned char* pool = static_cast<const unsigned char*>(a.pool);
    const unsigned char* xh = static_cast<const unsigned char*>(a.x0);
    const int first = it.blk_begin + w;
    const int nb = first < it.blk_end ? (it.blk_end - first + kWaves - 1) / kWaves : 0;
    const int units = nb * G;

    acc_t acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r] = acc_t{0, 0, 0, 0};
    vec4 a0[RT], a1[RT];
    T b0[4], b1[4];

    auto load = [&](int n, vec4* av, T* bv) {
        const int j = n / G, g = n - j * G;
        const BlkDesc d = a.blks[first + kWaves * j];
        const unsigned char* Ab = pool + int64_t(d.a_off) * E + gstep * g;
        const unsigned char* Xb = xh + (int64_t(d.src) * RHS_TILE + 256 * g) * E;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool in = 16 * g + 4 * u + int(kk) < kvalid;
            const T v = ld<T>(Xb, in ? E * (64u * u + lane) : 0u);
            bv[u] = in ? v : T(0);
        }
#pragma unroll
        for (int r = 0; r < RT; ++r) av[r] = ld<vec4>(Ab, goff[r]);
    };
    auto compute = [&](const vec4* av, const T* bv) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = Mfma<T>::mma(ok[r] ? av[r][u] : T(0), bv[u], acc[r]);
    };
    int n = 0;
    if (units > 0) load(0, a0, b0);
    for (; n + 2 <= units; n += 2) {
        load(n + 1, a1, b1);
        compute(a0, b0);
        if (n + 2 < units) load(n + 2, a0, b0);
        compute(a1, b1);
    }
    if (n < units) compute(a0, b0);

    // fixed-order reduction of the 4 waves, then store rows < M
    if (w > 0) {
        T* slot = red + (w - 1) * RT * 256;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) slot[(r * 4 + v) * 64 + lane] = acc[r][v];
    }
    __syncthreads();
    if (w > 0) return;
    for (int g = 1; g < kWaves; ++g) {
        const T* slot = red + (g - 1) * RT * 256;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[r][v] += slot[(r * 4 + v) * 64 + lane];
    }
    const int q = lane & 15;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * r + Mfma<T>::row(lane >> 4, v);
            if (row < M) static_cast<T*>(a.y)[(int64_t(it.out_row) + row) * RHS_TILE + q] = acc[r][v];
        }
}

// Generated coupling products (orders 1..5): yhat_t = sum_s S_ts xhat_s with
// S_ts(nu, mu) = 1/(4 pi |eta^t_nu - eta^s_mu|) computed in registers instead
// of read from memory.  eta^t_nu - eta^s_mu = (c_t - c_s) + h_t o_nu - h_s o_mu,
// with c the box centre, h the half extent and o the unit Chebyshev nodes: the
// centre difference is taken in FP64 and rounded once, the offsets are at most
// a box size, so the difference keeps the precision of T even for close
// blocks.  1/(4 pi) is applied once to the output.
//
// The sum over mu may run in any order (B rows follow the same order), so the
// 4 lane groups of the MFMA's K dimension are given columns that keep the
// work separable: in the main part lane group g always has mu_x = 4 q + g
// (q < m / 4) while (mu_y, mu_z) is the same for the whole wave in a k-step,
// so |d|^2 = dx^2[row] + dy^2[row][mu_y] + dz^2[row][mu_z] from per-block
// tables; the remaining mu_x (m mod 4 values, all m^2 pairs) form a tail of
// k-steps with per-lane columns.  FP32 uses v_rsq_f32 and FP64 refines v_rsq_f64
// with two Newton steps.
//
// Padding takes no masks: a row past K (its offset is that of node 0) only
// feeds an output row that is never stored, and a tail column past the block
// (again a real node's offset) meets a zero B value; both distances are
// between two separated boxes, so every entry is finite.
struct UnitNodes {
    double o[8];
};

template <typename T>
__device__ inline T rsqrt_kernel(T d2);
template <>
__device__ inline float rsqrt_kernel<float>(float d2) {
    return __builtin_amdgcn_rsqf(d2);
}
template <>
__device__ inline double rsqrt_kernel<double>(double d2) {
    double y = __builtin_amdgcn_rsq(d2);
    const double hd = 0.5 * d2;
    y = y * (1.5 - hd * y * y);
    y = y * (1.5 - hd * y * y);
    return y;
}

#ifndef H2DLP_GEN_WAVES
#define H2DLP_GEN_WAVES 2      // minimum waves per SIMD the register allocation must allow
#endif

// ROWS = false: the 4 waves split the item's blocks and meet in LDS; ROWS =
// true (RT a multiple of 4): wave w owns row tiles [w RT/4, (w + 1) RT/4) of
// every block, so each wave keeps a quarter of the accumulators and stores its
// rows itself.
template <typename T, int M, bool ROWS>
__device__ inline void coupling_gen_item(const ProductArgs& a, const UnitNodes& un, int item, T* red) {
    typedef typename Mfma<T>::acc acc_t;
    constexpr int K = M * M * M, MM = M * M, RTA = (K + 15) / 16;
    static_assert(!ROWS || RTA % kWaves == 0, "row split needs a multiple of 4 row tiles");
    constexpr int RT = ROWS ? RTA / kWaves : RTA;    // row tiles of this wave
    constexpr int Q = M / 4, R = M % 4;
    constexpr int KS_TAIL = (R * MM + 3) / 4;
    // the nodes, and the target rows' offsets h_t o_nu from the box centre
    // (the same for the 4 waves: all work on one target cluster)
    __shared__ T su[8];
    __shared__ T sot[3][16 * RTA];

    const ItemDesc it = a.items[item];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned lane = threadIdx.x & 63;
    const int i = int(lane & 15), g = int(lane >> 4);
    const double* geo = static_cast<const double*>(a.pool);
    const T* xh = static_cast<const T*>(a.x0);
    T u[M];
#pragma unroll
    for (int l = 0; l < M; ++l) u[l] = T(un.o[l]);
#pragma unroll
    for (int l = 0; l < M; ++l)
        if (threadIdx.x == unsigned(l)) su[l] = u[l];
    const int t = it.out_row / K;
    const double ctx = geo[6 * t], cty = geo[6 * t + 1], ctz = geo[6 * t + 2];
    if (threadIdx.x < 16 * RTA) {
        const int nu = int(threadIdx.x) < K ? int(threadIdx.x) : 0;
        T vx = u[0], vy = u[0], vz = u[0];
#pragma unroll
        for (int l = 1; l < M; ++l) {
            vx = nu % M == l ? u[l] : vx;
            vy = (nu / M) % M == l ? u[l] : vy;
            vz = nu / MM == l ? u[l] : vz;
        }
        sot[0][threadIdx.x] = T(geo[6 * t + 3]) * vx;
        sot[1][threadIdx.x] = T(geo[6 * t + 4]) * vy;
        sot[2][threadIdx.x] = T(geo[6 * t + 5]) * vz;
    }
    __syncthreads();

    acc_t acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r] = acc_t{0, 0, 0, 0};

    const int r0 = ROWS ? w * RT : 0;                // first row tile of this wave
    const int first = ROWS ? it.blk_begin : it.blk_begin + w;
    const int stride = ROWS ? 1 : kWaves;
    constexpr int NB = Q * MM + KS_TAIL;               // k-steps (B values) per block
    constexpr bool kTables = ROWS;                     // few row tiles per wave: per-block distance tables
    // order 5: the tail (mu_x = 4, all 25 (mu_y, mu_z)) also reads the tables;
    // k-steps 0-4 give lane group g mu_y = g with mu_z = step, k-step 5 gives
    // mu_y = 4 with mu_z = g, and k-step 6 the last pair (4, 4) to group 0
    constexpr bool kTail5 = kTables && M == 5;

    // B operands of a block: x rows through L2
    auto load_b = [&](int b, T* bv) {
        const T* X = xh + int64_t(a.blks[b].src) * RHS_TILE + i;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int p = 0; p < MM; ++p) bv[q * MM + p] = X[(4 * q + g + M * p) * RHS_TILE];
        if constexpr (kTail5) {
#pragma unroll
            for (int ts = 0; ts < KS_TAIL; ++ts) {
                const int mu = ts < 5 ? 4 + M * (g + M * ts) : (ts == 5 ? 4 + M * (4 + M * g) : K - 1);
                const T v = X[mu * RHS_TILE];
                bv[Q * MM + ts] = ts < 6 || g == 0 ? v : T(0);
            }
        } else {
#pragma unroll
            for (int ts = 0; ts < KS_TAIL; ++ts) {
                const int c = 4 * ts + g;
                const int cc = c < R * MM ? c : 0;
                const T v = X[(4 * Q + cc % (R > 0 ? R : 1) + M * (cc / (R > 0 ? R : 1))) * RHS_TILE];
                bv[Q * MM + ts] = c < R * MM ? v : T(0);
            }
        }
    };
    auto block = [&](int b, const T* bv) {
        const int sc = int(a.blks[b].a_off);
        const T dx0 = T(ctx - geo[6 * sc]), dy0 = T(cty - geo[6 * sc + 1]), dz0 = T(ctz - geo[6 * sc + 2]);
        const T hsx = T(geo[6 * sc + 3]), hsy = T(geo[6 * sc + 4]), hsz = T(geo[6 * sc + 5]);
        T ax[RT], ay[RT], az[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            ax[r] = dx0 + sot[0][16 * (r0 + r) + i];
            ay[r] = dy0 + sot[1][16 * (r0 + r) + i];
            az[r] = dz0 + sot[2][16 * (r0 + r) + i];
        }
        // dy^2 and dz^2 per row and node, for the tables of every k-step
        T dy2[kTables ? RT : 1][kTables ? M : 1], dz2[kTables ? RT : 1][kTables ? M : 1];
        if constexpr (kTables) {
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int l = 0; l < M; ++l) {
                    const T ey = ay[r] - hsy * u[l], ez = az[r] - hsz * u[l];
                    dy2[r][l] = ey * ey;
                    dz2[r][l] = ez * ez;
                }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const T osx = hsx * su[4 * q + g];
            T dx2[RT];
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const T e = ax[r] - osx;
                dx2[r] = e * e;
            }
            // |d|^2 = (dx^2 + dy^2)[row][mu_y] + dz^2[row][mu_z]
            T dxy2[kTables ? RT : 1][kTables ? M : 1];
            if constexpr (kTables) {
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int l = 0; l < M; ++l) dxy2[r][l] = dx2[r] + dy2[r][l];
            }
#pragma unroll
            for (int p = 0; p < MM; ++p) {
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    T d2;
                    if constexpr (kTables) {
                        d2 = dxy2[r][p % M] + dz2[r][p / M];
                    } else {
                        const T ey = ay[r] - hsy * u[p % M], ez = az[r] - hsz * u[p / M];
                        d2 = dx2[r] + ey * ey + ez * ez;
                    }
                    acc[r] = Mfma<T>::mma(rsqrt_kernel<T>(d2), bv[q * MM + p], acc[r]);
                }
            }
        }
        if constexpr (kTail5) {
            const T ug = su[g], osx = hsx * su[4];
            T base[RT], b4[RT], ezg2[RT];
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const T ex = ax[r] - osx, eyg = ay[r] - hsy * ug, ezg = az[r] - hsz * ug;
                const T dx2 = ex * ex;
                base[r] = dx2 + eyg * eyg;             // mu_x = 4, mu_y = g
                b4[r] = dx2 + dy2[r][4];               // mu_x = 4, mu_y = 4
                ezg2[r] = ezg * ezg;                   // mu_z = g
            }
#pragma unroll
            for (int ts = 0; ts < 5; ++ts)
#pragma unroll
                for (int r = 0; r < RT; ++r)
                    acc[r] = Mfma<T>::mma(rsqrt_kernel<T>(base[r] + dz2[r][ts]), bv[Q * MM + ts], acc[r]);
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = Mfma<T>::mma(rsqrt_kernel<T>(b4[r] + ezg2[r]), bv[Q * MM + 5], acc[r]);
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = Mfma<T>::mma(rsqrt_kernel<T>(b4[r] + dz2[r][4]), bv[Q * MM + 6], acc[r]);
        } else {
#pragma unroll
            for (int ts = 0; ts < KS_TAIL; ++ts) {
                const int c = 4 * ts + g;
                const bool ok = c < R * MM;
                const int cc = ok ? c : 0;
                const int p = cc / (R > 0 ? R : 1);
                const T osx = hsx * su[4 * Q + cc % (R > 0 ? R : 1)], osy = hsy * su[p % M], osz = hsz * su[p / M];
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    const T ex = ax[r] - osx, ey = ay[r] - osy, ez = az[r] - osz;
                    const T d2 = ex * ex + ey * ey + ez * ez;
                    acc[r] = Mfma<T>::mma(rsqrt_kernel<T>(d2), bv[Q * MM + ts], acc[r]);
                }
            }
        }
    };

    // one block at a time: holding the next block's B values as well would cost
    // registers, and a fourth wave per SIMD hides the load latency better
    // (measured 1.9 against 2.9 ms at L8 beside the near field)
    T b0[NB];
    for (int b = first; b < it.blk_end; b += stride) {
        load_b(b, b0);
        block(b, b0);
    }

    const T scale = T(0.25 / 3.14159265358979323846);
    if constexpr (ROWS) {                          // each wave stores its own rows
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * (r0 + r) + Mfma<T>::row(g, v);
                if (row < K) static_cast<T*>(a.y)[(int64_t(it.out_row) + row) * RHS_TILE + i] = acc[r][v] * scale;
            }
        return;
    }
    // fixed-order reduction of the 4 waves, then store rows < K scaled by 1/(4 pi)
    if (w > 0) {
        T* slot = red + (w - 1) * RT * 256;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) slot[(r * 4 + v) * 64 + lane] = acc[r][v];
    }
    __syncthreads();
    if (w > 0) return;
    for (int q = 1; q < kWaves; ++q) {
        const T* slot = red + (q - 1) * RT * 256;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[r][v] += slot[(r * 4 + v) * 64 + lane];
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * r + Mfma<T>::row(g, v);
            if (row < K) static_cast<T*>(a.y)[(int64_t(it.out_row) + row) * RHS_TILE + i] = acc[r][v] * scale;
        }
}

template <typename T, int M, bool ROWS>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(H2DLP_GEN_WAVES)))
k_coupling_gen(ProductArgs a, UnitNodes un) {
    extern __shared__ unsigned char smem_raw[];
    const int item = xcd_item(a.n_items);
    if (item >= 0) coupling_gen_item<T, M, ROWS>(a, un, item, reinterpret_cast<T*>(smem_raw));
}

// Split-bfloat16 coupling products (k <= 128).  S_ts is pre-split at build time
// into P bfloat16 terms (layout.h, split layout); xhat is split here into P
// terms the same way.  P = 2 (BF16X3): S xhat ~ S1 x1 + S1 x2 + S2 x1.  P = 3
// (BF16X6): S1 x1 + S1 x2 + S2 x1 + S1 x3 + S2 x2 + S3 x1, every product of
// combined order <= 3.  All on the 16x16x32 bf16 MFMA with FP32 accumulation.
// A k-step covers 32 columns: lane group g, slot j holds column 32 ks + 8 g + j
// in both operands, so the sum over the MFMA's K dimension is the sum over
// those columns whatever order the unit uses inside.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <int RT, int P>
__global__ void __launch_bounds__(kThreads) k_coupling_bf16s(ProductArgs a, int kvalid) {
    constexpr int KS = (RT + 1) / 2;          // 32-column k-steps per block
    extern __shared__ unsigned char smem_raw[];
    float* red = reinterpret_cast<float*>(smem_raw);
    const int item = xcd_item(a.n_items);
    if (item < 0) return;
    const ItemDesc it = a.items[item];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned lane = threadIdx.x & 63;
    const unsigned i = lane & 15, g = lane >> 4;
    const int M = it.m;
    unsigned loff[RT];
    bool ok[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const unsigned rv = unsigned(M - 16 * r < 16 ? M - 16 * r : 16);
        ok[r] = i < rv;
        loff[r] = ok[r] ? 1024u * P * r + 16u * P * (g * rv + i) : 0u;   // bytes
    }
    const unsigned kbytes = 64u * P * unsigned(M);                       // one k-step: M rows x 32 entries
    const unsigned char* pool = static_cast<const unsigned char*>(a.pool);
    const float* xh = static_cast<const float*>(a.x0);
    const int first = it.blk_begin + w;
    const int nb = first < it.blk_end ? (it.blk_end - first + kWaves - 1) / kWaves : 0;
    const int units = nb * KS;

    f32x4 acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r] = f32x4{0, 0, 0, 0};
    u32x4 s0[P][RT], s1[P][RT];
    float x0v[8], x1v[8];

    auto load = [&](int n, u32x4 (*sv)[RT], float* xv) {
        const int j = n / KS, ks = n - j * KS;
        const BlkDesc d = a.blks[first + kWaves * j];
        const unsigned char* Ab = pool + int64_t(d.a_off) * (2 * P) + kbytes * ks;
        const float* X = xh + int64_t(d.src) * RHS_TILE;
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const int row = 32 * ks + 8 * int(g) + jj;
            const float v = X[(row < kvalid ? row : 32 * ks) * RHS_TILE + i];
            xv[jj] = row < kvalid ? v : 0.f;
        }
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int q = 0; q < P; ++q) sv[q][r] = ld<u32x4>(Ab, loff[r] + 16u * q);
    };
    auto compute = [&](u32x4 (*sv)[RT], const float* xv) {
        bf16x8 bx[P];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            float rem = xv[jj];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const __bf16 t = __bf16(rem);
                bx[q][jj] = t;
                rem -= float(t);                   // exact: what the earlier terms leave
            }
        }
        const u32x4 zero = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            bf16x8 as[P];
#pragma unroll
            for (int q = 0; q < P; ++q) as[q] = __builtin_bit_cast(bf16x8, ok[r] ? sv[q][r] : zero);
            // products S_a x_b with a + b <= P - 1 (0-based term indices), highest order first
#pragma unroll
            for (int o = P - 1; o >= 0; --o)
#pragma unroll
                for (int q = 0; q <= o; ++q)
                    acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as[q], bx[o - q], acc[r], 0, 0, 0);
        }
    };
    int n = 0;
    if (units > 0) load(0, s0, x0v);
    for (; n + 2 <= units; n += 2) {
        load(n + 1, s1, x1v);
        compute(s0, x0v);
        if (n + 2 < units) load(n + 2, s0, x0v);
        compute(s1, x1v);
    }
    if (n < units) compute(s0, x0v);

    if (w > 0) {
        float* slot = red + (w - 1) * RT * 256;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) slot[(r * 4 + v) * 64 + lane] = acc[r][v];
    }
    __syncthreads();
    if (w > 0) return;
    for (int q = 1; q < kWaves; ++q) {
        const float* slot = red + (q - 1) * RT * 256;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[r][v] += slot[(r * 4 + v) * 64 + lane];
    }
    const int col = lane & 15;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * r + 4 * int(g) + v;
            if (row < M) static_cast<float*>(a.y)[(int64_t(it.out_row) + row) * RHS_TILE + col] = acc[r][v];
        }
}

// x[p][q] = u1[q][node] for the node at cluster position p = iperm[node];
// one thread per node: coalesced reads of u1, one contiguous row write.
template <typename IO, typename T>
__global__ void __launch_bounds__(256) k_permute(const IO* __restrict__ u1, int64_t n, int nr,
                                                 const int32_t* __restrict__ iperm, T* __restrict__ x,
                                                 double* __restrict__ x64) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t p = iperm[i];
    T v[RHS_TILE];
    double w[RHS_TILE];
#pragma unroll
    for (int q = 0; q < RHS_TILE; ++q) {
        w[q] = q < nr ? double(u1[int64_t(q) * n + i]) : 0.0;
        v[q] = T(w[q]);
    }
#pragma unroll
    for (int q = 0; q < RHS_TILE; ++q) x[p * RHS_TILE + q] = v[q];
    if (x64 != nullptr)
#pragma unroll
        for (int q = 0; q < RHS_TILE; ++q) x64[p * RHS_TILE + q] = w[q];
}

// u2[q][node] = y64[iperm[node]][q]; one thread per node.
template <typename IO>
__global__ void __launch_bounds__(256) k_unpermute(const double* __restrict__ y64, int64_t n, int nr,
                                                   const int32_t* __restrict__ iperm, IO* __restrict__ u2) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t p = iperm[i];
    double v[RHS_TILE];
#pragma unroll
    for (int q = 0; q < RHS_TILE; ++q) v[q] = y64[p * RHS_TILE + q];
#pragma unroll
    for (int q = 0; q < RHS_TILE; ++q)
        if (q < nr) u2[int64_t(q) * n + i] = IO(v[q]);
}

// Leaf output with the row basis regenerated: y64|_t += V_t yhat_t, where
// V_t(i, nu) = Lx_a(x) Ly_b(y) Lz_c(z), nu = a + m b + m^2 c, is evaluated
// here instead of read from memory (Section 4: the row factors are the
// Lagrange polynomials of the leaf box's Chebyshev points at the collocation
// nodes).  Each 1D value is w_l prod_{p != l} (x - p_p) with the barycentric
// weight w_l = 1 / prod_{p != l} (p_l - p_p); the product of the three is
// taken in FP64 and rounded once to T, as the stored basis is.  One wave per
// leaf (at most 64 nodes), one lane per node with the 16 columns in
// registers; the leaf's yhat (k x 16) is staged in LDS with coalesced loads
// and every lane reads the same row of it (broadcast).
template <typename T, int M>
__global__ void __launch_bounds__(64) k_leaf_regen(const VLeaf* __restrict__ leaves, const double* __restrict__ xyz,
                                                   const T* __restrict__ yh, double* __restrict__ y64) {
    constexpr int K = M * M * M;
    constexpr int VEC = 16 / int(sizeof(T));                 // values per 16-byte load
    __shared__ double pts[3][M], wts[3][M];
    __shared__ __attribute__((aligned(16))) T ys[K * RHS_TILE];
    const VLeaf* L = leaves + blockIdx.x;
    const int32_t pos = L->pos, n = L->n;
    const int i = int(threadIdx.x);
    {
        using V4 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
        const V4* src = reinterpret_cast<const V4*>(yh + int64_t(L->yrow) * RHS_TILE);
        V4* dst = reinterpret_cast<V4*>(ys);
        for (int q = i; q < K * RHS_TILE / VEC; q += 64) dst[q] = src[q];
    }
    if (i < 3 * M) pts[i / M][i % M] = cheb_point(L->box, i / M, M, i % M);
    __syncthreads();
    if (i < 3 * M) {
        const int a = i / M, l = i % M;
        double d = 1.0;
        for (int p = 0; p < M; ++p)
            if (p != l) d *= pts[a][l] - pts[a][p];
        wts[a][l] = 1.0 / d;
    }
    __syncthreads();
    if (i >= n) return;
    const double* x = xyz + 3 * int64_t(pos + i);
    double lx[M], ly[M];
#pragma unroll
    for (int l = 0; l < M; ++l) {
        double vx = wts[0][l], vy = wts[1][l];
#pragma unroll
        for (int p = 0; p < M; ++p)
            if (p != l) {
                vx *= x[0] - pts[0][p];
                vy *= x[1] - pts[1][p];
            }
        lx[l] = vx;
        ly[l] = vy;
    }
    T acc[RHS_TILE];
#pragma unroll
    for (int r = 0; r < RHS_TILE; ++r) acc[r] = T(0);
    for (int c = 0; c < M; ++c) {
        double lz = wts[2][c];
#pragma unroll
        for (int p = 0; p < M; ++p)
            if (p != c) lz *= x[2] - pts[2][p];
#pragma unroll
        for (int b = 0; b < M; ++b)
#pragma unroll
            for (int a = 0; a < M; ++a) {
                const T v = T(lx[a] * ly[b] * lz);
                const T* yr = ys + RHS_TILE * (a + M * b + M * M * c);
#pragma unroll
                for (int r = 0; r < RHS_TILE; ++r) acc[r] = fma(v, yr[r], acc[r]);
            }
    }
    double* out = y64 + int64_t(pos + i) * RHS_TILE;
#pragma unroll
    for (int r = 0; r < RHS_TILE; ++r) out[r] += double(acc[r]);
}

// One mode product of the Kronecker transfer E = Ex (x) Ey (x) Ez on a k x QC
// slab in LDS (index nu = lx + m ly + m^2 lz, columns innermost), one thread
// per line of M values along the axis:
//   UP: out[l] = sum_l' E[l'][l] in[l']  (E^T)     else  out[l'] = sum_l E[l'][l] in[l]
// One mode product of a Kronecker transfer on a k x QC slab in LDS, done by
// `nt` threads starting at `t0`: along AXIS, out = E^T in (UP) or E in
// (out += ... with ADD).
template <typename T, int M, int QC, int AXIS, bool UP, bool ADD = false>
__device__ inline void mode_product(const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ e, int t0,
                                    int nt) {
    constexpr int STRIDE = AXIS == 0 ? 1 : (AXIS == 1 ? M : M * M);
    for (int line = int(threadIdx.x) - t0; line < M * M * QC; line += nt) {
        const int q = line % QC, rest = line / QC;
        const int j1 = rest % M, j2 = rest / M;
        const int base = AXIS == 0 ? M * j1 + M * M * j2 : (AXIS == 1 ? j1 + M * M * j2 : j1 + M * j2);
        T v[M];
#pragma unroll
        for (int p = 0; p < M; ++p) v[p] = in[(base + p * STRIDE) * QC + q];
#pragma unroll
        for (int l = 0; l < M; ++l) {
            T s = 0;
#pragma unroll
            for (int p = 0; p < M; ++p) s += (UP ? e[p * M + l] : e[l * M + p]) * v[p];
            T* o = out + (base + l * STRIDE) * QC + q;
            *o = ADD ? *o + s : s;
        }
    }
}

// columns per slab: three k x QC slabs must fit in 48 KB of LDS
template <typename T, int M>
constexpr int transfer_qc() {
    int qc = RHS_TILE;
    while (qc > 1 && 3 * M * M * M * qc * int(sizeof(T)) > 48 * 1024) qc >>= 1;
    return qc;
}

// Upward transfer of one level: xhat_t = E_c0^T xhat_c0 + E_c1^T xhat_c1 per
// workgroup, one child after the other through its three mode products.
template <typename T, int M>
__global__ void __launch_bounds__(256) k_upward(int32_t c_begin, const int32_t* __restrict__ child0,
                                                const int32_t* __restrict__ child1, const T* __restrict__ efac,
                                                T* __restrict__ xh) {
    constexpr int K = M * M * M, QC = transfer_qc<T, M>(), MM = M * M;
    __shared__ T e[2][3][MM];
    __shared__ T b0[K * QC], b1[K * QC], acc[K * QC];
    const int32_t c = c_begin + blockIdx.x;
    const int32_t ch[2] = {child0[c], child1[c]};
    if (ch[0] < 0) return;   // leaf: its xhat comes from the leaf forward
    for (int idx = threadIdx.x; idx < 6 * MM; idx += blockDim.x) {
        const int w = idx / (3 * MM), r = idx % (3 * MM);
        e[w][r / MM][r % MM] = efac[int64_t(ch[w]) * 3 * MM + r];
    }
    const int nt = int(blockDim.x);
    for (int q0 = 0; q0 < RHS_TILE; q0 += QC) {
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            __syncthreads();
            const T* src = xh + int64_t(ch[w]) * K * RHS_TILE + q0;
            for (int idx = threadIdx.x; idx < K * QC; idx += blockDim.x) b0[idx] = src[(idx / QC) * RHS_TILE + idx % QC];
            __syncthreads();
            mode_product<T, M, QC, 2, true>(b0, b1, e[w][2], 0, nt);
            __syncthreads();
            mode_product<T, M, QC, 1, true>(b1, b0, e[w][1], 0, nt);
            __syncthreads();
            if (w == 0) mode_product<T, M, QC, 0, true>(b0, acc, e[w][0], 0, nt);
            else mode_product<T, M, QC, 0, true, true>(b0, acc, e[w][0], 0, nt);
        }
        __syncthreads();
        T* dst = xh + int64_t(c) * K * RHS_TILE + q0;
        for (int idx = threadIdx.x; idx < K * QC; idx += blockDim.x) dst[(idx / QC) * RHS_TILE + idx % QC] = acc[idx];
    }
}

// Downward transfer of one level: yhat_c += E_c yhat_parent per workgroup; the
// parent's and the child's slabs come in with one round trip.
template <typename T, int M>
__global__ void __launch_bounds__(256) k_downward(int32_t c_begin, const int32_t* __restrict__ parent,
                                                  const T* __restrict__ efac, T* __restrict__ yh) {
    constexpr int K = M * M * M, QC = transfer_qc<T, M>(), MM = M * M;
    __shared__ T e[3][MM];
    __shared__ T b0[K * QC], b1[K * QC], own[K * QC];
    const int32_t c = c_begin + blockIdx.x;
    const int32_t p = parent[c];
    if (p < 0) return;
    for (int idx = threadIdx.x; idx < 3 * MM; idx += blockDim.x) e[idx / MM][idx % MM] = efac[int64_t(c) * 3 * MM + idx];
    T* dst = yh + int64_t(c) * K * RHS_TILE;
    const T* src = yh + int64_t(p) * K * RHS_TILE;
    for (int q0 = 0; q0 < RHS_TILE; q0 += QC) {
        for (int idx = threadIdx.x; idx < K * QC; idx += blockDim.x) {
            const int64_t o = (idx / QC) * RHS_TILE + q0 + idx % QC;
            b0[idx] = src[o];
            own[idx] = dst[o];
        }
        __syncthreads();
        mode_product<T, M, QC, 2, false>(b0, b1, e[2], 0, int(blockDim.x));
        __syncthreads();
        mode_product<T, M, QC, 1, false>(b1, b0, e[1], 0, int(blockDim.x));
        __syncthreads();
        mode_product<T, M, QC, 0, false>(b0, b1, e[0], 0, int(blockDim.x));
        __syncthreads();
        for (int idx = threadIdx.x; idx < K * QC; idx += blockDim.x)
            dst[(idx / QC) * RHS_TILE + q0 + idx % QC] = own[idx] + b1[idx];
        __syncthreads();
    }
}

// Downward pass over the top levels in one launch: workgroup b takes cluster
// d = front[b] and walks its path from the root, z = yhat_root, then
// z = yhat_a + E_a z for each cluster a below, down to d; only yhat_d is
// written.  The arithmetic of every step is that of k_downward, so the result
// is the same as level by level; the clusters above the front are computed
// once per path that passes through them instead of once (a few thousand
// extra transfers at most) to save a launch per level.  No cluster is both
// read and written: front clusters are at the front level or leaves, never
// on another front cluster's path.
template <typename T, int M>
__global__ void __launch_bounds__(256) k_downward_paths(const int32_t* __restrict__ front,
                                                        const int32_t* __restrict__ parent,
                                                        const T* __restrict__ efac, T* __restrict__ yh) {
    constexpr int K = M * M * M, QC = transfer_qc<T, M>(), MM = M * M;
    __shared__ T e[3][MM];
    __shared__ T b0[K * QC], b1[K * QC], own[K * QC];
    __shared__ int32_t path[kMaxPath];
    __shared__ int n_path;
    const int32_t d = front[blockIdx.x];
    if (threadIdx.x == 0) {
        int n = 0;
        for (int32_t c = d; c >= 0 && n < kMaxPath; c = parent[c]) path[n++] = c;
        n_path = n;
    }
    __syncthreads();
    const int n = n_path;
    if (n < 2) return;                                 // the root: its yhat is complete
    for (int q0 = 0; q0 < RHS_TILE; q0 += QC) {
        const T* root = yh + int64_t(path[n - 1]) * K * RHS_TILE;
        for (int idx = threadIdx.x; idx < K * QC; idx += blockDim.x) b0[idx] = root[(idx / QC) * RHS_TILE + q0 + idx % QC];
        for (int j = n - 2; j >= 0; --j) {
            const int32_t c = path[j];
            __syncthreads();
            for (int idx = threadIdx.x; idx < 3 * MM; idx += blockDim.x)
                e[idx / MM][idx % MM] = efac[int64_t(c) * 3 * MM + idx];
            const T* src = yh + int64_t(c) * K * RHS_TILE;
            for (int idx = threadIdx.x; idx < K * QC; idx += blockDim.x) own[idx] = src[(idx / QC) * RHS_TILE + q0 + idx % QC];
            __syncthreads();
            mode_product<T, M, QC, 2, false>(b0, b1, e[2], 0, int(blockDim.x));
            __syncthreads();
            mode_product<T, M, QC, 1, false>(b1, b0, e[1], 0, int(blockDim.x));
            __syncthreads();
            mode_product<T, M, QC, 0, false>(b0, b1, e[0], 0, int(blockDim.x));
            __syncthreads();
            for (int idx = threadIdx.x; idx < K * QC; idx += blockDim.x) b0[idx] = own[idx] + b1[idx];
        }
        __syncthreads();
        T* dst = yh + int64_t(d) * K * RHS_TILE;
        for (int idx = threadIdx.x; idx < K * QC; idx += blockDim.x) dst[(idx / QC) * RHS_TILE + q0 + idx % QC] = b0[idx];
        __syncthreads();
    }
}

inline int pow2ceil(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

template <typename T, int EPI>
hipError_t dispatch(const ProductArgs& a, double* y64, int rtw, int nrg, hipStream_t st) {
    const unsigned grid = a.n_items > 0 ? xcd_grid(a.n_items) : 0u;
    if (grid == 0) return hipSuccess;
    const int nbg = kWaves / nrg;
    const size_t lds = size_t(nbg - 1) * nrg * rtw * 256 * sizeof(T);
#define H2DLP_CASE(RTW_, NRG_)                                                                         \
    if (rtw == RTW_ && nrg == NRG_) {                                                                  \
        hipLaunchKernelGGL((k_product<T, RTW_, NRG_, EPI>), dim3(grid), dim3(kThreads), lds, st, a, y64); \
        return hipGetLastError();                                                                      \
    }
    H2DLP_CASE(1, 1) H2DLP_CASE(2, 1) H2DLP_CASE(4, 1) H2DLP_CASE(8, 1)
    H2DLP_CASE(1, 2) H2DLP_CASE(2, 2) H2DLP_CASE(4, 2) H2DLP_CASE(8, 2)
    H2DLP_CASE(1, 4) H2DLP_CASE(2, 4) H2DLP_CASE(4, 4) H2DLP_CASE(8, 4)
#undef H2DLP_CASE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t upward_m(int m, unsigned grid, hipStream_t st, int32_t c_begin, const int32_t* child0,
                    const int32_t* child1, const T* e, T* xh) {
    switch (m) {
#define H2DLP_M(MM_) case MM_: hipLaunchKernelGGL((k_upward<T, MM_>), dim3(grid), dim3(256), 0, st, c_begin, child0, child1, e, xh); break;
        H2DLP_M(1) H2DLP_M(2) H2DLP_M(3) H2DLP_M(4) H2DLP_M(5) H2DLP_M(6) H2DLP_M(7) H2DLP_M(8)
#undef H2DLP_M
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t downward_m(int m, unsigned grid, hipStream_t st, int32_t c_begin, const int32_t* parent, const T* e,
                      T* yh) {
    switch (m) {
#define H2DLP_M(MM_) case MM_: hipLaunchKernelGGL((k_downward<T, MM_>), dim3(grid), dim3(256), 0, st, c_begin, parent, e, yh); break;
        H2DLP_M(1) H2DLP_M(2) H2DLP_M(3) H2DLP_M(4) H2DLP_M(5) H2DLP_M(6) H2DLP_M(7) H2DLP_M(8)
#undef H2DLP_M
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_permute(const void* u1, int io, int64_t n_nodes, int nr, const int32_t* iperm, void* x,
                          double* x64, int prec, hipStream_t st) {
    const unsigned grid = unsigned((n_nodes + 255) / 256);
    if (io == 1) {
        if (prec == P_FP64)
            hipLaunchKernelGGL((k_permute<float, double>), dim3(grid), dim3(256), 0, st, static_cast<const float*>(u1),
                               n_nodes, nr, iperm, static_cast<double*>(x), nullptr);
        else
            hipLaunchKernelGGL((k_permute<float, float>), dim3(grid), dim3(256), 0, st, static_cast<const float*>(u1),
                               n_nodes, nr, iperm, static_cast<float*>(x), x64);
    } else {
        if (prec == P_FP64)
            hipLaunchKernelGGL((k_permute<double, double>), dim3(grid), dim3(256), 0, st, static_cast<const double*>(u1),
                               n_nodes, nr, iperm, static_cast<double*>(x), nullptr);
        else
            hipLaunchKernelGGL((k_permute<double, float>), dim3(grid), dim3(256), 0, st, static_cast<const double*>(u1),
                               n_nodes, nr, iperm, static_cast<float*>(x), x64);
    }
    return hipGetLastError();
}

hipError_t launch_unpermute(const double* y64, int io, int64_t n_nodes, int nr, const int32_t* iperm, void* u2,
                            hipStream_t st) {
    const unsigned grid = unsigned((n_nodes + 255) / 256);
    if (io == 1)
        hipLaunchKernelGGL((k_unpermute<float>), dim3(grid), dim3(256), 0, st, y64, n_nodes, nr, iperm,
                           static_cast<float*>(u2));
    else
        hipLaunchKernelGGL((k_unpermute<double>), dim3(grid), dim3(256), 0, st, y64, n_nodes, nr, iperm,
                           static_cast<double*>(u2));
    return hipGetLastError();
}

namespace {
template <typename T>
hipError_t leaf_regen_m(const VLeaf* leaves, unsigned n, const double* xyz, int m, const void* yh, double* y64,
                        hipStream_t st) {
    const T* y = static_cast<const T*>(yh);
    switch (m) {
#define H2DLP_REGEN_CASE(M_)                                                                                  \
    case M_:                                                                                                  \
        hipLaunchKernelGGL((k_leaf_regen<T, M_>), dim3(n), dim3(64), 0, st, leaves, xyz, y, y64);             \
        break;
        H2DLP_REGEN_CASE(1) H2DLP_REGEN_CASE(2) H2DLP_REGEN_CASE(3) H2DLP_REGEN_CASE(4)
        H2DLP_REGEN_CASE(5) H2DLP_REGEN_CASE(6) H2DLP_REGEN_CASE(7) H2DLP_REGEN_CASE(8)
#undef H2DLP_REGEN_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_leaf_regen(const VLeaf* leaves, int64_t n_leaves, const double* xyz, int m, const void* yh,
                             double* y64, int prec, hipStream_t st) {
    if (n_leaves == 0) return hipSuccess;
    if (prec == P_FP64) return leaf_regen_m<double>(leaves, unsigned(n_leaves), xyz, m, yh, y64, st);
    return leaf_regen_m<float>(leaves, unsigned(n_leaves), xyz, m, yh, y64, st);
}

hipError_t launch_product_store(const ProductArgs& a, int prec, bool prefer_rows, hipStream_t st) {
    const int rt = a.rt;
    int nrg, rtw;
    if (prefer_rows) {
        nrg = rt >= 4 ? 4 : pow2ceil(rt);
        rtw = pow2ceil((rt + nrg - 1) / nrg);
    } else {
        nrg = rt <= 8 ? 1 : (rt <= 16 ? 2 : 4);
        rtw = pow2ceil((rt + nrg - 1) / nrg);
    }
    if (rtw > 8) return hipErrorInvalidValue;
    if (prec == P_FP64) return dispatch<double, EPI_STORE>(a, nullptr, rtw, nrg, st);
    return dispatch<float, EPI_STORE>(a, nullptr, rtw, nrg, st);
}

hipError_t launch_coupling_generated(const ProductArgs& a, int m, int prec, size_t lds_floor, hipStream_t st) {
    if (m < 1 || m > 5 || (prec != P_FP32 && prec != P_FP64)) return hipErrorInvalidValue;
    const unsigned grid = a.n_items > 0 ? xcd_grid(a.n_items) : 0u;
    if (grid == 0) return hipSuccess;
    UnitNodes un{};
    for (int l = 0; l < m; ++l) un.o[l] = std::cos((2.0 * l + 1.0) * 3.14159265358979323846 / (2.0 * m));
    const int rt = (m * m * m + 15) / 16;
    // orders 4 and 5 split rows over waves (no LDS reduction); lower orders split blocks
    const size_t lds = std::max(m >= 4 ? size_t(0) : size_t(kWaves - 1) * rt * 256 * (prec == P_FP64 ? 8 : 4),
                                lds_floor);
#define H2DLP_GEN_LAUNCH(MM, ROWS)                                                                              \
    if (prec == P_FP64)                                                                                         \
        hipLaunchKernelGGL((k_coupling_gen<double, MM, ROWS>), dim3(grid), dim3(kThreads), lds, st, a, un);    \
    else                                                                                                        \
        hipLaunchKernelGGL((k_coupling_gen<float, MM, ROWS>), dim3(grid), dim3(kThreads), lds, st, a, un);
    switch (m) {
        case 1: H2DLP_GEN_LAUNCH(1, false) break;
        case 2: H2DLP_GEN_LAUNCH(2, false) break;
        case 3: H2DLP_GEN_LAUNCH(3, false) break;
        case 4: H2DLP_GEN_LAUNCH(4, true) break;
        case 5: H2DLP_GEN_LAUNCH(5, true) break;
        default: return hipErrorInvalidValue;
    }
#undef H2DLP_GEN_LAUNCH
    return hipGetLastError();
}

hipError_t launch_coupling(const ProductArgs& a, int k, int prec, hipStream_t st) {
    const int rt = (k + 15) / 16;
    if (prec == P_BF16X3 || prec == P_BF16X6) {
        const unsigned grid = a.n_items > 0 ? xcd_grid(a.n_items) : 0u;
        if (grid == 0) return hipSuccess;
        const size_t lds = size_t(kWaves - 1) * rt * 256 * sizeof(float);
#define H2DLP_SPLIT_CASE(R)                                                                                  \
    case R:                                                                                                  \
        if (prec == P_BF16X3)                                                                                \
            hipLaunchKernelGGL((k_coupling_bf16s<R, 2>), dim3(grid), dim3(kThreads), lds, st, a, k);         \
        else                                                                                                 \
            hipLaunchKernelGGL((k_coupling_bf16s<R, 3>), dim3(grid), dim3(kThreads), lds, st, a, k);         \
        break;
        switch (rt) {
            H2DLP_SPLIT_CASE(1)
            H2DLP_SPLIT_CASE(2)
            H2DLP_SPLIT_CASE(4)
            H2DLP_SPLIT_CASE(8)
            default: return hipErrorInvalidValue;
        }
#undef H2DLP_SPLIT_CASE
        return hipGetLastError();
    }
    if (rt > 8 || (rt & (rt - 1)) != 0) {   // large orders: generic product (blocks stored k x k)
        if (rt <= 8) return hipErrorInvalidValue;
        return launch_product_store(a, prec, false, st);
    }
    const unsigned grid = a.n_items > 0 ? xcd_grid(a.n_items) : 0u;
    if (grid == 0) return hipSuccess;
    const size_t lds = size_t(kWaves - 1) * rt * 256 * (prec == P_FP64 ? 8 : 4);
#define H2DLP_CPL(T_, RT_)                                                                              \
    if (rt == RT_) {                                                                                    \
        hipLaunchKernelGGL((k_coupling<T_, RT_>), dim3(grid), dim3(kThreads), lds, st, a, k);           \
        return hipGetLastError();                                                                       \
    }
    if (prec == P_FP64) {
        H2DLP_CPL(double, 1) H2DLP_CPL(double, 2) H2DLP_CPL(double, 4) H2DLP_CPL(double, 8)
    } else {
        H2DLP_CPL(float, 1) H2DLP_CPL(float, 2) H2DLP_CPL(float, 4) H2DLP_CPL(float, 8)
    }
#undef H2DLP_CPL
    return hipErrorInvalidValue;
}

hipError_t launch_product_add(const ProductArgs& a, int prec, bool prefer_rows, hipStream_t st) {
    const int rt = a.rt;
    int nrg, rtw;
    if (prefer_rows) {
        nrg = rt >= 4 ? 4 : pow2ceil(rt);
        rtw = pow2ceil((rt + nrg - 1) / nrg);
    } else {
        nrg = rt <= 8 ? 1 : (rt <= 16 ? 2 : 4);
        rtw = pow2ceil((rt + nrg - 1) / nrg);
    }
    if (rtw > 8) return hipErrorInvalidValue;
    if (prec == P_FP64) return dispatch<double, EPI_ADD>(a, nullptr, rtw, nrg, st);
    return dispatch<float, EPI_ADD>(a, nullptr, rtw, nrg, st);
}

hipError_t launch_product_add64(const ProductArgs& a, double* y64, int prec, hipStream_t st) {
    const int rt = a.rt;
    const int nrg = rt >= 4 ? 4 : pow2ceil(rt);       // one block per item: the waves split its rows
    const int rtw = pow2ceil((rt + nrg - 1) / nrg);
    if (rtw > 8) return hipErrorInvalidValue;
    if (prec == P_FP64) return dispatch<double, EPI_ADD64>(a, y64, rtw, nrg, st);
    return dispatch<float, EPI_ADD64>(a, y64, rtw, nrg, st);
}

hipError_t launch_product_near(const ProductArgs& a, double* y64, int prec, hipStream_t st) {
    const int rtw = pow2ceil(a.rt);
    if (rtw > 8) return hipErrorInvalidValue;
    if (prec == P_FP64) return dispatch<double, EPI_ADD64>(a, y64, rtw, 1, st);
    return dispatch<float, EPI_ADD64>(a, y64, rtw, 1, st);
}

hipError_t launch_diag_nearsing(const LeafEpilogue& e, int64_t n_pos, hipStream_t st) {
    if (n_pos <= 0) return hipSuccess;
    const int64_t blocks = (n_pos * 4 + 255) / 256;
    hipLaunchKernelGGL(k_diag_nearsing, dim3(unsigned(blocks)), dim3(256), 0, st, n_pos, e);
    return hipGetLastError();
}

hipError_t launch_upward(int32_t c_begin, int32_t c_end, const int32_t* child0, const int32_t* child1, const void* e,
                         void* xh, int m, int prec, hipStream_t st) {
    if (c_end <= c_begin) return hipSuccess;
    const unsigned grid = unsigned(c_end - c_begin);
    if (prec == P_FP64)
        return upward_m<double>(m, grid, st, c_begin, child0, child1, static_cast<const double*>(e), static_cast<double*>(xh));
    return upward_m<float>(m, grid, st, c_begin, child0, child1, static_cast<const float*>(e), static_cast<float*>(xh));
}

hipError_t launch_downward_paths(int32_t n_front, const int32_t* front, const int32_t* parent, const void* e, void* yh,
                                 int m, int prec, hipStream_t st) {
    if (n_front <= 0) return hipSuccess;
    const unsigned grid = unsigned(n_front);
    switch (m) {
#define H2DLP_M(MM_)                                                                                              \
    case MM_:                                                                                                     \
        if (prec == P_FP64)                                                                                       \
            hipLaunchKernelGGL((k_downward_paths<double, MM_>), dim3(grid), dim3(256), 0, st, front, parent,       \
                               static_cast<const double*>(e), static_cast<double*>(yh));                          \
        else                                                                                                      \
            hipLaunchKernelGGL((k_downward_paths<float, MM_>), dim3(grid), dim3(256), 0, st, front, parent,        \
                               static_cast<const float*>(e), static_cast<float*>(yh));                            \
        break;
        H2DLP_M(1) H2DLP_M(2) H2DLP_M(3) H2DLP_M(4) H2DLP_M(5) H2DLP_M(6) H2DLP_M(7) H2DLP_M(8)
#undef H2DLP_M
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_downward(int32_t c_begin, int32_t c_end, const int32_t* parent, const void* e, void* yh, int m,
                           int prec, hipStream_t st) {
    if (c_end <= c_begin) return hipSuccess;
    const unsigned grid = unsigned(c_end - c_begin);
    if (prec == P_FP64)
        return downward_m<double>(m, grid, st, c_begin, parent, static_cast<const double*>(e), static_cast<double*>(yh));
    return downward_m<float>(m, grid, st, c_begin, parent, static_cast<const float*>(e), static_cast<float*>(yh));
}

}  // namespace h2dlp
