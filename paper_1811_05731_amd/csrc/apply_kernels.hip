// Apply kernels: u2 = (K_H2 + D) u1, 16 right-hand sides per pass.
//
//   permute      x = P u1 (node order -> cluster order), cast to the operator precision
//   product      grouped block products Y_item = sum_b A_b X_b on MFMA 16x16x4
//                (FP32 or FP64), used three times:
//                  leaf forward   xhat_s = W_s^T x|_s                     (one block per leaf)
//                  coupling       yhat_t = sum_{s admissible} S_ts xhat_s  (one item per cluster)
//                  leaf output    y|_t = V_t yhat_t + sum_{s near} K_ts x|_s, then
//                                 u2 = y + D x (+ FP64 near-singular part), scattered
//   upward       xhat_t = sum_c E_c^T xhat_c     (Kronecker mode products, per level)
//   downward     yhat_c += E_c yhat_parent        (per level)
//
// The product kernel owns every output row it writes (no atomics): a
// workgroup of 4 waves takes one item, the waves split its blocks (or its row
// tiles), and partial sums meet in LDS in a fixed order, so results are
// bitwise reproducible.  A blocks are streamed straight from HBM into MFMA
// operand registers (layout.h); X rows come through L2.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace h2dlp {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kUnroll = 4;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// A operand: lane l holds A[l % 16][l / 16]; B operand: B[l / 16][l % 16].
// The 16 x 16 result comes back as 4 values per lane, column l % 16; the row
// of value v in lane group g = l / 16 differs by type: 4 g + v for f32, g + 4 v
// for f64 (measured on gfx950, pinned by the GPU parity tests).
template <>
struct Mfma<float> {
    typedef f32x4 acc;
    static __device__ inline acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Mfma<double> {
    typedef f64x4 acc;
    static __device__ inline acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int g, int v) { return g + 4 * v; }
};

// Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous
// range of items (neighbouring clusters share sources in its L2).
__device__ inline int xcd_item(int n_items) {
    const int per = gridDim.x >> 3;
    const int item = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    return item < n_items ? item : -1;
}

enum { EPI_STORE = 0, EPI_LEAF = 1 };

// Accumulate sum_b A_b X_b of one item into acc[RTW] (row tiles rg*RTW ...).
// Inside a full k-step the chunk of row tile rt starts at 64 rt and lane l
// reads entry kk*rv + i (= l for a full tile); each lane keeps that 32-bit
// offset per row tile, so a load is uniform base + lane offset.  Lanes outside
// a partial tile read entry 0 of the chunk and discard it; tiles past the
// item's rows multiply zeros (branch-free MFMA issue).
template <typename T>
__device__ inline T ld(const unsigned char* base, unsigned byte_off) {
    return *reinterpret_cast<const T*>(base + byte_off);   // SGPR base + 32-bit VGPR offset
}

template <typename T, int RTW>
__device__ inline void accumulate(const ItemDesc& it, const BlkDesc* __restrict__ blks, const T* __restrict__ pool,
                                  const T* __restrict__ x0, const T* __restrict__ x1, int rg, int bg, int nbg,
                                  typename Mfma<T>::acc* acc) {
    constexpr unsigned E = sizeof(T);
    const unsigned lane = threadIdx.x & 63;
    const unsigned i = lane & 15, kk = lane >> 4;
    const int M = it.m;
    const int RT = (M + 15) >> 4;
    unsigned off[RTW];   // byte offset of this lane's entry of row tile r inside a full k-step
    bool ok[RTW];
#pragma unroll
    for (int r = 0; r < RTW; ++r) {
        const int rt = rg * RTW + r;
        const unsigned rv = unsigned(M - 16 * rt < 16 ? M - 16 * rt : 16);
        ok[r] = rt < RT && i < rv;
        off[r] = ok[r] ? E * (64u * rt + kk * rv + i) : 0u;
    }
    const unsigned xoff = E * lane;
    for (int b = it.blk_begin + bg; b < it.blk_end; b += nbg) {
        const BlkDesc d = blks[b];
        const unsigned char* Ak = reinterpret_cast<const unsigned char*>(pool + d.a_off);
        const unsigned char* Xk = reinterpret_cast<const unsigned char*>(
            ((d.src & SRC1) ? x1 : x0) + int64_t(d.src & 0x7fffffff) * RHS_TILE);
        const int K = d.k;
        const int ksfull = K >> 2;
        const unsigned step = E * 4u * unsigned(M);   // bytes per full k-step
        int ks = 0;
        for (; ks + kUnroll <= ksfull; ks += kUnroll) {
            T bv[kUnroll];
            T av[kUnroll][RTW];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) bv[u] = ld<T>(Xk + E * 64u * u, xoff);
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const unsigned char* Au = Ak + step * u;
#pragma unroll
                for (int r = 0; r < RTW; ++r) {
                    const T v = ld<T>(Au, off[r]);
                    av[u][r] = ok[r] ? v : T(0);
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int r = 0; r < RTW; ++r) acc[r] = Mfma<T>::mma(av[u][r], bv[u], acc[r]);
            Ak += step * kUnroll;
            Xk += E * 64u * kUnroll;
        }
        const int ks_end = (K + 3) >> 2;
        for (; ks < ks_end; ++ks) {
            const unsigned kv = unsigned(K - 4 * ks < 4 ? K - 4 * ks : 4);
            const T bl = ld<T>(Xk, kk < kv ? xoff : 0u);
            const T bv = kk < kv ? bl : T(0);
#pragma unroll
            for (int r = 0; r < RTW; ++r) {
                const int rt = rg * RTW + r;
                const unsigned rv = unsigned(M - 16 * rt < 16 ? M - 16 * rt : 16);
                const bool valid = rt < RT && i < rv && kk < kv;
                const T al = ld<T>(Ak, valid ? E * (16u * rt * kv + kk * rv + i) : 0u);
                acc[r] = Mfma<T>::mma(valid ? al : T(0), bv, acc[r]);
            }
            Ak += step;
            Xk += E * 64u;
        }
    }
}

template <typename IO>
__device__ inline double io_load(const void* p, int64_t i) { return double(static_cast<const IO*>(p)[i]); }

template <typename T, int RTW, int NRG, int EPI>
__global__ void __launch_bounds__(kThreads) k_product(ProductArgs a, LeafEpilogue epi) {
    typedef typename Mfma<T>::acc acc_t;
    constexpr int NBG = kWaves / NRG;
    extern __shared__ unsigned char smem_raw[];
    T* red = reinterpret_cast<T*>(smem_raw);

    const int item = xcd_item(a.n_items);
    if (item < 0) return;
    const ItemDesc it = a.items[item];
    // the wave index is uniform per wave: keep block descriptors and base pointers in SGPRs
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int rg = w % NRG, bg = w / NRG;

    acc_t acc[RTW];
#pragma unroll
    for (int r = 0; r < RTW; ++r) acc[r] = acc_t{0, 0, 0, 0};
    accumulate<T, RTW>(it, a.blks, static_cast<const T*>(a.pool), static_cast<const T*>(a.x0),
                       static_cast<const T*>(a.x1), rg, bg, NBG, acc);

    if (NBG > 1) {   // fixed-order reduction of the block groups
        if (bg > 0) {
            T* slot = red + ((bg - 1) * NRG + rg) * RTW * 256;
#pragma unroll
            for (int r = 0; r < RTW; ++r)
#pragma unroll
                for (int v = 0; v < 4; ++v) slot[(r * 4 + v) * 64 + lane] = acc[r][v];
        }
        __syncthreads();
        if (bg > 0) return;
        for (int g = 1; g < NBG; ++g) {
            const T* slot = red + ((g - 1) * NRG + rg) * RTW * 256;
#pragma unroll
            for (int r = 0; r < RTW; ++r)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[r][v] += slot[(r * 4 + v) * 64 + lane];
        }
    }

    const int M = it.m;
    const int q = lane & 15;
#pragma unroll
    for (int r = 0; r < RTW; ++r) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * (rg * RTW + r) + Mfma<T>::row(lane >> 4, v);
            if (row >= M) continue;
            if (EPI == EPI_STORE) {
                static_cast<T*>(a.y)[(int64_t(it.out_row) + row) * RHS_TILE + q] = acc[r][v];
            } else {
                if (q >= epi.nr) continue;
                const int64_t pos = int64_t(it.out_row) + row;
                const int64_t node = epi.perm[pos];
                const int64_t base = int64_t(q) * epi.n_nodes;
                const bool f32 = epi.io == 1;
                double y = double(acc[r][v]);
                y += epi.diag[pos] * (f32 ? io_load<float>(epi.u1, base + node) : io_load<double>(epi.u1, base + node));
                if (epi.ns_off != nullptr) {
                    double s = 0.0;
                    for (int64_t e = epi.ns_off[pos]; e < epi.ns_off[pos + 1]; ++e) {
                        const int64_t c = epi.ns_col[e];
                        s += epi.ns_val[e] * (f32 ? io_load<float>(epi.u1, base + c) : io_load<double>(epi.u1, base + c));
                    }
                    y += s;
                }
                if (f32) static_cast<float*>(epi.u2)[base + node] = float(y);
                else static_cast<double*>(epi.u2)[base + node] = y;
            }
        }
    }
}

template <typename IO, typename T>
__global__ void __launch_bounds__(256) k_permute(const IO* __restrict__ u1, int64_t n, int nr,
                                                 const int32_t* __restrict__ perm, T* __restrict__ x) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n * RHS_TILE) return;
    const int64_t p = g >> 4;
    const int q = int(g & 15);
    x[g] = q < nr ? T(u1[int64_t(q) * n + perm[p]]) : T(0);
}

// Mode products of the Kronecker transfer E = Ex (x) Ey (x) Ez on one cluster's
// k x QC slab (index nu = lx + m ly + m^2 lz, columns innermost).
//   TRANS: out[l] = sum_l' E[l'][l] in[l']  (E^T, upward)   else  out[l'] = sum_l E[l'][l] in[l]
template <typename T, bool TRANS>
__device__ inline void mode_product(const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ e, int m,
                                    int axis, int qc) {
    const int k = m * m * m;
    const int stride = axis == 0 ? 1 : (axis == 1 ? m : m * m);
    for (int idx = threadIdx.x; idx < k * qc; idx += blockDim.x) {
        const int nu = idx / qc, q = idx % qc;
        const int l = (nu / stride) % m;
        const int base = nu - l * stride;
        T s = 0;
        for (int p = 0; p < m; ++p) {
            const T ev = TRANS ? e[p * m + l] : e[l * m + p];
            s += ev * in[(base + p * stride) * qc + q];
        }
        out[idx] = s;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_upward(int32_t c_begin, const int32_t* __restrict__ child0,
                                                const int32_t* __restrict__ child1, const T* __restrict__ efac,
                                                T* __restrict__ xh, int m, int qc) {
    extern __shared__ unsigned char smem_raw[];
    T* s = reinterpret_cast<T*>(smem_raw);
    const int k = m * m * m;
    const int32_t c = c_begin + blockIdx.x;
    const int32_t ch[2] = {child0[c], child1[c]};
    if (ch[0] < 0) return;   // leaf: its xhat comes from the leaf forward
    T* e = s;                             // 2 children x 3 axes x m x m
    T* b0 = s + 6 * 64;
    T* b1 = b0 + k * qc;
    T* acc = b1 + k * qc;
    for (int idx = threadIdx.x; idx < 6 * m * m; idx += blockDim.x) {
        const int which = idx / (3 * m * m);
        e[which * 3 * 64 + (idx % (3 * m * m)) / (m * m) * 64 + idx % (m * m)] =
            efac[int64_t(ch[which]) * 3 * m * m + idx % (3 * m * m)];
    }
    for (int q0 = 0; q0 < RHS_TILE; q0 += qc) {
        for (int idx = threadIdx.x; idx < k * qc; idx += blockDim.x) acc[idx] = 0;
        for (int w = 0; w < 2; ++w) {
            __syncthreads();
            const T* src = xh + int64_t(ch[w]) * k * RHS_TILE;
            for (int idx = threadIdx.x; idx < k * qc; idx += blockDim.x)
                b0[idx] = src[(idx / qc) * RHS_TILE + q0 + idx % qc];
            __syncthreads();
            mode_product<T, true>(b0, b1, e + w * 3 * 64 + 2 * 64, m, 2, qc);
            __syncthreads();
            mode_product<T, true>(b1, b0, e + w * 3 * 64 + 1 * 64, m, 1, qc);
            __syncthreads();
            mode_product<T, true>(b0, b1, e + w * 3 * 64 + 0 * 64, m, 0, qc);
            __syncthreads();
            for (int idx = threadIdx.x; idx < k * qc; idx += blockDim.x) acc[idx] += b1[idx];
        }
        __syncthreads();
        T* dst = xh + int64_t(c) * k * RHS_TILE;
        for (int idx = threadIdx.x; idx < k * qc; idx += blockDim.x) dst[(idx / qc) * RHS_TILE + q0 + idx % qc] = acc[idx];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_downward(int32_t c_begin, const int32_t* __restrict__ parent,
                                                  const T* __restrict__ efac, T* __restrict__ yh, int m, int qc) {
    extern __shared__ unsigned char smem_raw[];
    T* s = reinterpret_cast<T*>(smem_raw);
    const int k = m * m * m;
    const int32_t c = c_begin + blockIdx.x;
    const int32_t p = parent[c];
    if (p < 0) return;
    T* e = s;
    T* b0 = s + 3 * 64;
    T* b1 = b0 + k * qc;
    for (int idx = threadIdx.x; idx < 3 * m * m; idx += blockDim.x)
        e[(idx / (m * m)) * 64 + idx % (m * m)] = efac[int64_t(c) * 3 * m * m + idx];
    for (int q0 = 0; q0 < RHS_TILE; q0 += qc) {
        __syncthreads();
        const T* src = yh + int64_t(p) * k * RHS_TILE;
        for (int idx = threadIdx.x; idx < k * qc; idx += blockDim.x) b0[idx] = src[(idx / qc) * RHS_TILE + q0 + idx % qc];
        __syncthreads();
        mode_product<T, false>(b0, b1, e + 2 * 64, m, 2, qc);
        __syncthreads();
        mode_product<T, false>(b1, b0, e + 1 * 64, m, 1, qc);
        __syncthreads();
        mode_product<T, false>(b0, b1, e + 0 * 64, m, 0, qc);
        __syncthreads();
        T* dst = yh + int64_t(c) * k * RHS_TILE;
        for (int idx = threadIdx.x; idx < k * qc; idx += blockDim.x) dst[(idx / qc) * RHS_TILE + q0 + idx % qc] += b1[idx];
    }
}

inline int pow2ceil(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

template <typename T, int EPI>
hipError_t dispatch(const ProductArgs& a, const LeafEpilogue& e, int rtw, int nrg, hipStream_t st) {
    const unsigned grid = unsigned(8 * ((a.n_items + 7) / 8));
    if (grid == 0) return hipSuccess;
    const int nbg = kWaves / nrg;
    const size_t lds = size_t(nbg - 1) * nrg * rtw * 256 * sizeof(T);
#define H2DLP_CASE(RTW_, NRG_)                                                                       \
    if (rtw == RTW_ && nrg == NRG_) {                                                                \
        hipLaunchKernelGGL((k_product<T, RTW_, NRG_, EPI>), dim3(grid), dim3(kThreads), lds, st, a, e); \
        return hipGetLastError();                                                                    \
    }
    H2DLP_CASE(1, 1) H2DLP_CASE(2, 1) H2DLP_CASE(4, 1) H2DLP_CASE(8, 1)
    if (EPI == EPI_STORE) {
        H2DLP_CASE(1, 2) H2DLP_CASE(2, 2) H2DLP_CASE(4, 2) H2DLP_CASE(8, 2)
        H2DLP_CASE(1, 4) H2DLP_CASE(2, 4) H2DLP_CASE(4, 4) H2DLP_CASE(8, 4)
    }
#undef H2DLP_CASE
    return hipErrorInvalidValue;
}

inline int transfer_qc(int k, size_t elem, int buffers) {
    int qc = RHS_TILE;
    while (qc > 1 && size_t(buffers) * k * qc * elem > 48 * 1024) qc >>= 1;
    return qc;
}

}  // namespace

hipError_t launch_permute(const void* u1, int io, int64_t n_nodes, int nr, const int32_t* perm, void* x, int prec,
                          hipStream_t st) {
    const unsigned grid = unsigned((n_nodes * RHS_TILE + 255) / 256);
    if (io == 1) {
        if (prec == P_FP64)
            hipLaunchKernelGGL((k_permute<float, double>), dim3(grid), dim3(256), 0, st, static_cast<const float*>(u1), n_nodes, nr, perm, static_cast<double*>(x));
        else
            hipLaunchKernelGGL((k_permute<float, float>), dim3(grid), dim3(256), 0, st, static_cast<const float*>(u1), n_nodes, nr, perm, static_cast<float*>(x));
    } else {
        if (prec == P_FP64)
            hipLaunchKernelGGL((k_permute<double, double>), dim3(grid), dim3(256), 0, st, static_cast<const double*>(u1), n_nodes, nr, perm, static_cast<double*>(x));
        else
            hipLaunchKernelGGL((k_permute<double, float>), dim3(grid), dim3(256), 0, st, static_cast<const double*>(u1), n_nodes, nr, perm, static_cast<float*>(x));
    }
    return hipGetLastError();
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
    LeafEpilogue none{};
    if (prec == P_FP64) return dispatch<double, EPI_STORE>(a, none, rtw, nrg, st);
    return dispatch<float, EPI_STORE>(a, none, rtw, nrg, st);
}

hipError_t launch_product_leaf(const ProductArgs& a, const LeafEpilogue& e, int prec, hipStream_t st) {
    const int rtw = pow2ceil(a.rt);
    if (rtw > 8) return hipErrorInvalidValue;
    if (prec == P_FP64) return dispatch<double, EPI_LEAF>(a, e, rtw, 1, st);
    return dispatch<float, EPI_LEAF>(a, e, rtw, 1, st);
}

hipError_t launch_upward(int32_t c_begin, int32_t c_end, const int32_t* child0, const int32_t* child1, const void* e,
                         void* xh, int m, int prec, hipStream_t st) {
    if (c_end <= c_begin) return hipSuccess;
    const int k = m * m * m;
    if (prec == P_FP64) {
        const int qc = transfer_qc(k, sizeof(double), 3);
        const size_t lds = (6 * 64 + 3 * size_t(k) * qc) * sizeof(double);
        hipLaunchKernelGGL(k_upward<double>, dim3(unsigned(c_end - c_begin)), dim3(256), lds, st, c_begin, child0,
                           child1, static_cast<const double*>(e), static_cast<double*>(xh), m, qc);
    } else {
        const int qc = transfer_qc(k, sizeof(float), 3);
        const size_t lds = (6 * 64 + 3 * size_t(k) * qc) * sizeof(float);
        hipLaunchKernelGGL(k_upward<float>, dim3(unsigned(c_end - c_begin)), dim3(256), lds, st, c_begin, child0,
                           child1, static_cast<const float*>(e), static_cast<float*>(xh), m, qc);
    }
    return hipGetLastError();
}

hipError_t launch_downward(int32_t c_begin, int32_t c_end, const int32_t* parent, const void* e, void* yh, int m,
                           int prec, hipStream_t st) {
    if (c_end <= c_begin) return hipSuccess;
    const int k = m * m * m;
    if (prec == P_FP64) {
        const int qc = transfer_qc(k, sizeof(double), 2);
        const size_t lds = (3 * 64 + 2 * size_t(k) * qc) * sizeof(double);
        hipLaunchKernelGGL(k_downward<double>, dim3(unsigned(c_end - c_begin)), dim3(256), lds, st, c_begin, parent,
                           static_cast<const double*>(e), static_cast<double*>(yh), m, qc);
    } else {
        const int qc = transfer_qc(k, sizeof(float), 2);
        const size_t lds = (3 * 64 + 2 * size_t(k) * qc) * sizeof(float);
        hipLaunchKernelGGL(k_downward<float>, dim3(unsigned(c_end - c_begin)), dim3(256), lds, st, c_begin, parent,
                           static_cast<const float*>(e), static_cast<float*>(yh), m, qc);
    }
    return hipGetLastError();
}

}  // namespace h2dlp
