// Algebraic recompression of the interpolation H2 matrix (recompress.h).
//
// Every step is a QR or an SVD of an explicit matrix in FP64, batched over the
// clusters of one level with rocSOLVER, the products between them batched
// with rocBLAS; nothing is squared, so singular values near the truncation
// threshold are resolved to rounding and the rank decisions are stable.
// Each cluster owns fixed slots: k x k (ld k) for R factors, weights L and
// projections P, rows x k (ld rows) for its stacked basis Y, its weighted
// basis X and the left singular vectors U.
//
// Rows (columns: W for V, V for W, S^T for S):
//   1. R'_s, from the leaves up: QR(W_s) at a leaf, QR([R'_c0 E_c0; R'_c1 E_c1]) above.
//   2. L_t, from the root down: condense [L_p^T E_t^T; R'_s1 S_ts1^T; R'_s2 S_ts2^T; ...]
//      by QR, three blocks per round on top of the previous R; L_t = R^T.
//   3. from the leaves up: Y_t = V_t (leaf) or [P_c0 E_c0; P_c1 E_c1], SVD of
//      Y_t L_t, rank r_t = #{sigma_i > eps sigma_1} (at most the rows of Y_t
//      that can be nonzero), P_t = U_r^T Y_t.
//   4. S'_ts = P_t S_ts P'_s^T.
#include "recompress.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.h"
#include "layout.h"

namespace h2dlp {

void RecompressResult::release() {
    for (double** p : {&u_row, &u_col, &p_row, &p_col}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    bytes = 0;
}

namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ inline void cheb_pts(const double* box, int axis, int m, double* p) {
    const double lo = box[axis], hi = box[3 + axis];
    const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
    for (int l = 0; l < m; ++l) p[l] = c + h * cos((2.0 * l + 1.0) * kPi / (2.0 * m));
}

__device__ inline double lag(const double* pts, int m, int l, double x) {
    double v = 1.0;
    for (int q = 0; q < m; ++q)
        if (q != l) v *= (x - pts[q]) / (pts[l] - pts[q]);
    return v;
}

// Dense transfer of every non-root cluster c with parent p, k x k column-major:
// E(nu', nu) = L^p_nu(eta^c_nu') = prod over the axes of the 1D Lagrange values.
__global__ void __launch_bounds__(256) k_dense_transfer(const double* __restrict__ boxes,
                                                       const int32_t* __restrict__ parent, int m,
                                                       double* __restrict__ E) {
    __shared__ double f[3][8][8];
    const int32_t c = blockIdx.x, p = parent[c];
    const int k = m * m * m;
    double* out = E + int64_t(c) * k * k;
    if (p < 0) {
        for (int e = threadIdx.x; e < k * k; e += blockDim.x) out[e] = 0.0;
        return;
    }
    if (int(threadIdx.x) < 3 * m * m) {
        const int axis = threadIdx.x / (m * m), lp = (threadIdx.x / m) % m, l = threadIdx.x % m;
        double pc[8], pp[8];
        cheb_pts(boxes + 6 * int64_t(c), axis, m, pc);
        cheb_pts(boxes + 6 * int64_t(p), axis, m, pp);
        f[axis][lp][l] = lag(pp, m, l, pc[lp]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int a = e % k, b = e / k;          // row nu' (child), column nu (parent)
        out[e] = f[0][a % m][b % m] * f[1][(a / m) % m][(b / m) % m] * f[2][a / (m * m)][b / (m * m)];
    }
}

// Coupling matrices of a list of blocks, k x k column-major each:
// S(nu, mu) = 1/(4 pi |eta^t_nu - eta^s_mu|).
__global__ void __launch_bounds__(256) k_coupling64(const double* __restrict__ boxes, int m,
                                                   const int32_t* __restrict__ bt, const int32_t* __restrict__ bs,
                                                   double* __restrict__ S) {
    __shared__ double pt[3][8], ps[3][8];
    const int b = blockIdx.x;
    if (threadIdx.x < 3) cheb_pts(boxes + 6 * int64_t(bt[b]), threadIdx.x, m, pt[threadIdx.x]);
    else if (threadIdx.x < 6) cheb_pts(boxes + 6 * int64_t(bs[b]), threadIdx.x - 3, m, ps[threadIdx.x - 3]);
    __syncthreads();
    const int k = m * m * m;
    double* out = S + int64_t(b) * k * k;
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int nu = e % k, mu = e / k;
        const double dx = pt[0][nu % m] - ps[0][mu % m];
        const double dy = pt[1][(nu / m) % m] - ps[1][(mu / m) % m];
        const double dz = pt[2][nu / (m * m)] - ps[2][mu / (m * m)];
        out[e] = 1.0 / (4.0 * kPi * sqrt(dx * dx + dy * dy + dz * dz));
    }
}

// dst = the upper triangle of the first k rows of src (rows x k, ld lda),
// zero below; transposed into dst when `transpose` (then lower triangular).
__global__ void __launch_bounds__(256) k_upper(double* const* __restrict__ src, int lda, int k,
                                              double* const* __restrict__ dst, int transpose) {
    const double* a = src[blockIdx.x];
    double* d = dst[blockIdx.x];
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int i = e % k, j = e / k;
        const double v = i <= j ? a[i + int64_t(lda) * j] : 0.0;
        if (transpose) d[j + int64_t(k) * i] = v;
        else d[e] = v;
    }
}

// In place: keep the upper triangle of the first k rows of a rows x k matrix, zero the rest.
__global__ void __launch_bounds__(256) k_keep_upper(double* const* __restrict__ A, int rows, int k) {
    double* a = A[blockIdx.x];
    for (int e = threadIdx.x; e < rows * k; e += blockDim.x) {
        const int i = e % rows, j = e / rows;
        if (i >= k || i > j) a[e] = 0.0;
    }
}

// Rows >= rank[g] of P_g (k x k, ld k) set to zero, for the gids [g0, g0 + gridDim.x).
__global__ void __launch_bounds__(256) k_mask_rows(double* __restrict__ P, const int32_t* __restrict__ rank, int k) {
    double* p = P + int64_t(blockIdx.x) * k * k;
    const int r = rank[blockIdx.x];
    for (int e = threadIdx.x; e < k * k; e += blockDim.x)
        if (e % k >= r) p[e] = 0.0;
}

__global__ void __launch_bounds__(256) k_store_layout(const StoreDesc* __restrict__ desc, int prec, void* pool) {
    const StoreDesc d = desc[blockIdx.x];
    for (int e = threadIdx.x; e < d.M * d.K; e += blockDim.x) {
        const int i = e % d.M, j = e / d.M;
        const double v = d.transpose ? d.src[j + int64_t(d.ld) * i] : d.src[i + int64_t(d.ld) * j];
        const int64_t o = d.a_off + a_offset(d.M, d.K, i, j);
        if (prec == P_FP64) static_cast<double*>(pool)[o] = v;
        else static_cast<float*>(pool)[o] = float(v);
    }
}

__global__ void __launch_bounds__(256) k_gather_leaf(const GatherDesc* __restrict__ desc, const double* __restrict__ pool,
                                                    int k, int rows, int transposed, double* __restrict__ out) {
    const GatherDesc d = desc[blockIdx.x];
    double* o = out + int64_t(d.gid) * rows * k;
    for (int e = threadIdx.x; e < d.n * k; e += blockDim.x) {
        const int i = e % d.n, nu = e / d.n;      // row i of the basis (node), column nu
        o[i + int64_t(rows) * nu] = transposed ? pool[d.a_off + a_offset(k, d.n, nu, i)]
                                               : pool[d.a_off + a_offset(d.n, k, i, nu)];
    }
}

// ---------------------------------------------------------------- host helpers

struct Ctx {
    hipStream_t st;
    rocblas_handle h = nullptr;
    std::string err;
    std::vector<void*> owned;
    ~Ctx() {
        for (void* p : owned) (void)hipFree(p);
        if (h) (void)rocblas_destroy_handle(h);
    }
    bool ok() const { return err.empty(); }
    bool hip(hipError_t e, const char* what) {
        if (e != hipSuccess && err.empty()) err = std::string(what) + ": " + hipGetErrorString(e);
        return e == hipSuccess;
    }
    bool blas(rocblas_status s, const char* what) {
        if (s != rocblas_status_success && err.empty())
            err = std::string(what) + " failed (rocBLAS/rocSOLVER status " + std::to_string(int(s)) + ")";
        return s == rocblas_status_success;
    }
    template <typename T>
    T* alloc(size_t n, bool keep = false) {
        void* p = nullptr;
        if (n == 0) n = 1;
        if (!hip(hipMalloc(&p, n * sizeof(T)), "device allocation")) return nullptr;
        if (!keep) owned.push_back(p);
        return static_cast<T*>(p);
    }
    // host array -> device (synchronised: the host vector may go out of scope)
    template <typename T>
    bool put(T* d, const std::vector<T>& v) {
        if (v.empty()) return true;
        return hip(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st), "upload") &&
               hip(hipStreamSynchronize(st), "upload");
    }
};

const double kOne = 1.0, kZero = 0.0;

// C_i = op(A_i) op(B_i) for pointer lists (square k x k operands unless stated)
bool gemm(Ctx& c, rocblas_operation ta, rocblas_operation tb, int m, int n, int kk, const std::vector<double*>& A,
          int lda, const std::vector<double*>& B, int ldb, const std::vector<double*>& C, int ldc, double** dptr) {
    const int nb = int(A.size());
    if (nb == 0) return true;
    std::vector<double*> all;
    all.reserve(3 * nb);
    all.insert(all.end(), A.begin(), A.end());
    all.insert(all.end(), B.begin(), B.end());
    all.insert(all.end(), C.begin(), C.end());
    if (!c.put(dptr, all)) return false;
    return c.blas(rocblas_dgemm_batched(c.h, ta, tb, m, n, kk, &kOne, dptr, lda, dptr + nb, ldb, &kZero, dptr + 2 * nb,
                                        ldc, nb),
                  "rocblas_dgemm_batched");
}

}  // namespace

hipError_t launch_store_layout(const StoreDesc* d_desc, int64_t n, int prec, void* pool, hipStream_t st) {
    for (int64_t b = 0; b < n; b += 65535) {
        const unsigned g = unsigned(std::min<int64_t>(65535, n - b));
        hipLaunchKernelGGL(k_store_layout, dim3(g), dim3(256), 0, st, d_desc + b, prec, pool);
    }
    return hipGetLastError();
}

hipError_t launch_gather_leaf_basis(const GatherDesc* d_desc, int64_t n_leaves, const double* pool, int k, int rows,
                                    bool transposed, double* out, hipStream_t st) {
    for (int64_t b = 0; b < n_leaves; b += 65535) {
        const unsigned g = unsigned(std::min<int64_t>(65535, n_leaves - b));
        hipLaunchKernelGGL(k_gather_leaf, dim3(g), dim3(256), 0, st, d_desc + b, pool, k, rows, int(transposed), out);
    }
    return hipGetLastError();
}

std::string recompress(const RecompressPlan& P, const double* d_boxes, const double* d_vleaf, const double* d_wleaf,
                       hipStream_t stream, RecompressResult* out) {
    Ctx c;
    c.st = stream;
    const int k = P.k, rows = P.rows, m = P.m;
    const int32_t C = P.n_clusters;
    const int64_t kk = int64_t(k) * k, rk = int64_t(rows) * k;
    if (k < 1 || k > 128 || rows < 2 * k) return "recompression needs k <= 128 and rows >= 2k";
    if (!c.blas(rocblas_create_handle(&c.h), "rocblas_create_handle") ||
        !c.blas(rocblas_set_stream(c.h, stream), "rocblas_set_stream"))
        return c.err;
    int32_t maxlev = 1;
    for (int l = 0; l <= P.depth; ++l) maxlev = std::max(maxlev, P.level_off[l + 1] - P.level_off[l]);
    const int32_t CH = std::min<int32_t>(maxlev, 4096);     // clusters per condensing chunk
    constexpr int kPerRound = 3;                            // blocks folded per QR round
    const int wr = (kPerRound + 1) * k;                     // rows of a condensing work matrix

    double* E = c.alloc<double>(size_t(C) * kk);
    double* Rv = c.alloc<double>(size_t(C) * kk);
    double* Rw = c.alloc<double>(size_t(C) * kk);
    double* Lr = c.alloc<double>(size_t(C) * kk);
    double* Lc = c.alloc<double>(size_t(C) * kk);
    double* Y = c.alloc<double>(size_t(maxlev) * rk);
    double* X = c.alloc<double>(size_t(maxlev) * rk);
    double* work = c.alloc<double>(size_t(CH) * wr * k);
    double* Sbuf = c.alloc<double>(size_t(CH) * kPerRound * kk);
    double* sig = c.alloc<double>(size_t(maxlev) * k);
    double* tau = c.alloc<double>(size_t(std::max(maxlev, CH)) * k);
    double* ework = c.alloc<double>(size_t(maxlev) * k);
    rocblas_int* info = c.alloc<rocblas_int>(size_t(std::max(maxlev, CH)));
    int32_t* d_rank = c.alloc<int32_t>(size_t(maxlev));
    int32_t* d_bt = c.alloc<int32_t>(size_t(CH) * kPerRound);
    int32_t* d_bs = c.alloc<int32_t>(size_t(CH) * kPerRound);
    double** dptr = c.alloc<double*>(size_t(3) * std::max(maxlev, CH * kPerRound));
    out->release();
    out->u_row = c.alloc<double>(size_t(C) * rk, true);
    out->u_col = c.alloc<double>(size_t(C) * rk, true);
    out->p_row = c.alloc<double>(size_t(C) * kk, true);
    out->p_col = c.alloc<double>(size_t(C) * kk, true);
    out->bytes = size_t(C) * (2 * rk + 2 * kk) * sizeof(double);
    if (!c.ok()) {
        out->release();
        return c.err;
    }
    int32_t* d_parent = c.alloc<int32_t>(size_t(C));
    if (!c.put(d_parent, P.parent)) {
        out->release();
        return c.err;
    }
    hipLaunchKernelGGL(k_dense_transfer, dim3(C), dim3(256), 0, stream, d_boxes, d_parent, m, E);
    c.hip(hipGetLastError(), "dense transfers");
    auto slot = [&](double* base, int32_t g, int64_t size) { return base + int64_t(g) * size; };
    const auto N = rocblas_operation_none, T = rocblas_operation_transpose;

    // stacked bases of the clusters of one level into Y (slot per level index):
    // leaves from `leaf` (whose slots of inner clusters are zero, so this also
    // clears them), inner clusters [A_c0 E_c0; A_c1 E_c1] from `coef`
    auto stack = [&](int32_t a, int32_t b, const double* leaf, double* coef) {
        c.hip(hipMemcpyAsync(Y, leaf + int64_t(a) * rk, size_t(b - a) * rk * sizeof(double), hipMemcpyDeviceToDevice,
                             stream), "stack leaves");
        std::vector<double*> A0, B0, C0, A1, B1, C1;
        for (int32_t g = a; g < b; ++g) {
            if (P.child0[g] < 0) continue;
            double* y = Y + int64_t(g - a) * rk;
            A0.push_back(slot(coef, P.child0[g], kk)); B0.push_back(slot(E, P.child0[g], kk)); C0.push_back(y);
            A1.push_back(slot(coef, P.child1[g], kk)); B1.push_back(slot(E, P.child1[g], kk)); C1.push_back(y + k);
        }
        gemm(c, N, N, k, k, k, A0, k, B0, k, C0, rows, dptr);
        gemm(c, N, N, k, k, k, A1, k, B1, k, C1, rows, dptr);
    };

    // 1. orthogonalisation factors of both interpolation bases, leaves up
    for (int side = 0; side < 2 && c.ok(); ++side) {
        const double* leaf = side == 0 ? d_vleaf : d_wleaf;
        double* R = side == 0 ? Rv : Rw;
        for (int l = P.depth; l >= 0 && c.ok(); --l) {
            const int32_t a = P.level_off[l], b = P.level_off[l + 1], n = b - a;
            stack(a, b, leaf, R);
            c.blas(rocsolver_dgeqrf_strided_batched(c.h, rows, k, Y, rows, rk, tau, k, n), "rocsolver_dgeqrf");
            std::vector<double> none;
            std::vector<double*> src(n), dst(n);
            for (int32_t q = 0; q < n; ++q) { src[q] = Y + int64_t(q) * rk; dst[q] = slot(R, a + q, kk); }
            std::vector<double*> both(src);
            both.insert(both.end(), dst.begin(), dst.end());
            if (!c.put(dptr, both)) break;
            hipLaunchKernelGGL(k_upper, dim3(n), dim3(256), 0, stream, dptr, rows, k, dptr + n, 0);
            c.hip(hipGetLastError(), "upper");
        }
    }

    // 2. weights, root down: condense [L_p^T E_t^T; blocks] three blocks per QR round
    std::vector<std::vector<int32_t>> served_row(C), served_col(C);
    for (size_t q = 0; q < P.far_t.size(); ++q) {
        served_row[P.far_t[q]].push_back(P.far_s[q]);
        served_col[P.far_s[q]].push_back(P.far_t[q]);
    }
    for (int side = 0; side < 2 && c.ok(); ++side) {
        const auto& served = side == 0 ? served_row : served_col;
        double* L = side == 0 ? Lr : Lc;
        double* Ro = side == 0 ? Rw : Rv;              // the other side's factors
        for (int l = 0; l <= P.depth && c.ok(); ++l) {
            for (int32_t a = P.level_off[l]; a < P.level_off[l + 1] && c.ok(); a += CH) {
                const int32_t b = std::min(P.level_off[l + 1], a + CH), n = b - a;
                c.hip(hipMemsetAsync(work, 0, size_t(n) * wr * k * sizeof(double), stream), "weights clear");
                {
                    std::vector<double*> A, B, Cc;
                    for (int32_t g = a; g < b; ++g)
                        if (P.parent[g] >= 0) {
                            A.push_back(slot(L, P.parent[g], kk));
                            B.push_back(slot(E, g, kk));
                            Cc.push_back(work + int64_t(g - a) * wr * k);
                        }
                    gemm(c, T, T, k, k, k, A, k, B, k, Cc, wr, dptr);     // L_p^T E_t^T
                }
                size_t most = 0;
                for (int32_t g = a; g < b; ++g) most = std::max(most, served[g].size());
                for (size_t j0 = 0; (j0 == 0 || j0 < most) && c.ok(); j0 += kPerRound) {
                    std::vector<int32_t> bt, bs;
                    std::vector<double*> A, B, Cc, part;
                    for (int32_t g = a; g < b; ++g) {
                        if (j0 > 0 && served[g].size() <= j0) continue;
                        double* w = work + int64_t(g - a) * wr * k;
                        part.push_back(w);
                        for (int q = 0; q < kPerRound && j0 + q < served[g].size(); ++q) {
                            const int32_t o = served[g][j0 + q];
                            const size_t idx = bt.size();
                            bt.push_back(side == 0 ? g : o);
                            bs.push_back(side == 0 ? o : g);
                            A.push_back(slot(Ro, o, kk));
                            B.push_back(Sbuf + int64_t(idx) * kk);
                            Cc.push_back(w + (q + 1) * k);
                        }
                    }
                    if (!bt.empty()) {
                        if (!c.put(d_bt, bt) || !c.put(d_bs, bs)) break;
                        hipLaunchKernelGGL(k_coupling64, dim3(unsigned(bt.size())), dim3(256), 0, stream, d_boxes, m,
                                           d_bt, d_bs, Sbuf);
                        c.hip(hipGetLastError(), "coupling");
                        // rows: R'_s S_ts^T;  columns: R_t S_ts
                        gemm(c, N, side == 0 ? T : N, k, k, k, A, k, B, k, Cc, wr, dptr);
                    }
                    if (!c.put(dptr, part)) break;
                    c.blas(rocsolver_dgeqrf_batched(c.h, wr, k, dptr, wr, tau, k, int(part.size())), "rocsolver_dgeqrf");
                    hipLaunchKernelGGL(k_keep_upper, dim3(unsigned(part.size())), dim3(256), 0, stream, dptr, wr, k);
                    c.hip(hipGetLastError(), "keep upper");
                }
                std::vector<double*> both;
                for (int32_t g = a; g < b; ++g) both.push_back(work + int64_t(g - a) * wr * k);
                for (int32_t g = a; g < b; ++g) both.push_back(slot(L, g, kk));
                if (!c.put(dptr, both)) break;
                hipLaunchKernelGGL(k_upper, dim3(n), dim3(256), 0, stream, dptr, wr, k, dptr + n, 1);   // L = R^T
                c.hip(hipGetLastError(), "weights");
            }
        }
    }

    // 3. truncation, leaves up
    out->rank_row.assign(C, 0);
    out->rank_col.assign(C, 0);
    std::vector<double> hsig;
    for (int side = 0; side < 2 && c.ok(); ++side) {
        const double* leaf = side == 0 ? d_vleaf : d_wleaf;
        double* L = side == 0 ? Lr : Lc;
        double* U = side == 0 ? out->u_row : out->u_col;
        double* Pm = side == 0 ? out->p_row : out->p_col;
        std::vector<int32_t>& rank = side == 0 ? out->rank_row : out->rank_col;
        for (int l = P.depth; l >= 0 && c.ok(); --l) {
            const int32_t a = P.level_off[l], b = P.level_off[l + 1], n = b - a;
            stack(a, b, leaf, Pm);
            c.blas(rocblas_dgemm_strided_batched(c.h, N, N, rows, k, k, &kOne, Y, rows, rk, slot(L, a, kk), k, kk,
                                                 &kZero, X, rows, rk, n),
                   "rocblas_dgemm_strided_batched");
            c.blas(rocsolver_dgesvd_strided_batched(c.h, rocblas_svect_singular, rocblas_svect_none, rows, k, X, rows,
                                                    rk, sig, k, slot(U, a, rk), rows, rk, nullptr, 1, 0, ework, k,
                                                    rocblas_outofplace, info, n),
                   "rocsolver_dgesvd");
            hsig.resize(size_t(n) * k);
            if (!c.hip(hipMemcpyAsync(hsig.data(), sig, hsig.size() * sizeof(double), hipMemcpyDeviceToHost, stream),
                       "singular values") ||
                !c.hip(hipStreamSynchronize(stream), "singular values"))
                break;
            std::vector<int32_t> rl(n);
            for (int32_t q = 0; q < n; ++q) {
                const int32_t g = a + q;
                // at most the rows of Y_t that can be nonzero (a thin SVD has no more)
                const int cap = P.child0[g] < 0 ? std::min(P.leaf_n[g], k)
                                                : std::min(rank[P.child0[g]] + rank[P.child1[g]], k);
                const double* s = hsig.data() + size_t(q) * k;
                int r = 0;
                if (s[0] > 0.0)
                    while (r < cap && s[r] > P.eps * s[0]) ++r;
                rl[q] = r;
                rank[g] = r;
            }
            if (!c.put(d_rank, rl)) break;
            // P_t = U^T Y_t (all k columns of U), then rows >= r_t cleared
            c.blas(rocblas_dgemm_strided_batched(c.h, T, N, k, k, rows, &kOne, slot(U, a, rk), rows, rk, Y, rows, rk,
                                                 &kZero, slot(Pm, a, kk), k, kk, n),
                   "rocblas_dgemm_strided_batched");
            hipLaunchKernelGGL(k_mask_rows, dim3(n), dim3(256), 0, stream, slot(Pm, a, kk), d_rank, k);
            c.hip(hipGetLastError(), "mask");
        }
    }
    if (c.ok()) c.hip(hipStreamSynchronize(stream), "recompression");
    if (!c.ok()) out->release();
    return c.err;
}

std::string recompress_couplings(const RecompressPlan& P, const double* d_boxes, const RecompressResult& res,
                                 const std::vector<int64_t>& a_off, int prec, void* pool, hipStream_t stream) {
    Ctx c;
    c.st = stream;
    const int k = P.k;
    const int64_t kk = int64_t(k) * k;
    if (!c.blas(rocblas_create_handle(&c.h), "rocblas_create_handle") ||
        !c.blas(rocblas_set_stream(c.h, stream), "rocblas_set_stream"))
        return c.err;
    const int64_t nb_all = int64_t(P.far_t.size());
    const int64_t BATCH = std::min<int64_t>(std::max<int64_t>(nb_all, 1), 8192);
    double* S = c.alloc<double>(size_t(BATCH) * kk);
    double* Tm = c.alloc<double>(size_t(BATCH) * kk);
    double* Sp = c.alloc<double>(size_t(BATCH) * kk);
    int32_t* d_bt = c.alloc<int32_t>(size_t(BATCH));
    int32_t* d_bs = c.alloc<int32_t>(size_t(BATCH));
    double** dptr = c.alloc<double*>(size_t(3) * BATCH);
    StoreDesc* d_desc = c.alloc<StoreDesc>(size_t(BATCH));
    const auto N = rocblas_operation_none, T = rocblas_operation_transpose;
    for (int64_t b0 = 0; b0 < nb_all && c.ok(); b0 += BATCH) {
        const int64_t n = std::min(BATCH, nb_all - b0);
        std::vector<int32_t> bt(P.far_t.begin() + b0, P.far_t.begin() + b0 + n);
        std::vector<int32_t> bs(P.far_s.begin() + b0, P.far_s.begin() + b0 + n);
        if (!c.put(d_bt, bt) || !c.put(d_bs, bs)) break;
        hipLaunchKernelGGL(k_coupling64, dim3(unsigned(n)), dim3(256), 0, stream, d_boxes, P.m, d_bt, d_bs, S);
        c.hip(hipGetLastError(), "coupling");
        std::vector<double*> A, B, Cc;
        for (int64_t q = 0; q < n; ++q) {                       // T = S P'_s^T
            A.push_back(S + q * kk);
            B.push_back(res.p_col + int64_t(bs[q]) * kk);
            Cc.push_back(Tm + q * kk);
        }
        gemm(c, N, T, k, k, k, A, k, B, k, Cc, k, dptr);
        A.clear(); B.clear(); Cc.clear();
        for (int64_t q = 0; q < n; ++q) {                       // S' = P_t T
            A.push_back(res.p_row + int64_t(bt[q]) * kk);
            B.push_back(Tm + q * kk);
            Cc.push_back(Sp + q * kk);
        }
        gemm(c, N, N, k, k, k, A, k, B, k, Cc, k, dptr);
        std::vector<StoreDesc> desc(n);
        for (int64_t q = 0; q < n; ++q)
            desc[q] = StoreDesc{Sp + q * kk, k, res.rank_row[bt[q]], res.rank_col[bs[q]], 0, a_off[b0 + q]};
        if (!c.put(d_desc, desc)) break;
        c.hip(launch_store_layout(d_desc, n, prec, pool, stream), "store couplings");
        c.hip(hipStreamSynchronize(stream), "couplings");
    }
    return c.err;
}

}  // namespace h2dlp
