// Algebraic recompression of the interpolation H2 matrix (recompress.h).
//
// Every step is a QR or an SVD of an explicit matrix in FP64, batched over the
// clusters of one level; nothing is squared, so singular values near the
// truncation threshold are resolved to rounding and the rank decisions are
// stable.  The QR factors come from k_fold (Householder folding of row
// chunks into an R kept in LDS, one workgroup per matrix), the SVDs from
// k_jacobi (one-sided Jacobi on a k x k matrix in LDS), the products between
// them from rocBLAS.  Each cluster owns fixed slots: k x k (ld k) for R
// factors, weights L and projections P, rows x k (ld rows) for its stacked
// basis Y and its left singular vectors U.
//
// Rows (columns: W for V, V for W, S^T for S):
//   1. R'_s, from the leaves up: QR(W_s) at a leaf, QR([R'_c0 E_c0; R'_c1 E_c1]) above.
//   2. L_t, from the root down: condense [L_p^T E_t^T; R'_s1 S_ts1^T; R'_s2 S_ts2^T; ...]
//      by QR, nine blocks per round on top of the previous R; L_t = R^T.
//   3. from the leaves up: Y_t = V_t (leaf) or [P_c0 E_c0; P_c1 E_c1]; with
//      Y_t = Q R_Y, the singular values and right singular vectors Z of
//      Y_t L_t are those of R_Y L_t; rank r_t = #{sigma_i > eps sigma_1} (at
//      most the rows of Y_t that can be nonzero); left singular vectors
//      U_r = Y_t L_t Z_r / sigma_r; P_t = U_r^T Y_t.
//   4. S'_ts = P_t S_ts P'_s^T.
#include "recompress.h"

#include <rocblas/rocblas.h>

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

// ---------------------------------------------------------------- QR by folding

// Rows to fold into one R: up to kFoldSeg segments [begin, begin + n) of the
// rows of a column-major source (ld), folded in order.
constexpr int kFoldSeg = 10;
constexpr int kFoldChunk = 64;              // rows folded per Householder sweep (one wavefront's lanes)
struct FoldDesc {
    double* R;                              // k x k column-major, upper triangle: in (first init rows) and out
    const double* src;
    int32_t ld, init, nseg, pad;            // init: rows of R filled on entry (0: R starts at zero)
    int32_t seg_begin[kFoldSeg], seg_n[kFoldSeg];
};

// R(i, j), j >= i, in the packed upper triangle of a k x k R (row-major rows
// of k - i entries)
__device__ inline int packed(int i, int j, int k) { return i * k - (i * (i - 1)) / 2 + (j - i); }

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// R := R factor of [R; the descriptor's rows] by Householder reflections,
// kFoldChunk rows at a time, in the order of an unblocked QR of the stacked
// rows: with p rows of R filled (init on entry, 0 = start from zero), the
// reflection for column j < p mixes R(j, :) with the chunk's rows, and for
// p <= j < p + nrow the chunk's next row becomes R(j, :) first (it is zero
// left of j by then) and the reflection mixes it with the chunk rows after
// it.  R therefore holds its content in its first min(rows folded, k) rows,
// also when the rows are rank-deficient (an unpivoted reflection from a zero
// pivot would spread content into later rows).  A reflection touches only
// R(j, :) and the chunk (R is triangular), so both stay in LDS; R(j, j) keeps
// the sign the reflection gives.  R is kept as its packed upper triangle, so
// that LDS holds a chunk of 64 rows beside it.  kFoldTpc threads per column
// apply a reflection (kFoldChunk / kFoldTpc chunk rows each); the workgroup
// is kFoldThreads wide, since its LDS admits one per CU anyway.
constexpr int kFoldThreads = 1024;
constexpr int kFoldTpc = 8;
static_assert(kFoldThreads / kFoldTpc >= 128, "one thread group per column of k <= 128");
static_assert(kFoldChunk <= 64 && kFoldChunk % kFoldTpc == 0, "the first wavefront sums a chunk column");
__global__ void __launch_bounds__(kFoldThreads) k_fold(const FoldDesc* __restrict__ desc, int k) {
    extern __shared__ double sm[];
    double* Rs = sm;                        // packed upper triangle of R, k (k + 1) / 2
    double* Cs = Rs + k * (k + 1) / 2;      // kFoldChunk x k row-major
    double* us = Cs + kFoldChunk * k;       // the reflection's chunk part
    __shared__ double s_tau;
    const FoldDesc& d = desc[blockIdx.x];       // read in place: its segment arrays are indexed at run time
    const int tid = threadIdx.x;
    int filled = min(max(d.init, 0), k);
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int i = e / k, j = e % k;
        if (i <= j) Rs[packed(i, j, k)] = i < filled ? d.R[i + int64_t(k) * j] : 0.0;
    }
    int total = 0;
    for (int q = 0; q < d.nseg; ++q) total += d.seg_n[q];
    for (int c0 = 0; c0 < total; c0 += kFoldChunk) {
        const int nrow = min(kFoldChunk, total - c0);
        __syncthreads();
        for (int e = tid; e < kFoldChunk * k; e += blockDim.x) {
            const int i = e % kFoldChunk, l = e / kFoldChunk;
            double v = 0.0;
            if (i < nrow) {
                int r = c0 + i, q = 0;
                while (r >= d.seg_n[q]) r -= d.seg_n[q++];
                v = d.src[int64_t(d.seg_begin[q] + r) + int64_t(d.ld) * l];
            }
            Cs[i * k + l] = v;
        }
        __syncthreads();
        for (int j = 0; j < k; ++j) {
            // chunk row moved into R(j, :) at this column (-1: none); the
            // chunk rows before it were moved earlier and take no part
            const int mv = (j >= filled && j - filled < nrow) ? j - filled : -1;
            const int first = j >= filled ? j - filled + 1 : 0;
            if (tid < 64) {
                const double cj = (tid < nrow && tid >= first) ? Cs[tid * k + j] : 0.0;
                const double s2 = wave_sum(cj * cj);
                const double a = mv >= 0 ? Cs[mv * k + j] : Rs[packed(j, j, k)];
                double tau = 0.0, scale = 0.0, diag = a;
                if (s2 > 0.0) {
                    const double nrm = sqrt(a * a + s2);
                    const double beta = a > 0.0 ? -nrm : nrm;
                    tau = (beta - a) / beta;
                    scale = 1.0 / (a - beta);
                    diag = beta;
                }
                if (tid < kFoldChunk) us[tid] = cj * scale;
                if (tid == 0) {
                    s_tau = tau;
                    Rs[packed(j, j, k)] = diag;
                }
            }
            __syncthreads();
            const double tau = s_tau;
            const int l = j + 1 + tid / kFoldTpc, h = tid % kFoldTpc;
            if (l < k && (tau != 0.0 || mv >= 0)) {
                const double r0 = mv >= 0 ? Cs[mv * k + l] : Rs[packed(j, l, k)];
                double w = 0.0;
                if (tau != 0.0) {
                    constexpr int H = kFoldChunk / kFoldTpc;
#pragma unroll
                    for (int i = 0; i < H; ++i) w += us[h * H + i] * Cs[(h * H + i) * k + l];
                    for (int o = 1; o < kFoldTpc; o <<= 1) w += __shfl_xor(w, o);
                    w = tau * (w + r0);
#pragma unroll
                    for (int i = 0; i < H; ++i) Cs[(h * H + i) * k + l] -= w * us[h * H + i];
                }
                if (h == 0) Rs[packed(j, l, k)] = r0 - w;
            }
            __syncthreads();
        }
        filled = min(filled + nrow, k);
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int i = e % k, j = e / k;
        d.R[e] = i <= j ? Rs[packed(i, j, k)] : 0.0;
    }
}

// ---------------------------------------------------------------- SVD by one-sided Jacobi

// Singular values and right singular vectors of a k x k matrix M (column-
// major, ld k): one-sided Jacobi rotations of the columns of A = M^T until
// they are orthogonal (A J = W); then the normalised columns of W are the
// right singular vectors of M and their norms the singular values.  Only the
// columns of A that hold a nonzero (the rows of M that can be nonzero: the
// rows folded into R_Y, at most min(rows of Y, k)) take part; the others are
// zero and stay so.  Pairs of those nz columns follow the circle method
// (n - 1 steps of n/2 disjoint pairs per sweep, n = nz rounded up to even,
// the spare column k standing in as the zero one); tpp threads share a pair,
// as many as the kJacThreads of the workgroup allow (its LDS admits one per
// CU).  Output: sigma descending, V with the matching columns (zero for
// sigma = 0).
constexpr int kJacThreads = 1024;
__global__ void __launch_bounds__(kJacThreads) k_jacobi(double* const* __restrict__ Ms, int k,
                                                       double* __restrict__ sig, double* __restrict__ V) {
    extern __shared__ double sm[];
    const int na = k + 1;                   // columns in LDS: A's k and a spare zero one
    double* A = sm;                         // column c at A + c k
    double* nrm = A + int64_t(na) * k;      // na
    int* idx = reinterpret_cast<int*>(nrm + na);    // na: the columns that take part, then the spare
    __shared__ int s_rot, s_nz;
    const double* M = Ms[blockIdx.x];
    const int tid = threadIdx.x;
    for (int e = tid; e < na * k; e += blockDim.x) {
        const int c = e / k, r = e % k;     // A(r, c) = M(c, r)
        A[e] = c < k ? M[c + int64_t(k) * r] : 0.0;
    }
    __syncthreads();
    for (int c = tid; c < k; c += blockDim.x) {
        bool any = false;
        for (int r = 0; r < k && !any; ++r) any = A[int64_t(c) * k + r] != 0.0;
        nrm[c] = any ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        int nz = 0;
        for (int c = 0; c < k; ++c)
            if (nrm[c] != 0.0) idx[nz++] = c;
        idx[nz] = k;                        // the spare zero column, used when nz is odd
        s_nz = nz;
    }
    __syncthreads();
    const int n = (s_nz + 1) & ~1;
    int tpp = 32;                           // threads per pair: a power of two, (n / 2) tpp <= kJacThreads
    while (tpp > 1 && (n / 2) * tpp > kJacThreads) tpp >>= 1;
    const int p = tid / tpp, q = tid % tpp;
    for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int step = 0; step < n - 1; ++step) {
            if (p < n / 2) {
                const int a = p == 0 ? step : (step + p) % (n - 1);
                const int b = p == 0 ? n - 1 : (step - p + (n - 1)) % (n - 1);
                double* ca = A + int64_t(idx[a]) * k;
                double* cb = A + int64_t(idx[b]) * k;
                double aa = 0.0, bb = 0.0, ab = 0.0;
                for (int r = q; r < k; r += tpp) {
                    const double x = ca[r], y = cb[r];
                    aa += x * x;
                    bb += y * y;
                    ab += x * y;
                }
                for (int o = 1; o < tpp; o <<= 1) {
                    aa += __shfl_xor(aa, o);
                    bb += __shfl_xor(bb, o);
                    ab += __shfl_xor(ab, o);
                }
                if (ab != 0.0 && fabs(ab) > 4e-15 * sqrt(aa * bb)) {
                    const double zeta = (bb - aa) / (2.0 * ab);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                    for (int r = q; r < k; r += tpp) {
                        const double x = ca[r], y = cb[r];
                        ca[r] = cs * x - sn * y;
                        cb[r] = sn * x + cs * y;
                    }
                    if (q == 0) s_rot = 1;
                }
            }
            __syncthreads();
        }
        const int rotated = s_rot;
        __syncthreads();                    // every thread has read s_rot before it is reset
        if (!rotated) break;
    }
    for (int c = tid; c < k; c += blockDim.x) {
        double s2 = 0.0;
        for (int r = 0; r < k; ++r) s2 += A[int64_t(c) * k + r] * A[int64_t(c) * k + r];
        nrm[c] = sqrt(s2);
    }
    __syncthreads();
    double* so = sig + int64_t(blockIdx.x) * k;
    double* vo = V + int64_t(blockIdx.x) * k * k;
    for (int c = tid; c < k; c += blockDim.x) {
        int pos = 0;                        // descending, ties by column
        for (int o = 0; o < k; ++o) pos += nrm[o] > nrm[c] || (nrm[o] == nrm[c] && o < c);
        so[pos] = nrm[c];
        const double inv = nrm[c] > 0.0 ? 1.0 / nrm[c] : 0.0;
        for (int r = 0; r < k; ++r) vo[r + int64_t(k) * pos] = A[int64_t(c) * k + r] * inv;
    }
}

// Columns i < rank of V scaled by 1/sigma_i, the others zero (per matrix, k x k).
__global__ void __launch_bounds__(256) k_scale_cols(double* __restrict__ V, const double* __restrict__ sig,
                                                   const int32_t* __restrict__ rank, int k) {
    double* v = V + int64_t(blockIdx.x) * k * k;
    const double* s = sig + int64_t(blockIdx.x) * k;
    const int r = rank[blockIdx.x];
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int c = e / k;
        v[e] = c < r ? v[e] / s[c] : 0.0;
    }
}

// Z = (3 I - G) / 2 in place (k x k per matrix): one Newton-Schulz step
// towards the orthogonal polar factor, U Z for U with U^T U = G ~ I.
__global__ void __launch_bounds__(256) k_newton_schulz(double* __restrict__ G, int k) {
    double* g = G + int64_t(blockIdx.x) * k * k;
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) g[e] = (e % k == e / k ? 1.5 : 0.0) - 0.5 * g[e];
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
    const size_t lds_fold = sizeof(double) * (size_t(k) * (k + 1) / 2 + size_t(kFoldChunk) * k + kFoldChunk);
    const size_t lds_jac = sizeof(double) * (size_t(k + 1) * k + (k + 1)) + sizeof(int) * size_t(k + 1);
    {
        int dev = 0, lds = 0;
        if (!c.hip(hipGetDevice(&dev), "device") ||
            !c.hip(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "attribute"))
            return c.err;
        if (size_t(lds) < std::max(lds_fold, lds_jac))
            return "recompression needs " + std::to_string(std::max(lds_fold, lds_jac)) +
                   " bytes of LDS per workgroup, the device has " + std::to_string(lds);
        // dynamic LDS beyond 64 KB is granted to a kernel only up to its declared maximum
        if (!c.hip(hipFuncSetAttribute(reinterpret_cast<const void*>(k_fold),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_fold)), "fold LDS") ||
            !c.hip(hipFuncSetAttribute(reinterpret_cast<const void*>(k_jacobi),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_jac)), "jacobi LDS"))
            return c.err;
    }
    if (!c.blas(rocblas_create_handle(&c.h), "rocblas_create_handle") ||
        !c.blas(rocblas_set_stream(c.h, stream), "rocblas_set_stream"))
        return c.err;
    int32_t maxlev = 1;
    for (int l = 0; l <= P.depth; ++l) maxlev = std::max(maxlev, P.level_off[l + 1] - P.level_off[l]);
    const int32_t CH = std::min<int32_t>(maxlev, 4096);     // clusters per weight chunk
    constexpr int kPerRound = kFoldSeg - 1;                 // blocks folded per round, after the parent part
    const int wr = (kPerRound + 1) * k;                     // rows of a round buffer

    double* E = c.alloc<double>(size_t(C) * kk);
    double* Rv = c.alloc<double>(size_t(C) * kk);
    double* Rw = c.alloc<double>(size_t(C) * kk);
    double* Lr = c.alloc<double>(size_t(C) * kk);
    double* Lc = c.alloc<double>(size_t(C) * kk);
    double* Y = c.alloc<double>(size_t(maxlev) * rk);
    double* Ut = c.alloc<double>(size_t(maxlev) * rk);
    double* Ry = c.alloc<double>(size_t(maxlev) * kk);
    double* Mx = c.alloc<double>(size_t(maxlev) * kk);
    double* Vz = c.alloc<double>(size_t(maxlev) * kk);
    double* Cm = c.alloc<double>(size_t(maxlev) * kk);
    double* sig = c.alloc<double>(size_t(maxlev) * k);
    double* work = c.alloc<double>(size_t(CH) * wr * k);
    double* Racc = c.alloc<double>(size_t(CH) * kk);
    double* Sbuf = c.alloc<double>(size_t(CH) * kPerRound * kk);
    int32_t* d_rank = c.alloc<int32_t>(size_t(maxlev));
    int32_t* d_bt = c.alloc<int32_t>(size_t(CH) * kPerRound);
    int32_t* d_bs = c.alloc<int32_t>(size_t(CH) * kPerRound);
    double** dptr = c.alloc<double*>(size_t(3) * std::max(maxlev, CH * kPerRound));
    FoldDesc* d_fold = c.alloc<FoldDesc>(size_t(std::max(maxlev, CH)));
    out->release();
    out->u_row = c.alloc<double>(size_t(C) * rk, true);
    out->u_col = c.alloc<double>(size_t(C) * rk, true);
    out->p_row = c.alloc<double>(size_t(C) * kk, true);
    out->p_col = c.alloc<double>(size_t(C) * kk, true);
    out->bytes = size_t(C) * (2 * rk + 2 * kk) * sizeof(double);
    int32_t* d_parent = c.alloc<int32_t>(size_t(C));
    if (!c.ok() || !c.put(d_parent, P.parent)) {
        out->release();
        return c.err;
    }
    hipLaunchKernelGGL(k_dense_transfer, dim3(C), dim3(256), 0, stream, d_boxes, d_parent, m, E);
    c.hip(hipGetLastError(), "dense transfers");
    auto slot = [&](double* base, int32_t g, int64_t size) { return base + int64_t(g) * size; };
    const auto N = rocblas_operation_none, T = rocblas_operation_transpose;
    auto fold = [&](const std::vector<FoldDesc>& d) {
        if (d.empty() || !c.put(d_fold, d)) return;
        hipLaunchKernelGGL(k_fold, dim3(unsigned(d.size())), dim3(kFoldThreads), lds_fold, stream, d_fold, k);
        c.hip(hipGetLastError(), "fold");
    };

    // stacked bases of the clusters of one level into Y (slot per level index):
    // leaves from `leaf` (whose slots of inner clusters are zero, so this also
    // clears them), inner clusters [A_c0 E_c0; A_c1 E_c1] from `coef`, the
    // second child's rows from row k
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
    // fold descriptor of a stacked Y: a leaf's rows, or the two children's parts
    auto y_desc = [&](int32_t g, int32_t a, double* R, const std::vector<int32_t>& nrow) {
        FoldDesc d{};
        d.R = R;
        d.src = Y + int64_t(g - a) * rk;
        d.ld = rows;
        if (P.child0[g] < 0) {
            d.nseg = 1;
            d.seg_n[0] = P.leaf_n[g];
        } else {
            d.nseg = 2;
            d.seg_n[0] = nrow[P.child0[g]];
            d.seg_begin[1] = k;
            d.seg_n[1] = nrow[P.child1[g]];
        }
        return d;
    };

    // 1. R factors of both interpolation bases, leaves up (nr: rows of each R)
    std::vector<int32_t> nr_v(C, 0), nr_w(C, 0);
    for (int side = 0; side < 2 && c.ok(); ++side) {
        const double* leaf = side == 0 ? d_vleaf : d_wleaf;
        double* R = side == 0 ? Rv : Rw;
        std::vector<int32_t>& nr = side == 0 ? nr_v : nr_w;
        for (int l = P.depth; l >= 0 && c.ok(); --l) {
            const int32_t a = P.level_off[l], b = P.level_off[l + 1];
            stack(a, b, leaf, R);
            std::vector<FoldDesc> d;
            for (int32_t g = a; g < b; ++g) {
                d.push_back(y_desc(g, a, slot(R, g, kk), nr));
                int tot = 0;
                for (int q = 0; q < d.back().nseg; ++q) tot += d.back().seg_n[q];
                nr[g] = std::min(tot, k);
            }
            fold(d);
        }
    }

    // 2. weights, root down: fold [L_p^T E_t^T; R_s S_ts^T; ...], kPerRound blocks a round
    std::vector<std::vector<int32_t>> served_row(C), served_col(C);
    for (size_t q = 0; q < P.far_t.size(); ++q) {
        served_row[P.far_t[q]].push_back(P.far_s[q]);
        served_col[P.far_s[q]].push_back(P.far_t[q]);
    }
    for (int side = 0; side < 2 && c.ok(); ++side) {
        const auto& served = side == 0 ? served_row : served_col;
        double* L = side == 0 ? Lr : Lc;
        double* Ro = side == 0 ? Rw : Rv;               // the other side's factors
        const std::vector<int32_t>& nro = side == 0 ? nr_w : nr_v;
        std::vector<int32_t> nl(C, 0);                  // nonzero columns of each L
        for (int l = 0; l <= P.depth && c.ok(); ++l) {
            for (int32_t a = P.level_off[l]; a < P.level_off[l + 1] && c.ok(); a += CH) {
                const int32_t b = std::min(P.level_off[l + 1], a + CH);
                std::vector<int32_t> tot(b - a, 0);
                {
                    std::vector<double*> A, B, Cc;
                    for (int32_t g = a; g < b; ++g)
                        if (P.parent[g] >= 0 && nl[P.parent[g]] > 0) {
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
                    std::vector<double*> A, B, Cc;
                    std::vector<FoldDesc> d;
                    for (int32_t g = a; g < b; ++g) {
                        if (j0 > 0 && served[g].size() <= j0) continue;
                        double* w = work + int64_t(g - a) * wr * k;
                        FoldDesc f{};
                        f.R = Racc + int64_t(g - a) * kk;
                        f.src = w;
                        f.ld = wr;
                        f.init = j0 > 0 ? std::min(tot[g - a], k) : 0;
                        if (j0 == 0 && P.parent[g] >= 0 && nl[P.parent[g]] > 0) {
                            f.seg_n[f.nseg++] = nl[P.parent[g]];
                        }
                        for (int q = 0; q < kPerRound && j0 + q < served[g].size(); ++q) {
                            const int32_t o = served[g][j0 + q];
                            const size_t idx = bt.size();
                            bt.push_back(side == 0 ? g : o);
                            bs.push_back(side == 0 ? o : g);
                            A.push_back(slot(Ro, o, kk));
                            B.push_back(Sbuf + int64_t(idx) * kk);
                            Cc.push_back(w + (q + 1) * k);
                            f.seg_begin[f.nseg] = (q + 1) * k;
                            f.seg_n[f.nseg++] = nro[o];
                        }
                        for (int q = 0; q < f.nseg; ++q) tot[g - a] += f.seg_n[q];
                        d.push_back(f);
                    }
                    if (!bt.empty()) {
                        if (!c.put(d_bt, bt) || !c.put(d_bs, bs)) break;
                        hipLaunchKernelGGL(k_coupling64, dim3(unsigned(bt.size())), dim3(256), 0, stream, d_boxes, m,
                                           d_bt, d_bs, Sbuf);
                        c.hip(hipGetLastError(), "coupling");
                        // rows: R_s S_ts^T;  columns: R_t S_ts
                        gemm(c, N, side == 0 ? T : N, k, k, k, A, k, B, k, Cc, wr, dptr);
                    }
                    fold(d);
                }
                std::vector<double*> both;
                for (int32_t g = a; g < b; ++g) both.push_back(Racc + int64_t(g - a) * kk);
                for (int32_t g = a; g < b; ++g) both.push_back(slot(L, g, kk));
                if (!c.put(dptr, both)) break;
                hipLaunchKernelGGL(k_upper, dim3(unsigned(b - a)), dim3(256), 0, stream, dptr, k, k, dptr + (b - a),
                                   1);                                  // L = R^T
                c.hip(hipGetLastError(), "weights");
                for (int32_t g = a; g < b; ++g) nl[g] = std::min(tot[g - a], k);
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
            std::vector<FoldDesc> d;
            for (int32_t g = a; g < b; ++g) d.push_back(y_desc(g, a, Ry + int64_t(g - a) * kk, rank));
            fold(d);                                                     // Y = Q R_Y
            c.blas(rocblas_dgemm_strided_batched(c.h, N, N, k, k, k, &kOne, Ry, k, kk, slot(L, a, kk), k, kk, &kZero,
                                                 Mx, k, kk, n),
                   "rocblas_dgemm_strided_batched");                     // R_Y L
            std::vector<double*> mp(n);
            for (int32_t q = 0; q < n; ++q) mp[q] = Mx + int64_t(q) * kk;
            if (!c.put(dptr, mp)) break;
            hipLaunchKernelGGL(k_jacobi, dim3(n), dim3(kJacThreads), lds_jac, stream, dptr, k, sig, Vz);
            c.hip(hipGetLastError(), "jacobi");
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
                const double* sv = hsig.data() + size_t(q) * k;
                int r = 0;
                if (sv[0] > 0.0)
                    while (r < cap && sv[r] > P.eps * sv[0]) ++r;
                rl[q] = r;
                rank[g] = r;
            }
            if (!c.put(d_rank, rl)) break;
            hipLaunchKernelGGL(k_scale_cols, dim3(n), dim3(256), 0, stream, Vz, sig, d_rank, k);   // Z_r / sigma_r
            c.hip(hipGetLastError(), "scale");
            c.blas(rocblas_dgemm_strided_batched(c.h, N, N, k, k, k, &kOne, slot(L, a, kk), k, kk, Vz, k, kk, &kZero,
                                                 Cm, k, kk, n),
                   "rocblas_dgemm_strided_batched");                     // C = L Z_r / sigma_r
            c.blas(rocblas_dgemm_strided_batched(c.h, N, N, rows, k, k, &kOne, Y, rows, rk, Cm, k, kk, &kZero,
                                                 slot(U, a, rk), rows, rk, n),
                   "rocblas_dgemm_strided_batched");                     // U_r = Y C
            // Y L Z_r / sigma_r spans the leading left singular subspace to
            // rounding, but its columns mix within it by up to eps_mach times
            // sigma_1^2 / sigma_r^2; two Newton-Schulz steps make them
            // orthonormal without changing the span (the product depends on
            // the span only)
            for (int it = 0; it < 2 && c.ok(); ++it) {
                double* src = it == 0 ? slot(U, a, rk) : Ut;
                double* dst = it == 0 ? Ut : slot(U, a, rk);
                c.blas(rocblas_dgemm_strided_batched(c.h, T, N, k, k, rows, &kOne, src, rows, rk, src, rows, rk, &kZero,
                                                     Cm, k, kk, n),
                       "rocblas_dgemm_strided_batched");                 // G = U^T U
                hipLaunchKernelGGL(k_newton_schulz, dim3(n), dim3(256), 0, stream, Cm, k);
                c.hip(hipGetLastError(), "newton-schulz");
                c.blas(rocblas_dgemm_strided_batched(c.h, N, N, rows, k, k, &kOne, src, rows, rk, Cm, k, kk, &kZero,
                                                     dst, rows, rk, n),
                       "rocblas_dgemm_strided_batched");                 // U (3 I - G) / 2
            }
            c.blas(rocblas_dgemm_strided_batched(c.h, T, N, k, k, rows, &kOne, slot(U, a, rk), rows, rk, Y, rows, rk,
                                                 &kZero, slot(Pm, a, kk), k, kk, n),
                   "rocblas_dgemm_strided_batched");                     // P = U_r^T Y
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
