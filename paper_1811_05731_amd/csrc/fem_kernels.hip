// Kernels of the finite-element solves either side of the boundary operator
// (Section 2: u1 from the Poisson-Neumann problem, u2 from the Laplace-
// Dirichlet problem with the boundary operator's values, H = -grad u).
// P1 elements on tetrahedra, FP64 throughout.  Every sum has a fixed order:
// matrix entries and right sides are gathered per node over its incident
// tetrahedra, and every reduction goes through per-block partials that each
// consumer sums in the same order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fem.h"

namespace h2dlp {

namespace {

constexpr int kT = 256;

__device__ inline double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kT / 64; ++q) s += sh[q];
    __syncthreads();
    return s;                               // valid in thread 0
}

// sum of the first n partials, the same order in every block
__device__ inline double sum_partials(const double* __restrict__ part, int n, double* sh) {
    double v = 0.0;
    for (int q = threadIdx.x; q < n; q += kT) v += part[q];
    double s = block_sum(v, sh);
    if (threadIdx.x == 0) sh[kT / 64] = s;
    __syncthreads();
    s = sh[kT / 64];
    __syncthreads();
    return s;
}

// geo[t] = {vol, grad phi_0 (3), ..., grad phi_3 (3)}: with J = [x1-x0, x2-x0,
// x3-x0], the gradients of the barycentric coordinates of vertices 1..3 are
// the rows of J^-1, vertex 0's is minus their sum; vol = |det J| / 6
__global__ void __launch_bounds__(kT) k_geometry(int64_t n_tets, const double* __restrict__ xyz,
                                                const int32_t* __restrict__ tet, double* __restrict__ geo) {
    const int64_t t = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (t >= n_tets) return;
    double x[4][3];
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) x[a][d] = xyz[3 * int64_t(tet[4 * t + a]) + d];
    double J[3][3];                          // J[d][c] = (x_{c+1} - x_0)_d
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) J[d][c] = x[c + 1][d] - x[0][d];
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double inv = 1.0 / det;
    double Ji[3][3];                         // J^-1 = adj(J) / det
    Ji[0][0] = c00 * inv;
    Ji[1][0] = c01 * inv;
    Ji[2][0] = c02 * inv;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * inv;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * inv;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * inv;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * inv;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * inv;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * inv;
    double* g = geo + kGeo * t;
    g[0] = fabs(det) / 6.0;
    for (int d = 0; d < 3; ++d) {
        g[1 + d] = -(Ji[0][d] + Ji[1][d] + Ji[2][d]);
        for (int c = 0; c < 3; ++c) g[1 + 3 * (c + 1) + d] = Ji[c][d];
    }
}

// A_ij = sum over the tetrahedra at node i of vol grad phi_i . grad phi_j,
// one thread per row; the column of node j is found in the row's sorted list
__global__ void __launch_bounds__(kT) k_stiffness(int64_t n, const int64_t* __restrict__ inc_off,
                                                 const int32_t* __restrict__ inc, const int32_t* __restrict__ tet,
                                                 const double* __restrict__ geo, const int64_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col, double* __restrict__ val) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    const int64_t r0 = rowptr[i], r1 = rowptr[i + 1];
    for (int64_t k = r0; k < r1; ++k) val[k] = 0.0;
    for (int64_t e = inc_off[i]; e < inc_off[i + 1]; ++e) {
        const int64_t t = inc[e] >> 2;
        const int a = inc[e] & 3;
        const double* g = geo + kGeo * t;
        const double vol = g[0];
        for (int b = 0; b < 4; ++b) {
            const int32_t j = tet[4 * t + b];
            const double v = vol * (g[1 + 3 * a] * g[1 + 3 * b] + g[2 + 3 * a] * g[2 + 3 * b] +
                                    g[3 + 3 * a] * g[3 + 3 * b]);
            int64_t lo = r0, hi = r1 - 1;    // binary search: columns are sorted
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] < j) lo = mid + 1;
                else hi = mid;
            }
            val[lo] += v;
        }
    }
}

// b_i = sum over the tetrahedra at node i of vol M_t . grad phi_i
__global__ void __launch_bounds__(kT) k_rhs(int64_t n, const int64_t* __restrict__ inc_off,
                                           const int32_t* __restrict__ inc, const double* __restrict__ geo,
                                           const double* __restrict__ m, double* __restrict__ b) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t e = inc_off[i]; e < inc_off[i + 1]; ++e) {
        const int64_t t = inc[e] >> 2;
        const int a = inc[e] & 3;
        const double* g = geo + kGeo * t;
        s += g[0] * (m[3 * t] * g[1 + 3 * a] + m[3 * t + 1] * g[2 + 3 * a] + m[3 * t + 2] * g[3 + 3 * a]);
    }
    b[i] = s;
}

// q = A p, one thread per row over its slice's slots (all loads of a slot are
// contiguous across the wavefront and independent of each other), with the
// block partial of p . q
__global__ void __launch_bounds__(kT) k_spmv_dot(int64_t n, const int64_t* __restrict__ off,
                                                const int32_t* __restrict__ width, const int32_t* __restrict__ col,
                                                const double* __restrict__ val, const double* __restrict__ p,
                                                double* __restrict__ q, double* __restrict__ part) {
    __shared__ double sh[kT / 64 + 1];
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i - threadIdx.x < n; i += int64_t(gridDim.x) * kT) {
        if (i < n) {
            const int64_t sl = i / kSlice;
            const int64_t base = off[sl] + (i - sl * kSlice);
            const int w = width[sl];
            double s = 0.0;
#pragma unroll 4
            for (int k = 0; k < w; ++k) s += val[base + int64_t(kSlice) * k] * p[col[base + int64_t(kSlice) * k]];
            q[i] = s;
            acc += p[i] * s;
        }
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// ELL values from the CSR ones (row i's k-th entry into slot k; the rest of
// the row's slots hold 0 at its own column)
__global__ void __launch_bounds__(kT) k_to_ell(int64_t n, const int64_t* __restrict__ rowptr,
                                              const double* __restrict__ val, const int64_t* __restrict__ off,
                                              const int32_t* __restrict__ width, double* __restrict__ ell) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    const int64_t sl = i / kSlice;
    const int64_t base = off[sl] + (i - sl * kSlice);
    const int64_t r0 = rowptr[i], len = rowptr[i + 1] - r0;
    for (int k = 0; k < width[sl]; ++k) ell[base + int64_t(kSlice) * k] = k < len ? val[r0 + k] : 0.0;
}

// partials of a . b
__global__ void __launch_bounds__(kT) k_dot(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                                           double* __restrict__ part) {
    __shared__ double sh[kT / 64 + 1];
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kT) acc += a[i] * b[i];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// S[slot] = sum of the partials (one block)
__global__ void __launch_bounds__(kT) k_finish(const double* __restrict__ part, int n, double* __restrict__ S,
                                              int slot, double scale) {
    __shared__ double sh[kT / 64 + 1];
    const double s = sum_partials(part, n, sh);
    if (threadIdx.x == 0) S[slot] = scale * s;
}

// x -= S[slot] (a mean removed: S holds sum / n)
__global__ void __launch_bounds__(kT) k_shift(int64_t n, double* __restrict__ x, const double* __restrict__ S, int slot) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i < n) x[i] -= S[slot];
}

// Start of preconditioned CG from x = 0: r = mask(b), z = dinv r, p = z; the
// partials of r . z and r . r
__global__ void __launch_bounds__(kT) k_cg_start(int64_t n, const double* __restrict__ b,
                                                const double* __restrict__ dinv, double inv_theta,
                                                double* __restrict__ x, double* __restrict__ r, double* __restrict__ z,
                                                double* __restrict__ p, double* __restrict__ dk,
                                                double* __restrict__ part_rz, double* __restrict__ part_rr) {
    __shared__ double sh[kT / 64 + 1];
    double rz = 0.0, rr = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kT) {
        const double ri = dinv[i] != 0.0 ? b[i] : 0.0;
        const double zi = inv_theta * (dinv[i] * ri);
        x[i] = 0.0;
        r[i] = ri;
        z[i] = zi;
        p[i] = zi;
        if (dk) dk[i] = zi;
        rz += ri * zi;
        rr += ri * ri;
    }
    double t = block_sum(rz, sh);
    if (threadIdx.x == 0) part_rz[blockIdx.x] = t;
    t = block_sum(rr, sh);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = t;
}

// alpha = rz / (p . q) from the matrix-vector product's partials; x += alpha
// p, r -= alpha q (zero where fixed), z = inv_theta dinv r (and d = z for the
// Chebyshev steps that follow); partials of the new r . z and r . r
__global__ void __launch_bounds__(kT) k_cg_update(int64_t n, int nb, const double* __restrict__ part_pq,
                                                 const double* __restrict__ S, int rz_slot,
                                                 const double* __restrict__ dinv, double inv_theta,
                                                 double* __restrict__ x, double* __restrict__ r,
                                                 double* __restrict__ z, double* __restrict__ dk,
                                                 const double* __restrict__ p, const double* __restrict__ q,
                                                 double* __restrict__ part_rz, double* __restrict__ part_rr) {
    __shared__ double sh[kT / 64 + 1];
    const double pq = sum_partials(part_pq, nb, sh);
    const double alpha = pq != 0.0 ? S[rz_slot] / pq : 0.0;
    double rz = 0.0, rr = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kT) {
        x[i] += alpha * p[i];
        const double ri = dinv[i] != 0.0 ? r[i] - alpha * q[i] : 0.0;
        const double zi = inv_theta * (dinv[i] * ri);
        r[i] = ri;
        z[i] = zi;
        if (dk) dk[i] = zi;
        rz += ri * zi;
        rr += ri * ri;
    }
    double t = block_sum(rz, sh);
    if (threadIdx.x == 0) part_rz[blockIdx.x] = t;
    t = block_sum(rr, sh);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = t;
}

// One Chebyshev step of the preconditioner: per row, d = c1 d + c2 dinv (r -
// A z_in), z_out = z_in + d (and p = z_out when p is given, at the start of
// a solve); partials of r . z_out when part_rz is given (the last step).
__global__ void __launch_bounds__(kT) k_cheb_step(int64_t n, const int64_t* __restrict__ off,
                                                 const int32_t* __restrict__ width, const int32_t* __restrict__ col,
                                                 const double* __restrict__ val, const double* __restrict__ dinv,
                                                 const double* __restrict__ r, const double* __restrict__ zin,
                                                 double* __restrict__ zout, double* __restrict__ dk, double c1,
                                                 double c2, double* __restrict__ p, double* __restrict__ part_rz) {
    __shared__ double sh[kT / 64 + 1];
    double rz = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i - threadIdx.x < n; i += int64_t(gridDim.x) * kT) {
        if (i < n) {
            const int64_t sl = i / kSlice;
            const int64_t base = off[sl] + (i - sl * kSlice);
            const int w = width[sl];
            double s = 0.0;
#pragma unroll 4
            for (int k = 0; k < w; ++k) s += val[base + int64_t(kSlice) * k] * zin[col[base + int64_t(kSlice) * k]];
            const double d = c1 * dk[i] + c2 * (dinv[i] * (r[i] - s));
            const double zo = zin[i] + d;
            dk[i] = d;
            zout[i] = zo;
            if (p) p[i] = zo;
            rz += r[i] * zo;
        }
    }
    if (part_rz) {
        const double t = block_sum(rz, sh);
        if (threadIdx.x == 0) part_rz[blockIdx.x] = t;
    }
}

// per block the largest dinv_i sum_j |a_ij| of its rows
__global__ void __launch_bounds__(kT) k_gershgorin(int64_t n, const int64_t* __restrict__ off,
                                                  const int32_t* __restrict__ width, const double* __restrict__ val,
                                                  const double* __restrict__ dinv, double* __restrict__ part) {
    __shared__ double sh[kT / 64];
    double m = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kT) {
        const int64_t sl = i / kSlice;
        const int64_t base = off[sl] + (i - sl * kSlice);
        double s = 0.0;
        for (int k = 0; k < width[sl]; ++k) s += fabs(val[base + int64_t(kSlice) * k]);
        m = fmax(m, fabs(dinv[i]) * s);
    }
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int q = 1; q < kT / 64; ++q) t = fmax(t, sh[q]);
        part[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kT) k_max_partials(const double* __restrict__ part, int n, double* __restrict__ S,
                                                    int slot) {
    __shared__ double sh[kT / 64];
    double m = 0.0;
    for (int q = threadIdx.x; q < n; q += kT) m = fmax(m, part[q]);
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kT / 64; ++q) m = fmax(m, sh[q]);
        S[slot] = m;
    }
}

// beta = rz_new / rz_old; p = z + beta p.  Block 0 stores rz_new in the next
// iteration's slot and the residual r . r; the old slot is only read.
__global__ void __launch_bounds__(kT) k_cg_direction(int64_t n, int nb, const double* __restrict__ part_rz,
                                                    const double* __restrict__ part_rr, double* __restrict__ S,
                                                    int rz_old, int rz_new, const double* __restrict__ z,
                                                    double* __restrict__ p) {
    __shared__ double sh[kT / 64 + 1];
    const double rzn = sum_partials(part_rz, nb, sh);
    const double rz0 = S[rz_old];
    const double beta = rz0 != 0.0 ? rzn / rz0 : 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kT)
        p[i] = z[i] + beta * p[i];
    const double rr = sum_partials(part_rr, nb, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S[rz_new] = rzn;
        S[kSlotRR] = rr;
    }
}

__global__ void __launch_bounds__(kT) k_gather(int64_t nb_nodes, const int32_t* __restrict__ nodes,
                                              const double* __restrict__ u, double* __restrict__ ub) {
    const int64_t j = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (j < nb_nodes) ub[j] = u[nodes[j]];
}

// g = 0 except g[nodes[j]] = ub[j]
__global__ void __launch_bounds__(kT) k_scatter(int64_t nb_nodes, const int32_t* __restrict__ nodes,
                                               const double* __restrict__ ub, double* __restrict__ g) {
    const int64_t j = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (j < nb_nodes) g[nodes[j]] = ub[j];
}

__global__ void __launch_bounds__(kT) k_fill(int64_t n, double* __restrict__ x, double v) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i < n) x[i] = v;
}

// out = a + s b
__global__ void __launch_bounds__(kT) k_axpy(int64_t n, const double* __restrict__ a, double s,
                                            const double* __restrict__ b, double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i < n) out[i] = a[i] + s * b[i];
}

// h_t = -sum_a (u1 + u2)_a grad phi_a; partials of vol M . h
__global__ void __launch_bounds__(kT) k_field(int64_t n_tets, const int32_t* __restrict__ tet,
                                             const double* __restrict__ geo, const double* __restrict__ u1,
                                             const double* __restrict__ u2, const double* __restrict__ m,
                                             double* __restrict__ h, double* __restrict__ part) {
    __shared__ double sh[kT / 64 + 1];
    double acc = 0.0;
    for (int64_t t = int64_t(blockIdx.x) * kT + threadIdx.x; t < n_tets; t += int64_t(gridDim.x) * kT) {
        const double* g = geo + kGeo * t;
        double hx = 0.0, hy = 0.0, hz = 0.0;
        for (int a = 0; a < 4; ++a) {
            const int32_t v = tet[4 * t + a];
            const double u = u1[v] + u2[v];
            hx -= u * g[1 + 3 * a];
            hy -= u * g[2 + 3 * a];
            hz -= u * g[3 + 3 * a];
        }
        h[3 * t] = hx;
        h[3 * t + 1] = hy;
        h[3 * t + 2] = hz;
        acc += g[0] * (m[3 * t] * hx + m[3 * t + 1] * hy + m[3 * t + 2] * hz);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// inverse diagonals: dinv_free for the Neumann solve (every node free),
// dinv_fix for the Dirichlet solve (0 on the boundary nodes, which are fixed)
__global__ void __launch_bounds__(kT) k_dinv(int64_t n, const int64_t* __restrict__ rowptr,
                                            const int32_t* __restrict__ col, const double* __restrict__ val,
                                            const uint8_t* __restrict__ on_boundary, double* __restrict__ dinv_free,
                                            double* __restrict__ dinv_fix) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
        if (col[k] == i) d = val[k];
    const double inv = d > 0.0 ? 1.0 / d : 0.0;
    dinv_free[i] = inv;
    dinv_fix[i] = on_boundary[i] ? 0.0 : inv;
}

__global__ void __launch_bounds__(kT) k_scale(int64_t n, double s, const double* __restrict__ a, double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i < n) out[i] = s * a[i];
}

unsigned blocks_of(int64_t n) { return unsigned((n + kT - 1) / kT); }

}  // namespace

hipError_t fem_geometry(int64_t n_tets, const double* xyz, const int32_t* tet, double* geo, hipStream_t st) {
    if (n_tets > 0) hipLaunchKernelGGL(k_geometry, dim3(blocks_of(n_tets)), dim3(kT), 0, st, n_tets, xyz, tet, geo);
    return hipGetLastError();
}

hipError_t fem_stiffness(int64_t n, const int64_t* inc_off, const int32_t* inc, const int32_t* tet, const double* geo,
                         const int64_t* rowptr, const int32_t* col, double* val, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_stiffness, dim3(blocks_of(n)), dim3(kT), 0, st, n, inc_off, inc, tet, geo, rowptr, col, val);
    return hipGetLastError();
}

hipError_t fem_dinv(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val, const uint8_t* on_boundary,
                    double* dinv_free, double* dinv_fix, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_dinv, dim3(blocks_of(n)), dim3(kT), 0, st, n, rowptr, col, val, on_boundary, dinv_free,
                           dinv_fix);
    return hipGetLastError();
}

hipError_t fem_scale(int64_t n, double s, const double* a, double* out, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_scale, dim3(blocks_of(n)), dim3(kT), 0, st, n, s, a, out);
    return hipGetLastError();
}

hipError_t fem_to_ell(int64_t n, const int64_t* rowptr, const double* val, const FemCg& c, double* ell_val,
                      hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_to_ell, dim3(blocks_of(n)), dim3(kT), 0, st, n, rowptr, val, c.off, c.width, ell_val);
    return hipGetLastError();
}

hipError_t fem_rhs(int64_t n, const int64_t* inc_off, const int32_t* inc, const double* geo, const double* m,
                   double* b, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_rhs, dim3(blocks_of(n)), dim3(kT), 0, st, n, inc_off, inc, geo, m, b);
    return hipGetLastError();
}

hipError_t fem_dot(int64_t n, const double* a, const double* b, double* part, double* S, int slot, double scale,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_dot, dim3(kFemBlocks), dim3(kT), 0, st, n, a, b, part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kT), 0, st, part, int(kFemBlocks), S, slot, scale);
    return hipGetLastError();
}

hipError_t fem_shift(int64_t n, double* x, const double* S, int slot, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_shift, dim3(blocks_of(n)), dim3(kT), 0, st, n, x, S, slot);
    return hipGetLastError();
}

// the Chebyshev steps 1 .. deg - 1 after z_0 and d_0 are set in c.z and c.dk;
// returns the buffer holding the final z (p = that z too when p is given)
static double* cheb_steps(const FemCg& c, double* p, hipStream_t st) {
    double* zin = c.z;
    double* zout = c.z2;
    for (int k = 1; k < c.deg; ++k) {
        const bool last = k == c.deg - 1;
        hipLaunchKernelGGL(k_cheb_step, dim3(kFemBlocks), dim3(kT), 0, st, c.n, c.off, c.width, c.col, c.val, c.dinv,
                           c.r, zin, zout, c.dk, c.c1[k], c.c2[k], last ? p : nullptr, last ? c.part_rz : nullptr);
        double* t = zin;
        zin = zout;
        zout = t;
    }
    return zin;
}

hipError_t fem_cg_start(const FemCg& c, const double* b, double* x, hipStream_t st) {
    const bool cheb = c.deg > 1;
    hipLaunchKernelGGL(k_cg_start, dim3(kFemBlocks), dim3(kT), 0, st, c.n, b, c.dinv, c.inv_theta, x, c.r, c.z, c.p,
                       cheb ? c.dk : nullptr, c.part_rz, c.part_rr);
    if (cheb) cheb_steps(c, c.p, st);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kT), 0, st, c.part_rz, int(kFemBlocks), c.S, kSlotRZ0, 1.0);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kT), 0, st, c.part_rr, int(kFemBlocks), c.S, kSlotRR, 1.0);
    return hipGetLastError();
}

unsigned spmv_blocks(int64_t n) {
    return unsigned(std::max<int64_t>(1, std::min<int64_t>((n + kT - 1) / kT, kSpmvBlocks)));
}

hipError_t fem_cg_step(const FemCg& c, double* x, int iter, hipStream_t st) {
    const int rz_old = kSlotRZ0 + (iter & 1), rz_new = kSlotRZ0 + ((iter + 1) & 1);
    const unsigned nb = spmv_blocks(c.n);
    hipLaunchKernelGGL(k_spmv_dot, dim3(nb), dim3(kT), 0, st, c.n, c.off, c.width, c.col, c.val, c.p, c.q,
                       c.part_pq);
    const bool cheb = c.deg > 1;
    hipLaunchKernelGGL(k_cg_update, dim3(kFemBlocks), dim3(kT), 0, st, c.n, int(nb), c.part_pq, c.S, rz_old, c.dinv,
                       c.inv_theta, x, c.r, c.z, cheb ? c.dk : nullptr, c.p, c.q, c.part_rz, c.part_rr);
    const double* z = cheb ? cheb_steps(c, nullptr, st) : c.z;
    hipLaunchKernelGGL(k_cg_direction, dim3(kFemBlocks), dim3(kT), 0, st, c.n, int(kFemBlocks), c.part_rz, c.part_rr,
                       c.S, rz_old, rz_new, z, c.p);
    return hipGetLastError();
}

hipError_t fem_gershgorin(const FemCg& c, double* part, double* S, int slot, hipStream_t st) {
    hipLaunchKernelGGL(k_gershgorin, dim3(kFemBlocks), dim3(kT), 0, st, c.n, c.off, c.width, c.val, c.dinv, part);
    hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(kT), 0, st, part, int(kFemBlocks), S, slot);
    return hipGetLastError();
}

hipError_t fem_spmv(const FemCg& c, const double* x, double* y, hipStream_t st) {
    hipLaunchKernelGGL(k_spmv_dot, dim3(spmv_blocks(c.n)), dim3(kT), 0, st, c.n, c.off, c.width, c.col, c.val, x, y,
                       c.part_pq);
    return hipGetLastError();
}

hipError_t fem_gather(int64_t nb_nodes, const int32_t* nodes, const double* u, double* ub, hipStream_t st) {
    if (nb_nodes > 0) hipLaunchKernelGGL(k_gather, dim3(blocks_of(nb_nodes)), dim3(kT), 0, st, nb_nodes, nodes, u, ub);
    return hipGetLastError();
}

hipError_t fem_scatter(int64_t n, int64_t nb_nodes, const int32_t* nodes, const double* ub, double* g,
                       hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(blocks_of(n)), dim3(kT), 0, st, n, g, 0.0);
    if (nb_nodes > 0)
        hipLaunchKernelGGL(k_scatter, dim3(blocks_of(nb_nodes)), dim3(kT), 0, st, nb_nodes, nodes, ub, g);
    return hipGetLastError();
}

hipError_t fem_axpy(int64_t n, const double* a, double s, const double* b, double* out, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_axpy, dim3(blocks_of(n)), dim3(kT), 0, st, n, a, s, b, out);
    return hipGetLastError();
}

hipError_t fem_field(int64_t n_tets, const int32_t* tet, const double* geo, const double* u1, const double* u2,
                     const double* m, double* h, double* part, double* S, int slot, hipStream_t st) {
    hipLaunchKernelGGL(k_field, dim3(kFemBlocks), dim3(kT), 0, st, n_tets, tet, geo, u1, u2, m, h, part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kT), 0, st, part, int(kFemBlocks), S, slot, -0.5);
    return hipGetLastError();
}

}  // namespace h2dlp
