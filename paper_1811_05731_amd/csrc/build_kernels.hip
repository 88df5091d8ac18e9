// Build-time kernels: everything the apply streams is generated here, in FP64
// arithmetic, and stored in the precision of the operator (layout.h).
//
//  * triangle normals/areas and the node solid angle Psi (diagonal of M,
//    eq. matrix_definition of arXiv:1811.05731, Section 3);
//  * the interpolation setup of Section 4: Chebyshev points of every cluster
//    box, leaf row bases V_t, leaf column bases W_s (exact triangle
//    quadrature), transfer factors E_c, coupling matrices S_ts;
//  * the exact double-layer entries of the inadmissible leaf blocks from the
//    closed-form triangle integrals the paper cites in Section 3.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "interp.h"
#include "kernels.h"

namespace h2dlp {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kBuildThreads = 256;

__device__ inline void sub3(const double* a, const double* b, double* o) {
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
__device__ inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__device__ inline void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Contribution of triangle r (counter-clockwise about its outward normal) to
// K_ij for the node at local vertex a, seen from x = xi_i, x not a vertex:
//   L_a(x) = s_{a+1}/(8 pi A) [ (n x u_{a+1}).(x - r_{a+1}) Omega(x) + zeta sum_b (u_{a+1}.u_b) P_b ],
// with Omega the signed solid angle (Van Oosterom-Strackee), P_b the edge
// potential integral of 1/|x - y| and zeta the height of x above the plane.
__device__ double lindholm_weight(const double* x, const double r[3][3], int a) {
    double e[3][3], u[3][3], s[3], R[3][3], rho[3], P[3];
    for (int b = 0; b < 3; ++b) {
        sub3(r[(b + 1) % 3], r[b], e[b]);
        s[b] = sqrt(dot3(e[b], e[b]));
        for (int c = 0; c < 3; ++c) u[b][c] = e[b][c] / s[b];
        sub3(x, r[b], R[b]);
        rho[b] = sqrt(dot3(R[b], R[b]));
    }
    double d02[3], cr[3], n[3];
    sub3(r[2], r[0], d02);
    cross3(e[0], d02, cr);
    const double two_a = sqrt(dot3(cr, cr));
    for (int c = 0; c < 3; ++c) n[c] = cr[c] / two_a;
    for (int b = 0; b < 3; ++b) {
        const double ssum = rho[b] + rho[(b + 1) % 3];
        P[b] = log1p(2.0 * s[b] / (ssum - s[b]));
    }
    double c12[3];
    cross3(R[1], R[2], c12);
    const double num = dot3(R[0], c12);
    const double den = rho[0] * rho[1] * rho[2] + rho[0] * dot3(R[1], R[2]) + rho[1] * dot3(R[2], R[0]) +
                       rho[2] * dot3(R[0], R[1]);
    const double omega = 2.0 * atan2(num, den);
    const double zeta = dot3(n, R[0]);
    const int op = (a + 1) % 3;
    double eta[3];
    cross3(n, u[op], eta);
    const double term1 = dot3(eta, R[op]) * omega;
    double term2 = 0.0;
    for (int b = 0; b < 3; ++b) term2 += dot3(u[op], u[b]) * P[b];
    term2 *= zeta;
    return s[op] / (8.0 * kPi * (0.5 * two_a)) * (term1 + term2);
}

// the m Chebyshev points of one box axis
__device__ inline void cheb_axis(const double* box, int axis, int m, double* pts) {
    for (int l = 0; l < m; ++l) pts[l] = cheb_point(box, axis, m, l);
}

__device__ inline double lagrange(const double* pts, int m, int l, double x) {
    double v = 1.0;
    for (int p = 0; p < m; ++p)
        if (p != l) v *= (x - pts[p]) / (pts[l] - pts[p]);
    return v;
}

__device__ inline double lagrange_d(const double* pts, int m, int l, double x) {
    double d = 0.0;
    for (int p = 0; p < m; ++p) {
        if (p == l) continue;
        double t = 1.0 / (pts[l] - pts[p]);
        for (int q = 0; q < m; ++q)
            if (q != l && q != p) t *= (x - pts[q]) / (pts[l] - pts[q]);
        d += t;
    }
    return d;
}

template <typename T>
__device__ inline void put(void* pool, int64_t off, double v) {
    static_cast<T*>(pool)[off] = T(v);
}

__device__ inline void put_prec(void* pool, int64_t off, double v, int prec) {
    if (prec == P_FP64) put<double>(pool, off, v);
    else put<float>(pool, off, v);
}

__global__ void __launch_bounds__(kBuildThreads) k_tri_geometry(const double* xyz, const int32_t* tri, int64_t n_tris,
                                                                double* tgeo) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n_tris) return;
    const double* p = xyz + 3 * int64_t(tri[3 * e]);
    const double* q = xyz + 3 * int64_t(tri[3 * e + 1]);
    const double* r = xyz + 3 * int64_t(tri[3 * e + 2]);
    double a[3], b[3], c[3];
    sub3(q, p, a);
    sub3(r, p, b);
    cross3(a, b, c);
    const double two_a = sqrt(dot3(c, c));
    tgeo[4 * e + 0] = c[0] / two_a;
    tgeo[4 * e + 1] = c[1] / two_a;
    tgeo[4 * e + 2] = c[2] / two_a;
    tgeo[4 * e + 3] = 0.5 * two_a;
}

// Psi_i = 2 pi - sum over edges (i, k) of the signed turning angle between the
// normals of the triangle running i -> k and the one running k -> i; the
// diagonal is D = Psi/(4 pi) - 1.  Output by cluster position.
__global__ void __launch_bounds__(kBuildThreads) k_diagonal(DevMesh mesh, int64_t n_nodes, double* diag) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n_nodes) return;
    const int32_t i = mesh.perm[p];
    const int64_t b = mesh.inc_off[i], e = mesh.inc_off[i + 1];
    double psi = 2.0 * kPi;
    for (int64_t q = b; q < e; ++q) {
        const int32_t ta = mesh.inc_tri[q];
        const int32_t k = mesh.tri[3 * int64_t(ta) + (mesh.inc_loc[q] + 1) % 3];
        int32_t tb = -1;
        for (int64_t w = b; w < e; ++w) {
            const int32_t t2 = mesh.inc_tri[w];
            if (mesh.tri[3 * int64_t(t2) + (mesh.inc_loc[w] + 2) % 3] == k) { tb = t2; break; }
        }
        if (tb < 0) continue;   // cannot happen on a checked closed mesh
        const double* na = mesh.tgeo + 4 * int64_t(ta);
        const double* nb = mesh.tgeo + 4 * int64_t(tb);
        double ev[3], c[3];
        sub3(mesh.xyz + 3 * int64_t(k), mesh.xyz + 3 * int64_t(i), ev);
        const double len = sqrt(dot3(ev, ev));
        for (int d = 0; d < 3; ++d) ev[d] /= len;
        cross3(na, nb, c);
        psi -= atan2(dot3(c, ev), dot3(na, nb));
    }
    diag[p] = psi / (4.0 * kPi) - 1.0;
}

// Row basis of a leaf: V(i, nu) = L^t_nu(xi_i), nu = lx + m ly + m^2 lz; block n_t x k.
__global__ void __launch_bounds__(kBuildThreads) k_build_v(DevMesh mesh, const double* boxes, int m,
                                                           const LeafDesc* leaves, int prec, void* pool) {
    __shared__ double pts[3][8];
    const LeafDesc L = leaves[blockIdx.x];
    const double* box = boxes + 6 * int64_t(L.gid);
    if (threadIdx.x < 3) cheb_axis(box, threadIdx.x, m, pts[threadIdx.x]);
    __syncthreads();
    const int k = m * m * m;
    for (int e = threadIdx.x; e < L.n * k; e += blockDim.x) {
        const int i = e / k, nu = e % k;
        const int lx = nu % m, ly = (nu / m) % m, lz = nu / (m * m);
        const double* x = mesh.xyz + 3 * int64_t(mesh.perm[L.pos + i]);
        const double v = lagrange(pts[0], m, lx, x[0]) * lagrange(pts[1], m, ly, x[1]) * lagrange(pts[2], m, lz, x[2]);
        put_prec(pool, L.a_off + a_offset(L.n, k, i, nu), v, prec);
    }
}

// Transposed column basis of a leaf: A(mu, j) = W(j, mu) =
//   sum_{T incident to j} 2 A_T sum_q w_q phi_j(y_q) n_T . grad L^s_mu(y_q);
// block k x n_s.  quad: (u, v, weight) on the reference triangle, exact for the
// polynomial integrand.  One 64-lane workgroup per node j of a leaf: for each
// incident triangle the lanes first tabulate the 1D Lagrange values and
// derivatives of the three axes at every quadrature point (LDS, from the
// reciprocal differences of the leaf's Chebyshev points), then lane mu sums
// its entries over the points.  tab: n_quad x 3 x 2m doubles (dynamic LDS).
__global__ void __launch_bounds__(64) k_build_wt(DevMesh mesh, const double* boxes, int m, const double* quad,
                                                 int n_quad, const LeafDesc* leaves, int prec, void* pool) {
    extern __shared__ double tab[];
    __shared__ double pts[3][8], inv[3][8][8];
    const LeafDesc* L = leaves + blockIdx.x;
    const int n = L->n, j = int(blockIdx.y);
    if (j >= n) return;                       // uniform over the workgroup
    const double* box = boxes + 6 * int64_t(L->gid);
    const int t = int(threadIdx.x);
    if (t < 3 * m) pts[t / m][t % m] = cheb_point(box, t / m, m, t % m);
    __syncthreads();
    for (int e = t; e < 3 * m * m; e += 64) {
        const int a = e / (m * m), l = (e / m) % m, p = e % m;
        inv[a][l][p] = l == p ? 0.0 : 1.0 / (pts[a][l] - pts[a][p]);
    }
    __syncthreads();
    const int k = m * m * m;
    const int32_t node = mesh.perm[L->pos + j];
    double total[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) total[s] = 0.0;
    for (int64_t qi = mesh.inc_off[node]; qi < mesh.inc_off[node + 1]; ++qi) {
        const int64_t T = mesh.inc_tri[qi];
        const int loc = mesh.inc_loc[qi];
        const double* r1 = mesh.xyz + 3 * int64_t(mesh.tri[3 * T]);
        const double* r2 = mesh.xyz + 3 * int64_t(mesh.tri[3 * T + 1]);
        const double* r3 = mesh.xyz + 3 * int64_t(mesh.tri[3 * T + 2]);
        const double* g = mesh.tgeo + 4 * T;
        for (int e = t; e < 3 * n_quad; e += 64) {
            const int qq = e / 3, a = e % 3;
            const double u = quad[3 * qq], v = quad[3 * qq + 1];
            const double y = r1[a] + u * (r2[a] - r1[a]) + v * (r3[a] - r1[a]);
            double* fv = tab + int64_t(e) * 2 * m;
            for (int l = 0; l < m; ++l) {
                double f = 1.0, d = 0.0;
                for (int p = 0; p < m; ++p) {
                    if (p == l) continue;
                    f *= (y - pts[a][p]) * inv[a][l][p];
                    double dp = inv[a][l][p];
                    for (int q2 = 0; q2 < m; ++q2)
                        if (q2 != l && q2 != p) dp *= (y - pts[a][q2]) * inv[a][l][q2];
                    d += dp;
                }
                fv[l] = f;
                fv[m + l] = d;
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int mu = t + 64 * s;
            if (mu >= k) break;
            const int lx = mu % m, ly = (mu / m) % m, lz = mu / (m * m);
            double acc = 0.0;
            for (int qq = 0; qq < n_quad; ++qq) {
                const double u = quad[3 * qq], v = quad[3 * qq + 1], w = quad[3 * qq + 2];
                const double* tx = tab + int64_t(3 * qq) * 2 * m;
                const double* ty = tx + 2 * m;
                const double* tz = ty + 2 * m;
                const double fx = tx[lx], fy = ty[ly], fz = tz[lz];
                const double dn = g[0] * tx[m + lx] * fy * fz + g[1] * fx * ty[m + ly] * fz + g[2] * fx * fy * tz[m + lz];
                const double phi = loc == 0 ? 1.0 - u - v : (loc == 1 ? u : v);
                acc += w * phi * dn;
            }
            total[s] += 2.0 * g[3] * acc;
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int mu = t + 64 * s;
        if (mu < k) put_prec(pool, L->a_off + a_offset(k, n, mu, j), total[s], prec);
    }
}

// Transfer factors of every non-root cluster c with parent t, per axis:
// E[c][axis][l'][l] = L^t_l(eta^c_l').  The full transfer is their Kronecker product.
__global__ void __launch_bounds__(kBuildThreads) k_build_transfer(const double* boxes, const int32_t* parent,
                                                                  int64_t n_clusters, int m, int prec, void* e) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = 3 * m * m;
    if (g >= n_clusters * per) return;
    const int64_t c = g / per;
    const int r = int(g % per);
    const int axis = r / (m * m), lp = (r / m) % m, l = r % m;
    const int32_t t = parent[c];
    double v = 0.0;
    if (t >= 0) {
        double pc[8], pt[8];
        cheb_axis(boxes + 6 * c, axis, m, pc);
        cheb_axis(boxes + 6 * int64_t(t), axis, m, pt);
        v = lagrange(pt, m, l, pc[lp]);
    }
    put_prec(e, g, v, prec);
}

// Coupling matrix of an admissible block: S(nu, mu) = 1/(4 pi |eta^t_nu - eta^s_mu|),
// stored k x kp with zero columns mu >= k.
// BF16X3 stores each entry as (hi, lo) bfloat16, hi = bf16(S), lo = bf16(S - hi);
// BF16X6 as (hi, mid, lo), each term the bfloat16 rounding of what the earlier
// terms leave of S (remainders taken in FP64).
__global__ void __launch_bounds__(kBuildThreads) k_build_coupling(const double* boxes, int m, int kp,
                                                                  const FarDesc* far, int prec, void* pool) {
    __shared__ double pt[3][8], ps[3][8];
    const FarDesc F = far[blockIdx.x];
    if (threadIdx.x < 3) cheb_axis(boxes + 6 * int64_t(F.t), threadIdx.x, m, pt[threadIdx.x]);
    else if (threadIdx.x < 6) cheb_axis(boxes + 6 * int64_t(F.s), threadIdx.x - 3, m, ps[threadIdx.x - 3]);
    __syncthreads();
    const int k = m * m * m;
    for (int e = threadIdx.x; e < k * kp; e += blockDim.x) {
        const int nu = e / kp, mu = e % kp;
        double v = 0.0;
        if (mu < k) {
            const double dx = pt[0][nu % m] - ps[0][mu % m];
            const double dy = pt[1][(nu / m) % m] - ps[1][(mu / m) % m];
            const double dz = pt[2][nu / (m * m)] - ps[2][mu / (m * m)];
            v = 1.0 / (4.0 * kPi * sqrt(dx * dx + dy * dy + dz * dz));
        }
        const int P = bf16_parts(prec);
        if (P > 0) {
            // a_off counts entries of P bfloat16 terms each, placed by the split layout
            __bf16* base = static_cast<__bf16*>(pool) + int64_t(P) * F.a_off;
            double rem = v;
            for (int q = 0; q < P; ++q) {
                const __bf16 t = __bf16(float(rem));
                base[bf16s_offset(k, nu, mu, q, P)] = t;
                rem -= double(float(t));
            }
        } else {
            put_prec(pool, F.a_off + a_offset(k, kp, nu, mu), v, prec);
        }
    }
}

// Exact entries of an inadmissible leaf block:
//   K_ij = sum over triangles T incident to j, i not a vertex of T, of L_{loc(j,T)}(xi_i).
// With ns_val != NULL, entries whose column lies in the 2-ring of the row are
// written to ns_val (FP64) and stored as 0 in the block.
__global__ void __launch_bounds__(kBuildThreads) k_build_near(DevMesh mesh, const NearDesc* near, int prec, void* pool,
                                                              const int64_t* ring_off, const int32_t* ring_pos,
                                                              double* ns_val) {
    const NearDesc B = near[blockIdx.x];
    for (int e = threadIdx.x; e < B.nt * B.ns; e += blockDim.x) {
        const int i = e / B.ns, j = e % B.ns;
        const int32_t ni = mesh.perm[B.tpos + i], nj = mesh.perm[B.spos + j];
        const double* x = mesh.xyz + 3 * int64_t(ni);
        double v = 0.0;
        for (int64_t q = mesh.inc_off[nj]; q < mesh.inc_off[nj + 1]; ++q) {
            const int64_t T = mesh.inc_tri[q];
            const int32_t v0 = mesh.tri[3 * T], v1 = mesh.tri[3 * T + 1], v2 = mesh.tri[3 * T + 2];
            if (v0 == ni || v1 == ni || v2 == ni) continue;   // incident: exactly 0
            double r[3][3];
            for (int a = 0; a < 3; ++a) {
                r[0][a] = mesh.xyz[3 * int64_t(v0) + a];
                r[1][a] = mesh.xyz[3 * int64_t(v1) + a];
                r[2][a] = mesh.xyz[3 * int64_t(v2) + a];
            }
            v += lindholm_weight(x, r, mesh.inc_loc[q]);
        }
        const int64_t off = B.a_off + a_offset(B.nt, B.ns, i, j);
        if (ns_val != nullptr) {
            const int64_t lo0 = ring_off[B.tpos + i], hi0 = ring_off[B.tpos + i + 1];
            const int32_t want = B.spos + j;
            int64_t lo = lo0, hi = hi0;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (ring_pos[mid] < want) lo = mid + 1; else hi = mid;
            }
            if (lo < hi0 && ring_pos[lo] == want) {
                ns_val[lo] = v;
                v = 0.0;
            }
        }
        put_prec(pool, off, v, prec);
    }
}

inline unsigned blocks_for(int64_t n) { return unsigned((n + kBuildThreads - 1) / kBuildThreads); }

}  // namespace

hipError_t launch_tri_geometry(const double* xyz, const int32_t* tri, int64_t n_tris, double* tgeo, hipStream_t st) {
    if (n_tris == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tri_geometry, dim3(blocks_for(n_tris)), dim3(kBuildThreads), 0, st, xyz, tri, n_tris, tgeo);
    return hipGetLastError();
}

hipError_t launch_diagonal(DevMesh mesh, int64_t n_nodes, double* diag, hipStream_t st) {
    hipLaunchKernelGGL(k_diagonal, dim3(blocks_for(n_nodes)), dim3(kBuildThreads), 0, st, mesh, n_nodes, diag);
    return hipGetLastError();
}

hipError_t launch_build_v(DevMesh mesh, const double* boxes, int m, const LeafDesc* leaves, int64_t n_leaves,
                          int prec, void* pool, hipStream_t st) {
    if (n_leaves == 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_v, dim3(unsigned(n_leaves)), dim3(kBuildThreads), 0, st, mesh, boxes, m, leaves, prec,
                       pool);
    return hipGetLastError();
}

hipError_t launch_build_wt(DevMesh mesh, const double* boxes, int m, const double* quad, int n_quad,
                           const LeafDesc* leaves, int64_t n_leaves, int max_leaf, int prec, void* pool,
                           hipStream_t st) {
    if (n_leaves == 0) return hipSuccess;
    if (max_leaf < 1 || max_leaf > 64 || m < 1 || m > 8) return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * size_t(n_quad) * 6 * size_t(m);
    if (lds > 60 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_build_wt, dim3(unsigned(n_leaves), unsigned(max_leaf)), dim3(64), lds, st, mesh, boxes, m,
                       quad, n_quad, leaves, prec, pool);
    return hipGetLastError();
}

hipError_t launch_build_transfer(const double* boxes, const int32_t* parent, int64_t n_clusters, int m, int prec,
                                 void* e, hipStream_t st) {
    hipLaunchKernelGGL(k_build_transfer, dim3(blocks_for(n_clusters * 3 * m * m)), dim3(kBuildThreads), 0, st, boxes,
                       parent, n_clusters, m, prec, e);
    return hipGetLastError();
}

hipError_t launch_build_coupling(const double* boxes, int m, int kp, const FarDesc* far, int64_t n_far, int prec,
                                 void* pool, hipStream_t st) {
    if (n_far == 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_coupling, dim3(unsigned(n_far)), dim3(kBuildThreads), 0, st, boxes, m, kp, far, prec,
                       pool);
    return hipGetLastError();
}

hipError_t launch_build_near(DevMesh mesh, const NearDesc* near, int64_t n_near, int prec, void* pool,
                             const int64_t* ring_off, const int32_t* ring_pos, double* ns_val, hipStream_t st) {
    if (n_near == 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_near, dim3(unsigned(n_near)), dim3(kBuildThreads), 0, st, mesh, near, prec, pool,
                       ring_off, ring_pos, ns_val);
    return hipGetLastError();
}

}  // namespace h2dlp
