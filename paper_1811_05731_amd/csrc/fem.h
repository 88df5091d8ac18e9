// Finite-element solves either side of the boundary operator: kernels and
// their host-side arguments.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace h2dlp {

constexpr int kGeo = 13;                   // doubles per tetrahedron: volume, then grad phi_0..3
constexpr unsigned kFemBlocks = 1024;      // blocks of the reducing vector kernels (their partials)
constexpr unsigned kSpmvBlocks = 2048;     // most blocks of the matrix-vector product (one row a thread)
constexpr int kSlice = 64;                 // rows of a sliced-ELL slice (one wavefront)
constexpr int kMaxCheb = 8;                // largest degree of the Chebyshev preconditioner

// slots of the device scalar array
constexpr int kSlotRZ0 = 0;                // r . z of the current and of the next CG iteration (0, 1)
constexpr int kSlotRR = 2;                 // r . r after the last CG iteration
constexpr int kSlotBB = 3;                 // b . b of the system being solved
constexpr int kSlotMean = 4;               // a mean to remove
constexpr int kSlotEnergy = 5;             // -(1/2) sum vol M . H
constexpr int kSlotLambda = 6;             // the Gershgorin bound of D^-1 A (build)
constexpr int kSlots = 8;

// One preconditioned CG solve on the stiffness matrix, FP64 in sliced ELL:
// slice s (rows 64 s .. 64 s + 63) holds w[s] slots, entry (row 64 s + r,
// slot k) at off[s] + 64 k + r, its columns in ascending order, padding with
// the row's own column and 0.  Rows with dinv = 0 are fixed (their residual is
// held at zero).
//
// Preconditioner: deg steps of the Chebyshev iteration for D^-1 A z = D^-1 r
// from z = 0 on the interval [lmin, lmax] of D^-1 A's spectrum (D the
// diagonal): z_0 = inv_theta D^-1 r, d_0 = z_0, then for k = 1 .. deg - 1
// d_k = c1[k] d_{k-1} + c2[k] D^-1 (r - A z_{k-1}), z_k = z_{k-1} + d_k.
// deg = 1 with inv_theta = 1 is the Jacobi preconditioner.  The polynomial is
// positive on (0, lmax], so the preconditioner is symmetric positive definite
// when lmax bounds the spectrum.
struct FemCg {
    int64_t n;
    const int64_t* off;
    const int32_t* width;
    const int32_t* col;
    const double* val;
    const double* dinv;
    double *r, *z, *p, *q;
    double *part_pq;                       // kSpmvBlocks (one per block of the matrix-vector product)
    double *part_rz, *part_rr;             // kFemBlocks each
    double* S;                             // kSlots
    double *z2, *dk;                       // Chebyshev: the other z buffer and the step d_k
    int deg;
    double inv_theta;
    double c1[kMaxCheb], c2[kMaxCheb];
};

hipError_t fem_geometry(int64_t n_tets, const double* xyz, const int32_t* tet, double* geo, hipStream_t st);
hipError_t fem_stiffness(int64_t n, const int64_t* inc_off, const int32_t* inc, const int32_t* tet, const double* geo,
                         const int64_t* rowptr, const int32_t* col, double* val, hipStream_t st);
// the CSR values into the sliced-ELL layout of `c` (its columns already set)
hipError_t fem_to_ell(int64_t n, const int64_t* rowptr, const double* val, const FemCg& c, double* ell_val,
                      hipStream_t st);
hipError_t fem_dinv(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val, const uint8_t* on_boundary,
                    double* dinv_free, double* dinv_fix, hipStream_t st);
// out = s a
hipError_t fem_scale(int64_t n, double s, const double* a, double* out, hipStream_t st);
hipError_t fem_rhs(int64_t n, const int64_t* inc_off, const int32_t* inc, const double* geo, const double* m,
                   double* b, hipStream_t st);
// S[slot] = scale * (a . b)
hipError_t fem_dot(int64_t n, const double* a, const double* b, double* part, double* S, int slot, double scale,
                   hipStream_t st);
// x -= S[slot]
hipError_t fem_shift(int64_t n, double* x, const double* S, int slot, hipStream_t st);
hipError_t fem_cg_start(const FemCg& c, const double* b, double* x, hipStream_t st);
// max over the rows with dinv != 0 of dinv_i sum_j |a_ij| (a bound of the
// spectrum of D^-1 A by Gershgorin's theorem), into S[slot]
hipError_t fem_gershgorin(const FemCg& c, double* part, double* S, int slot, hipStream_t st);
hipError_t fem_cg_step(const FemCg& c, double* x, int iter, hipStream_t st);
// y = A x (the partials of x . y land in c.part_pq)
hipError_t fem_spmv(const FemCg& c, const double* x, double* y, hipStream_t st);
hipError_t fem_gather(int64_t nb_nodes, const int32_t* nodes, const double* u, double* ub, hipStream_t st);
// g = 0, then g[nodes[j]] = ub[j]
hipError_t fem_scatter(int64_t n, int64_t nb_nodes, const int32_t* nodes, const double* ub, double* g,
                       hipStream_t st);
hipError_t fem_axpy(int64_t n, const double* a, double s, const double* b, double* out, hipStream_t st);
// h per tetrahedron; S[slot] = -(1/2) sum vol M . h
hipError_t fem_field(int64_t n_tets, const int32_t* tet, const double* geo, const double* u1, const double* u2,
                     const double* m, double* h, double* part, double* S, int slot, hipStream_t st);

}  // namespace h2dlp
