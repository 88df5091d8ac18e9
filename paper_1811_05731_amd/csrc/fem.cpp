// The finite-element solves either side of the boundary operator (Section 2 of
// the paper): h2dlp_fem_build / h2dlp_fem_field of include/h2dlp.h.
//
// Build (once per volume mesh): the boundary surface is extracted on the host
// (faces of one tetrahedron only, oriented outward) and the boundary
// operator is built on it with the caller's options; the stiffness pattern
// (CSR, sorted columns) and each node's incident tetrahedra come from the
// host; element geometry, stiffness values and the Jacobi diagonals are
// computed on the GPU in FP64.
//
// Field (per magnetisation): right side, Jacobi-preconditioned CG for u1
// (zero node sum), u2 on the boundary through the boundary operator, CG for
// u2 on the interior nodes, H per tetrahedron and the energy, all on the
// caller's stream; the host only reads the residual every few iterations,
// and each run of iterations between two reads is one replayed HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/h2dlp.h"
#include "entry.h"
#include "fem.h"

using namespace h2dlp;

namespace {

struct FemError {
    hipError_t err;
    std::string where;
};

void hcheck(hipError_t e, const char* where) {
    if (e != hipSuccess) throw FemError{e, where};
}

constexpr int kCheckEvery = 8;   // CG iterations between two reads of the residual
// the preconditioner: Chebyshev steps on [lmax / kChebRatio, lmax] with lmax the
// Gershgorin bound of D^-1 A (fem.h)
constexpr int kChebDeg = 6;
constexpr double kChebRatio = 100.0;

}  // namespace

struct h2dlp_fem_ctx {
    int device = -1;
    int64_t n = 0, n_tets = 0, nnz = 0, ell_entries = 0;
    std::vector<int32_t> bnodes;             // boundary nodes (volume numbering), ascending
    h2dlp_handle bop = nullptr;              // the boundary operator on the surface of bnodes
    std::vector<void*> bufs;
    size_t bytes = 0;
    int32_t* d_tet = nullptr;
    double* d_geo = nullptr;
    int64_t* d_inc_off = nullptr;
    int32_t* d_inc = nullptr;
    int64_t* d_ell_off = nullptr;            // the stiffness matrix in sliced ELL (fem.h)
    int32_t* d_ell_w = nullptr;
    int32_t* d_ell_col = nullptr;
    double* d_ell_val = nullptr;
    double* d_dinv_free = nullptr;
    double* d_dinv_fix = nullptr;
    int32_t* d_bnode = nullptr;
    double *d_b = nullptr, *d_r = nullptr, *d_z = nullptr, *d_p = nullptr, *d_q = nullptr, *d_ones = nullptr;
    double *d_z2 = nullptr, *d_dk = nullptr;
    double lambda_max = 0.0;                 // Gershgorin bound of D^-1 A (0: Jacobi)
    double *d_u1 = nullptr, *d_u2 = nullptr, *d_g = nullptr, *d_ub1 = nullptr, *d_ub2 = nullptr;
    double *d_part = nullptr, *d_S = nullptr;
    double* h_S = nullptr;                   // pinned copy of the scalars
    // kCheckEvery CG iterations of each solve as one HIP graph (kernels only),
    // captured on `cap` at the first field evaluation; replayed on the caller's stream
    hipStream_t cap = nullptr;
    hipGraphExec_t g_u1 = nullptr, g_u2 = nullptr;
    bool graphs_tried = false;

    ~h2dlp_fem_ctx() {
        if (device < 0) return;
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        (void)hipDeviceSynchronize();
        if (g_u1) (void)hipGraphExecDestroy(g_u1);
        if (g_u2) (void)hipGraphExecDestroy(g_u2);
        if (cap) (void)hipStreamDestroy(cap);
        for (void* p : bufs) (void)hipFree(p);
        if (h_S) (void)hipHostFree(h_S);
        if (bop) h2dlp_free(bop);
        (void)hipSetDevice(cur);
    }
    std::vector<size_t> buf_bytes;
    template <typename T>
    T* alloc(size_t count) {
        void* p = nullptr;
        const size_t b = std::max<size_t>(count, 1) * sizeof(T);
        if (hipMalloc(&p, b) != hipSuccess) {
            (void)hipGetLastError();
            throw std::bad_alloc();
        }
        bufs.push_back(p);
        buf_bytes.push_back(b);
        bytes += b;
        return static_cast<T*>(p);
    }
    void release(void* p) {
        for (size_t q = 0; q < bufs.size(); ++q)
            if (bufs[q] == p) {
                (void)hipFree(p);
                bytes -= buf_bytes[q];
                bufs.erase(bufs.begin() + long(q));
                buf_bytes.erase(buf_bytes.begin() + long(q));
                return;
            }
    }
    template <typename T>
    T* upload(const std::vector<T>& v, hipStream_t st) {
        T* d = alloc<T>(v.size());
        if (!v.empty()) {
            hcheck(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st), "upload");
            hcheck(hipStreamSynchronize(st), "upload");
        }
        return d;
    }
    FemCg cg(const double* dinv) const {
        FemCg c{n, d_ell_off, d_ell_w, d_ell_col, d_ell_val, dinv, d_r, d_z, d_p, d_q, d_part,
                d_part + kSpmvBlocks, d_part + kSpmvBlocks + kFemBlocks, d_S, d_z2, d_dk, 1, 1.0, {}, {}};
        if (lambda_max > 0.0) {
            // Chebyshev iteration on [lmin, lmax]: theta the midpoint, delta
            // the half width, sigma = theta / delta; rho_0 = 1 / sigma and
            // rho_k = 1 / (2 sigma - rho_{k-1})
            const double lmax = lambda_max, lmin = lambda_max / kChebRatio;
            const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
            c.deg = kChebDeg;
            c.inv_theta = 1.0 / theta;
            double rho = 1.0 / sigma;
            for (int k = 1; k < kChebDeg; ++k) {
                const double rho_k = 1.0 / (2.0 * sigma - rho);
                c.c1[k] = rho_k * rho;
                c.c2[k] = 2.0 * rho_k / delta;
                rho = rho_k;
            }
        }
        return c;
    }
};

namespace {

h2dlp_fem_ctx* as_fem(h2dlp_fem f) { return reinterpret_cast<h2dlp_fem_ctx*>(f); }

// faces of one tetrahedron only, oriented so that (b - a) x (c - a) points away
// from the tetrahedron's fourth vertex
void boundary_faces(const double* xyz, const int32_t* tet, int64_t n_tets, std::vector<std::array<int32_t, 3>>* out) {
    struct Face {
        std::array<int32_t, 3> key;    // sorted
        int64_t t;
        int q;                         // the vertex left out
    };
    std::vector<Face> f;
    f.reserve(size_t(4 * n_tets));
    for (int64_t t = 0; t < n_tets; ++t)
        for (int q = 0; q < 4; ++q) {
            std::array<int32_t, 3> k{};
            int c = 0;
            for (int r = 0; r < 4; ++r)
                if (r != q) k[c++] = tet[4 * t + r];
            std::sort(k.begin(), k.end());
            f.push_back({k, t, q});
        }
    std::sort(f.begin(), f.end(), [](const Face& a, const Face& b) {
        return a.key != b.key ? a.key < b.key : (a.t != b.t ? a.t < b.t : a.q < b.q);
    });
    out->clear();
    for (size_t i = 0; i < f.size();) {
        size_t j = i + 1;
        while (j < f.size() && f[j].key == f[i].key) ++j;
        if (j - i == 1) {
            const int64_t t = f[i].t;
            std::array<int32_t, 3> v{};
            int c = 0;
            for (int r = 0; r < 4; ++r)
                if (r != f[i].q) v[c++] = tet[4 * t + r];
            const int32_t d = tet[4 * t + f[i].q];
            const double* a = xyz + 3 * int64_t(v[0]);
            const double* b = xyz + 3 * int64_t(v[1]);
            const double* cc = xyz + 3 * int64_t(v[2]);
            const double* dd = xyz + 3 * int64_t(d);
            const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
            const double e2[3] = {cc[0] - a[0], cc[1] - a[1], cc[2] - a[2]};
            const double nrm[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                   e1[0] * e2[1] - e1[1] * e2[0]};
            const double s = nrm[0] * (dd[0] - a[0]) + nrm[1] * (dd[1] - a[1]) + nrm[2] * (dd[2] - a[2]);
            if (s > 0.0) std::swap(v[1], v[2]);
            out->push_back(v);
        }
        i = j;
    }
}

int fem_build_impl(h2dlp_fem_ctx* f, const h2dlp_volume* vol, const h2dlp_options* opt, hipStream_t st) {
    const int64_t n = vol->n_nodes, T = vol->n_tets;
    f->n = n;
    f->n_tets = T;
    // boundary surface and the operator on it
    std::vector<std::array<int32_t, 3>> faces;
    boundary_faces(vol->xyz, vol->tet, T, &faces);
    std::vector<int32_t> mark(size_t(n), -1);
    for (const auto& fc : faces)
        for (int32_t v : fc) mark[v] = 0;
    for (int64_t i = 0; i < n; ++i)
        if (mark[i] == 0) {
            mark[i] = int32_t(f->bnodes.size());
            f->bnodes.push_back(int32_t(i));
        }
    if (f->bnodes.size() < 4 || faces.size() < 4) return set_error(H2DLP_EINVAL, "the volume mesh has no closed boundary");
    std::vector<double> sxyz(3 * f->bnodes.size());
    for (size_t j = 0; j < f->bnodes.size(); ++j)
        for (int d = 0; d < 3; ++d) sxyz[3 * j + d] = vol->xyz[3 * int64_t(f->bnodes[j]) + d];
    std::vector<int32_t> stri(3 * faces.size());
    for (size_t q = 0; q < faces.size(); ++q)
        for (int c = 0; c < 3; ++c) stri[3 * q + c] = mark[faces[q][c]];
    const h2dlp_mesh surf{int64_t(f->bnodes.size()), sxyz.data(), int64_t(faces.size()), stri.data()};
    h2dlp_options o = *opt;
    o.device = f->device;
    o.stream = st;
    int rc = h2dlp_build_ex(&surf, &o, &f->bop);
    if (rc != H2DLP_OK) return rc;
    // incidence (node -> tetrahedron * 4 + local vertex) and the stiffness pattern
    std::vector<int64_t> inc_off(size_t(n) + 1, 0);
    for (int64_t q = 0; q < 4 * T; ++q) ++inc_off[size_t(vol->tet[q]) + 1];
    for (int64_t i = 0; i < n; ++i) inc_off[i + 1] += inc_off[i];
    std::vector<int32_t> inc(size_t(4 * T));
    {
        std::vector<int64_t> fill(inc_off.begin(), inc_off.end() - 1);
        for (int64_t t = 0; t < T; ++t)
            for (int a = 0; a < 4; ++a) inc[size_t(fill[vol->tet[4 * t + a]]++)] = int32_t(4 * t + a);
    }
    std::vector<int64_t> rowptr(size_t(n) + 1, 0);
    std::vector<int32_t> col;
    col.reserve(size_t(16 * n));
    std::vector<int32_t> row;
    for (int64_t i = 0; i < n; ++i) {
        row.clear();
        for (int64_t e = inc_off[i]; e < inc_off[i + 1]; ++e)
            for (int b = 0; b < 4; ++b) row.push_back(vol->tet[4 * int64_t(inc[e] >> 2) + b]);
        if (row.empty()) row.push_back(int32_t(i));       // a node of no tetrahedron: its own row only
        std::sort(row.begin(), row.end());
        row.erase(std::unique(row.begin(), row.end()), row.end());
        col.insert(col.end(), row.begin(), row.end());
        rowptr[i + 1] = int64_t(col.size());
    }
    f->nnz = int64_t(col.size());
    // sliced ELL: slices of kSlice rows, each as wide as its longest row
    const int64_t n_slices = (n + kSlice - 1) / kSlice;
    std::vector<int64_t> ell_off(size_t(n_slices) + 1, 0);
    std::vector<int32_t> ell_w(size_t(n_slices), 0);
    for (int64_t sl = 0; sl < n_slices; ++sl) {
        int64_t w = 0;
        for (int64_t i = sl * kSlice; i < std::min(n, (sl + 1) * kSlice); ++i) w = std::max(w, rowptr[i + 1] - rowptr[i]);
        ell_w[sl] = int32_t(w);
        ell_off[sl + 1] = ell_off[sl] + w * kSlice;
    }
    std::vector<int32_t> ell_col(static_cast<size_t>(ell_off[n_slices]));
    for (int64_t sl = 0; sl < n_slices; ++sl)
        for (int64_t r = 0; r < kSlice; ++r) {
            const int64_t i = std::min(sl * kSlice + r, n - 1);      // rows past n repeat the last one
            for (int64_t k = 0; k < ell_w[sl]; ++k) {
                const int64_t e = rowptr[i] + k;
                ell_col[size_t(ell_off[sl] + kSlice * k + r)] = e < rowptr[i + 1] ? col[size_t(e)] : int32_t(i);
            }
        }
    f->ell_entries = ell_off[n_slices];
    std::vector<uint8_t> on_b(size_t(n), 0);
    for (int32_t v : f->bnodes) on_b[v] = 1;
    // device: geometry, stiffness, diagonals
    std::vector<double> xyz(vol->xyz, vol->xyz + 3 * n);
    std::vector<int32_t> tet(vol->tet, vol->tet + 4 * T);
    double* d_xyz = f->upload(xyz, st);
    f->d_tet = f->upload(tet, st);
    f->d_geo = f->alloc<double>(size_t(kGeo) * size_t(T));
    f->d_inc_off = f->upload(inc_off, st);
    f->d_inc = f->upload(inc, st);
    int64_t* d_rowptr = f->upload(rowptr, st);
    int32_t* d_col = f->upload(col, st);
    double* d_val = f->alloc<double>(col.size());
    f->d_ell_off = f->upload(ell_off, st);
    f->d_ell_w = f->upload(ell_w, st);
    f->d_ell_col = f->upload(ell_col, st);
    f->d_ell_val = f->alloc<double>(ell_col.size());
    f->d_dinv_free = f->alloc<double>(size_t(n));
    f->d_dinv_fix = f->alloc<double>(size_t(n));
    uint8_t* d_onb = f->upload(on_b, st);
    f->d_bnode = f->upload(f->bnodes, st);
    hcheck(fem_geometry(T, d_xyz, f->d_tet, f->d_geo, st), "element geometry");
    hcheck(fem_stiffness(n, f->d_inc_off, f->d_inc, f->d_tet, f->d_geo, d_rowptr, d_col, d_val, st), "stiffness");
    hcheck(fem_dinv(n, d_rowptr, d_col, d_val, d_onb, f->d_dinv_free, f->d_dinv_fix, st), "diagonal");
    hcheck(fem_to_ell(n, d_rowptr, d_val, f->cg(f->d_dinv_free), f->d_ell_val, st), "sliced ELL");
    for (double** v : {&f->d_b, &f->d_r, &f->d_z, &f->d_p, &f->d_q, &f->d_ones, &f->d_u1, &f->d_u2, &f->d_g,
                       &f->d_z2, &f->d_dk})
        *v = f->alloc<double>(size_t(n));
    f->d_ub1 = f->alloc<double>(f->bnodes.size());
    f->d_ub2 = f->alloc<double>(f->bnodes.size());
    f->d_part = f->alloc<double>(size_t(kSpmvBlocks) + 2 * size_t(kFemBlocks));
    f->d_S = f->alloc<double>(kSlots);
    std::vector<double> ones(size_t(n), 1.0);
    hcheck(hipMemcpyAsync(f->d_ones, ones.data(), sizeof(double) * size_t(n), hipMemcpyHostToDevice, st), "upload");
    if (hipHostMalloc(reinterpret_cast<void**>(&f->h_S), sizeof(double) * kSlots, hipHostMallocDefault) != hipSuccess) {
        f->h_S = nullptr;
        throw std::bad_alloc();
    }
    // the spectrum bound of D^-1 A for the preconditioner (it bounds the
    // Dirichlet system's too: its rows are a subset with fewer columns)
    hcheck(fem_gershgorin(f->cg(f->d_dinv_free), f->d_part, f->d_S, kSlotLambda, st), "spectrum bound");
    hcheck(hipMemcpyAsync(f->h_S, f->d_S, sizeof(double) * kSlots, hipMemcpyDeviceToHost, st), "spectrum bound");
    hcheck(hipStreamSynchronize(st), "build");
    f->lambda_max = f->h_S[kSlotLambda] > 0.0 && std::isfinite(f->h_S[kSlotLambda]) ? f->h_S[kSlotLambda] : 0.0;
    // build-only arrays: coordinates, boundary flags and the CSR form
    for (void* p : {static_cast<void*>(d_xyz), static_cast<void*>(d_onb), static_cast<void*>(d_rowptr),
                    static_cast<void*>(d_col), static_cast<void*>(d_val)})
        f->release(p);
    return H2DLP_OK;
}

// kCheckEvery CG iterations (an even count, so the r.z slots alternate the
// same way in every block of them) captured as one graph of kernels; NULL
// when capture is not available (the iterations are then launched one by one)
hipGraphExec_t capture_steps(h2dlp_fem_ctx* f, const FemCg& c, double* x) {
    static_assert(kCheckEvery % 2 == 0, "the r.z slot parity repeats every two iterations");
    if (!f->cap && hipStreamCreateWithFlags(&f->cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        f->cap = nullptr;
        return nullptr;
    }
    if (hipStreamBeginCapture(f->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    bool ok = true;
    for (int q = 0; q < kCheckEvery; ++q) ok = ok && fem_cg_step(c, x, q, f->cap) == hipSuccess;
    hipGraph_t g = nullptr;
    ok = hipStreamEndCapture(f->cap, &g) == hipSuccess && ok;
    hipGraphExec_t e = nullptr;
    if (ok && g && hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) e = nullptr;
    if (g) (void)hipGraphDestroy(g);
    if (!e) (void)hipGetLastError();
    return e;
}

// Preconditioned CG (Chebyshev steps on D^-1 A, fem.h) from zero on the rows
// with dinv != 0; returns the iterations and the relative residual |r| / |r0|.
// `graph`: kCheckEvery iterations of this solve as one graph, or NULL.
int cg_solve(h2dlp_fem_ctx* f, const FemCg& c, const double* b, double* x, double tol, int max_iter, hipStream_t st,
             hipGraphExec_t graph, int* iters, double* rel) {
    hcheck(fem_cg_start(c, b, x, st), "cg");
    hcheck(hipMemcpyAsync(f->h_S, f->d_S, sizeof(double) * kSlots, hipMemcpyDeviceToHost, st), "cg");
    hcheck(hipStreamSynchronize(st), "cg");
    const double rr0 = f->h_S[kSlotRR];
    *iters = 0;
    *rel = 0.0;
    if (!(rr0 > 0.0)) return H2DLP_OK;      // zero right side: x = 0
    int it = 0;
    while (it < max_iter) {
        const int steps = std::min(kCheckEvery, max_iter - it);
        if (graph && steps == kCheckEvery) {          // it is a multiple of kCheckEvery here
            hcheck(hipGraphLaunch(graph, st), "cg graph");
            it += steps;
        } else {
            for (int q = 0; q < steps; ++q, ++it) hcheck(fem_cg_step(c, x, it, st), "cg");
        }
        hcheck(hipMemcpyAsync(f->h_S, f->d_S, sizeof(double) * kSlots, hipMemcpyDeviceToHost, st), "cg");
        hcheck(hipStreamSynchronize(st), "cg");
        *rel = std::sqrt(std::max(0.0, f->h_S[kSlotRR]) / rr0);
        if (*rel <= tol) break;
    }
    *iters = it;
    return H2DLP_OK;
}

int fem_field_impl(h2dlp_fem_ctx* f, const double* m, double* h, double* u1_out, double* u2_out, double tol,
                   int max_iter, hipStream_t st, h2dlp_fem_result* res) {
    const int64_t n = f->n;
    h2dlp_fem_result r{};
    if (!f->graphs_tried) {
        f->graphs_tried = true;
        f->g_u1 = capture_steps(f, f->cg(f->d_dinv_free), f->d_u1);
        f->g_u2 = capture_steps(f, f->cg(f->d_dinv_fix), f->d_u2);
    }
    // u1: the Neumann problem, right side moved to zero sum, solution to zero node sum
    hcheck(fem_rhs(n, f->d_inc_off, f->d_inc, f->d_geo, m, f->d_b, st), "right side");
    hcheck(fem_dot(n, f->d_b, f->d_ones, f->d_part, f->d_S, kSlotMean, 1.0 / double(n), st), "mean");
    hcheck(fem_shift(n, f->d_b, f->d_S, kSlotMean, st), "mean");
    int rc = cg_solve(f, f->cg(f->d_dinv_free), f->d_b, f->d_u1, tol, max_iter, st, f->g_u1, &r.iters_u1,
                      &r.resid_u1);
    if (rc != H2DLP_OK) return rc;
    hcheck(fem_dot(n, f->d_u1, f->d_ones, f->d_part, f->d_S, kSlotMean, 1.0 / double(n), st), "mean");
    hcheck(fem_shift(n, f->d_u1, f->d_S, kSlotMean, st), "mean");
    // u2 on the boundary: the boundary operator (Section 3, eq. mainInt)
    const int64_t nb = int64_t(f->bnodes.size());
    hcheck(fem_gather(nb, f->d_bnode, f->d_u1, f->d_ub1, st), "gather");
    rc = apply_entry(f->bop, f->d_ub1, f->d_ub2, 1, H2DLP_IO_F64, st, nullptr, 0, false);
    if (rc != H2DLP_OK) return rc;
    // u2 in the volume: A x = -A g on the interior nodes, u2 = x + g
    hcheck(fem_scatter(n, nb, f->d_bnode, f->d_ub2, f->d_g, st), "scatter");
    const FemCg cd = f->cg(f->d_dinv_fix);
    hcheck(fem_spmv(cd, f->d_g, f->d_q, st), "Dirichlet right side");
    hcheck(fem_scale(n, -1.0, f->d_q, f->d_b, st), "Dirichlet right side");
    rc = cg_solve(f, cd, f->d_b, f->d_u2, tol, max_iter, st, f->g_u2, &r.iters_u2, &r.resid_u2);
    if (rc != H2DLP_OK) return rc;
    hcheck(fem_axpy(n, f->d_u2, 1.0, f->d_g, f->d_u2, st), "u2");
    // H = -grad (u1 + u2) and the energy
    hcheck(fem_field(f->n_tets, f->d_tet, f->d_geo, f->d_u1, f->d_u2, m, h, f->d_part, f->d_S, kSlotEnergy, st),
           "field");
    if (u1_out) hcheck(hipMemcpyAsync(u1_out, f->d_u1, sizeof(double) * size_t(n), hipMemcpyDeviceToDevice, st), "u1");
    if (u2_out) hcheck(hipMemcpyAsync(u2_out, f->d_u2, sizeof(double) * size_t(n), hipMemcpyDeviceToDevice, st), "u2");
    hcheck(hipMemcpyAsync(f->h_S, f->d_S, sizeof(double) * kSlots, hipMemcpyDeviceToHost, st), "energy");
    hcheck(hipStreamSynchronize(st), "field");
    r.energy = f->h_S[kSlotEnergy];
    if (res) *res = r;
    return H2DLP_OK;
}

}  // namespace

extern "C" {

int h2dlp_fem_build(const h2dlp_volume* vol, const h2dlp_options* opt, h2dlp_fem* out) {
    if (!out) return set_error(H2DLP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!vol || !opt) return set_error(H2DLP_EINVAL, "volume or options is NULL");
    if (!vol->xyz || !vol->tet) return set_error(H2DLP_EINVAL, "volume arrays are NULL");
    if (vol->n_nodes < 4 || vol->n_tets < 1) return set_error(H2DLP_EINVAL, "volume needs at least 4 nodes and a tetrahedron");
    if (vol->n_nodes > (int64_t(1) << 30) || vol->n_tets > (int64_t(1) << 28))
        return set_error(H2DLP_ENOTSUP, "volume larger than 2^30 nodes or 2^28 tetrahedra");
    for (int64_t q = 0; q < 4 * vol->n_tets; ++q)
        if (vol->tet[q] < 0 || vol->tet[q] >= vol->n_nodes) return set_error(H2DLP_EINVAL, "tetrahedron node out of range");
    for (int64_t t = 0; t < vol->n_tets; ++t) {
        const int32_t* v = vol->tet + 4 * t;
        const double* a = vol->xyz + 3 * int64_t(v[0]);
        double e[3][3];
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) e[c][d] = vol->xyz[3 * int64_t(v[c + 1]) + d] - a[d];
        const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                           e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                           e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
        if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return set_error(H2DLP_EINVAL, "degenerate tetrahedron");
    }
    std::unique_ptr<h2dlp_fem_ctx> f(new (std::nothrow) h2dlp_fem_ctx);
    if (!f) return set_error(H2DLP_ENOMEM, "host allocation failed");
    int dev = opt->device;
    const int drc = gfx950_device(&dev);
    if (drc != H2DLP_OK) return drc;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(dev) != hipSuccess)
        return set_error(H2DLP_EDEVICE, "hipSetDevice failed");
    f->device = dev;
    int rc;
    try {
        rc = fem_build_impl(f.get(), vol, opt, static_cast<hipStream_t>(opt->stream));
    } catch (const FemError& e) {
        rc = set_error(H2DLP_EDEVICE, e.where + ": " + hipGetErrorString(e.err));
    } catch (const std::bad_alloc&) {
        rc = set_error(H2DLP_ENOMEM, "device or host allocation failed");
    }
    if (rc != H2DLP_OK) {
        f.reset();
        (void)hipSetDevice(cur);
        return rc;
    }
    (void)hipSetDevice(cur);
    *out = reinterpret_cast<h2dlp_fem>(f.release());
    return H2DLP_OK;
}

int h2dlp_fem_info(h2dlp_fem ff, int64_t* n_boundary, int64_t* nnz, size_t* device_bytes, h2dlp_handle* boundary_op) {
    const h2dlp_fem_ctx* f = as_fem(ff);
    if (!f) return set_error(H2DLP_EINVAL, "handle is NULL");
    if (n_boundary) *n_boundary = int64_t(f->bnodes.size());
    if (nnz) *nnz = f->nnz;
    if (device_bytes) *device_bytes = f->bytes;
    if (boundary_op) *boundary_op = f->bop;
    return H2DLP_OK;
}

int h2dlp_fem_boundary_nodes(h2dlp_fem ff, int64_t* nodes) {
    const h2dlp_fem_ctx* f = as_fem(ff);
    if (!f) return set_error(H2DLP_EINVAL, "handle is NULL");
    if (!nodes) return set_error(H2DLP_EINVAL, "nodes is NULL");
    for (size_t j = 0; j < f->bnodes.size(); ++j) nodes[j] = f->bnodes[j];
    return H2DLP_OK;
}

int h2dlp_fem_field(h2dlp_fem ff, const double* m, double* h, double* u1, double* u2, double tol, int max_iter,
                    void* stream, h2dlp_fem_result* res) {
    h2dlp_fem_ctx* f = as_fem(ff);
    if (!f) return set_error(H2DLP_EINVAL, "handle is NULL");
    if (!m || !h) return set_error(H2DLP_EINVAL, "m or h is NULL");
    if (!(tol > 0.0) || max_iter < 1) return set_error(H2DLP_EINVAL, "tol must be > 0 and max_iter >= 1");
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (hipSetDevice(f->device) != hipSuccess) return set_error(H2DLP_EDEVICE, "hipSetDevice failed");
    const size_t vb = sizeof(double) * size_t(3 * f->n_tets), nbytes = sizeof(double) * size_t(f->n);
    struct Arg { const void* p; size_t bytes; const char* name; };
    for (const Arg& a : {Arg{m, vb, "m"}, Arg{h, vb, "h"}, Arg{u1, nbytes, "u1"}, Arg{u2, nbytes, "u2"}}) {
        std::string why;
        if (a.p && !device_memory_ok(a.p, a.bytes, f->device, a.name, &why)) {
            (void)hipSetDevice(cur);
            return set_error(H2DLP_EINVAL, why);
        }
    }
    int rc;
    try {
        rc = fem_field_impl(f, m, h, u1, u2, tol, max_iter, static_cast<hipStream_t>(stream), res);
    } catch (const FemError& e) {
        rc = set_error(H2DLP_EDEVICE, e.where + ": " + hipGetErrorString(e.err));
    }
    (void)hipSetDevice(cur);
    return rc;
}

void h2dlp_fem_free(h2dlp_fem f) { delete as_fem(f); }

}  // extern "C"
