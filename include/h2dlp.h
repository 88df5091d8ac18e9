/*
 * h2dlp -- H2-compressed boundary double-layer operator of the Fredkin-Koehler
 * FEM/BEM magnetostatic method, on AMD Instinct MI355X (gfx950).
 *
 * The operator (Hertel, Christophersen & Boerm, arXiv:1811.05731, Section 3,
 * eqs. matrix_definition and denseMat) maps the boundary trace u1 of the
 * Neumann potential to the Dirichlet data u2 of the harmonic part,
 *
 *     u2 = M u1 = (K + D) u1,
 *     K_ij = (1/4pi) int phi_j(y) n(y).(xi_i - y)/|xi_i - y|^3 dS_y,
 *     D_ii = Psi(xi_i)/(4 pi) - 1,
 *
 * with collocation at the mesh nodes xi_i, P1 hat functions phi_j and the
 * interior solid angle Psi.  K is held as an H2 matrix (Section 4): tensor
 * Chebyshev interpolation of order m on a bounding-box cluster tree with
 * eta-admissibility; inadmissible leaf blocks hold exact entries.
 *
 * Conventions shared by every call:
 *  - No call throws; every failure returns a negative code and leaves a
 *    message for h2dlp_last_error() (thread-local).
 *  - Host pointers are read during the call only; the caller keeps ownership.
 *  - Device pointers (u1, u2, workspace) are HIP device memory on the handle's
 *    device, owned by the caller.
 */
#ifndef H2DLP_H
#define H2DLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define H2DLP_OK       0
#define H2DLP_EINVAL  -1   /* bad argument, bad mesh (see h2dlp_last_error) */
#define H2DLP_ENOMEM  -2   /* device allocation failed or workspace too small */
#define H2DLP_EDEVICE -3   /* a HIP runtime call failed */
#define H2DLP_ENOTSUP -4   /* precision / device / size not supported */

/* arithmetic of the compressed operator (coupling, bases, transfers, near blocks) */
#define H2DLP_FP64    0    /* everything in FP64 */
#define H2DLP_FP32    1    /* FP32 storage and accumulation; FP64 diagonal and near-singular entries */
#define H2DLP_BF16X3  2    /* as FP32, coupling products as split bf16 x3 on MFMA, FP32 accumulation */
#define H2DLP_BF16X6  3    /* as BF16X3 with three-term splits and six products (6 bytes per coupling entry) */

/* element type of u1 / u2 */
#define H2DLP_IO_F64  0
#define H2DLP_IO_F32  1

/* Closed, consistently oriented triangle surface (Section 3: nodes xi_i and the
 * P1 basis on the boundary of the magnetic body).  xyz: n_nodes x 3 row-major
 * FP64; tri: n_tris x 3 row-major, 0-based node indices, counter-clockwise seen
 * from outside (outward normals).  Both host memory. */
typedef struct {
    int64_t        n_nodes;
    const double*  xyz;
    int64_t        n_tris;
    const int32_t* tri;
} h2dlp_mesh;

/* Build parameters.  order m in [1, 8] (k = m^3 interpolation points per
 * cluster); leaf in [1, 64] (maximum leaf cluster size); eta > 0
 * (admissibility max(diam_t, diam_s) <= eta dist(t, s)); alpha in [0, 1]
 * (each cluster box side is widened to at least alpha times its longest side);
 * device: HIP ordinal or -1 for the current device; stream: hipStream_t for the
 * build kernels, NULL for the null stream.
 * coupling: H2DLP_COUPLING_STORED keeps every coupling matrix S_ts in device
 * memory (k^2 values per admissible block, read once per apply);
 * H2DLP_COUPLING_GENERATED keeps only each cluster's box and recomputes
 * S_ts(nu, mu) = 1/(4 pi |eta^t_nu - eta^s_mu|) (Section 4: the kernel at the
 * interpolation points) inside the apply, from the FP64 difference of the box
 * centres plus the two points' offsets; the same operator without the
 * coupling bytes (FP64 and FP32 precision, order <= 5; else ENOTSUP).
 * dense_far_max >= 0: an admissible block with |t| |s| <= dense_far_max is
 * stored as its exact entries (Section 3, like an inadmissible block) instead
 * of through the cluster bases and a k x k coupling matrix: cheaper when
 * |t| |s| is small against k^2, and exact.  0 keeps every admissible block
 * low-rank (the plain H2 matrix).
 * recompress_eps: 0 keeps the interpolation bases.  In (0, 1) the build
 * recompresses the matrix algebraically (Section 4: the conversion to an H2
 * matrix whose ranks follow the accuracy): the row and column bases become
 * orthonormal nested bases of adaptive rank, from SVDs of each cluster's
 * basis weighted by every low-rank block it serves, truncated at
 * recompress_eps times the cluster's largest singular value, and every
 * coupling matrix is projected onto them and stored (r_t x r_s).  FP64 and
 * FP32, stored coupling, order <= 5 (else ENOTSUP).  h2dlp_plan reports the
 * interpolation sizes (an upper bound); the ranks are known after the build.
 * row_basis: H2DLP_ROW_BASIS_STORED keeps every leaf row basis V_t (n_t x k
 * values, Section 4: V_t(i, nu) is the nu-th Lagrange polynomial of the leaf
 * box's Chebyshev points at node xi_i).  H2DLP_ROW_BASIS_GENERATED keeps only
 * the node coordinates (24 bytes a node instead of k values) and evaluates
 * V_t inside the apply: the same operator without the row-basis bytes.
 * Interpolation bases only (recompress_eps 0, else ENOTSUP). */
typedef struct {
    int    order;
    int    leaf;
    double eta;
    int    precision;
    double alpha;
    int    device;
    void*  stream;
    int    coupling;
    int64_t dense_far_max;
    double recompress_eps;
    int    row_basis;
} h2dlp_options;

#define H2DLP_COUPLING_STORED     0
#define H2DLP_COUPLING_GENERATED  1

#define H2DLP_ROW_BASIS_STORED     0
#define H2DLP_ROW_BASIS_GENERATED  1

typedef struct h2dlp_ctx* h2dlp_handle;

/* Sizes of a built operator. */
typedef struct {
    int64_t n_nodes, n_tris;
    int32_t order, leaf, k, precision;
    int32_t depth;              /* deepest cluster level (root = 0) */
    int64_t n_clusters, n_leaves;
    int64_t n_far, n_near;      /* low-rank admissible blocks, inadmissible leaf blocks */
    int64_t coupling_entries;   /* n_far * k * k (sum of r_t r_s when recompressed) */
    int64_t near_entries;       /* sum over near blocks of |t| |s| */
    int64_t nearsing_entries;   /* near-singular entries kept in FP64 (all but FP64) */
    int64_t bytes_coupling, bytes_near, bytes_bases, bytes_transfer, bytes_other;
    int64_t bytes_resident;     /* all device memory held by the handle */
    int64_t workspace_bytes;    /* per concurrent apply (one 16-column pass) */
    double  compression;        /* 1 - (H2 bytes)/(8 N^2), the paper's ratio r (Section 6.1) */
    int64_t n_far_dense;        /* admissible blocks stored as exact entries (dense_far_max) */
    int64_t dense_far_entries;  /* their entries (counted in bytes_near, not in near_entries) */
    int64_t rank_sum_row;       /* sum over clusters of the row / column basis ranks (k each */
    int64_t rank_sum_col;       /*   without recompression)                                 */
    int32_t rank_max_row, rank_max_col;
} h2dlp_stats;

/* Fill *opt with defaults: order 4, leaf 32, eta 2, FP64, alpha 0.1, device -1,
 * stream NULL, coupling STORED, dense_far_max 0, recompress_eps 0, row_basis
 * STORED. */
void h2dlp_default_options(h2dlp_options* opt);

/* Build the H2 operator for `mesh` (copied; the caller may free it on return).
 * The handle owns its device memory until h2dlp_free.  Returns NULL on error. */
h2dlp_handle h2dlp_build(const h2dlp_mesh* mesh, int order, int leaf, double eta);

/* As h2dlp_build with full options; *out receives the handle.  Errors:
 * EINVAL (NULL pointers, order/leaf/eta/alpha out of range, index out of range,
 * repeated vertex or zero-area triangle, open or non-manifold edge, inconsistent
 * orientation, non-positive enclosed volume, coincident nodes), ENOMEM, EDEVICE,
 * ENOTSUP (no gfx950 device). */
int h2dlp_build_ex(const h2dlp_mesh* mesh, const h2dlp_options* opt, h2dlp_handle* out);

/* Host-only planning: the block structure and every byte count of h2dlp_stats
 * for `mesh` and `opt`, without touching a GPU (no HIP call).  The handle
 * supports h2dlp_info, h2dlp_bytes, h2dlp_export_structure and h2dlp_free;
 * apply on it returns EINVAL.  Meant for admission by HBM budget before a
 * build, and for checking the structure.  Errors as h2dlp_build_ex, without
 * EDEVICE/ENOTSUP for the device. */
int h2dlp_plan(const h2dlp_mesh* mesh, const h2dlp_options* opt, h2dlp_handle* out);

/* u2 = M u1 for nrhs right-hand sides (eq. denseMat).  u1, u2: device, FP64,
 * (nrhs, n_nodes) row-major, one contiguous vector per right-hand side, in the
 * caller's node order; must not overlap.  Asynchronous on the null stream, using
 * the handle's own workspace (not safe to call concurrently on one handle).
 * Errors: EINVAL (NULL, nrhs < 1, u1 or u2 not device memory of the handle's
 * GPU or ending before nrhs * n_nodes values), EDEVICE. */
int h2dlp_apply(h2dlp_handle h, const double* u1, double* u2, int nrhs);

/* As h2dlp_apply, with io_dtype (H2DLP_IO_F64 / H2DLP_IO_F32), a hipStream_t
 * (NULL = null stream) and a caller-owned device workspace of at least
 * h2dlp_stats.workspace_bytes (NULL = the handle's own).  Distinct workspaces
 * make concurrent applies of one handle on different streams safe.  Right-hand
 * sides are processed 16 at a time.  Errors: EINVAL (as h2dlp_apply; also a
 * workspace that is not device memory of the handle's GPU or whose allocation
 * ends before h2dlp_stats.workspace_bytes), ENOMEM (workspace_bytes too small),
 * EDEVICE. */
int h2dlp_apply_ex(h2dlp_handle h, const void* u1, void* u2, int nrhs, int io_dtype,
                   void* stream, void* workspace, size_t workspace_bytes);

/* Allocation-free apply, for callers that cannot allocate device memory: code
 * under HIP graph capture, fixed serving loops, harnesses that forbid
 * hipMalloc.  As h2dlp_apply_ex, with the workspace in a device array of the
 * library instead of the handle's or the caller's: H2DLP_NOALLOC_SCRATCH_BYTES
 * (128 MiB) per GPU, held from the load of the library until the process
 * ends.  The call allocates nothing (no hipMalloc, hipFree, stream or event
 * creation); its first use on a device looks up the array's address there.
 * All calls on one GPU share that GPU's array and it keeps the last call's
 * contents (nothing in it needs to start at zero): calls that overlap on one
 * GPU -- other streams, threads or handles -- race, so the caller runs them one
 * after another.  Profiling (h2dlp_profile) creates events: keep it off here.
 * Errors: as h2dlp_apply_ex; ENOMEM when h2dlp_stats.workspace_bytes exceeds
 * H2DLP_NOALLOC_SCRATCH_BYTES (use h2dlp_apply_ex with a workspace then). */
#define H2DLP_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
int h2dlp_apply_noalloc(h2dlp_handle h, const void* u1, void* u2, int nrhs, int io_dtype, void* stream);

/* Device bytes held by the handle and needed per concurrent apply (admission by HBM budget). */
int h2dlp_bytes(h2dlp_handle h, size_t* resident, size_t* workspace);

int h2dlp_info(h2dlp_handle h, h2dlp_stats* st);

/* Copy out the block structure (host arrays, sizes from h2dlp_info), in the
 * preorder numbering of the cluster tree (root 0, first child's subtree first):
 *   perm[n_nodes]          node index of each position in cluster order
 *   clusters[n_clusters*6] begin, end, level, parent, child0, child1 (-1 = none)
 *   boxes[n_clusters*6]    lo_x, lo_y, lo_z, hi_x, hi_y, hi_z of the inflated box
 *   far[n_far*2], near[n_near*2]  (target, source) cluster pairs, sorted;
 *                          far lists the low-rank admissible blocks only
 * Any pointer may be NULL to skip that array. */
int h2dlp_export_structure(h2dlp_handle h, int64_t* perm, int64_t* clusters, double* boxes,
                           int64_t* far, int64_t* near);

/* The diagonal D_ii = Psi_i/(4 pi) - 1 as computed on the device (host array, node order). */
int h2dlp_export_diagonal(h2dlp_handle h, double* diag);

/* Free the operator's device memory, keeping it in pinned host memory, and
 * bring it back: an operator evicted to make room for others returns without
 * a rebuild.  The operator does not change after the build, so the first
 * offload copies it to the host once and keeps that copy until h2dlp_free;
 * later offloads only free, reloads copy host to device.  h2dlp_offload
 * synchronises the device; h2dlp_reload returns when the copies are done.
 * h2dlp_reload_ex only enqueues the copies on `stream` (a hipStream_t, NULL =
 * the default stream) and returns: every later apply, on any stream, waits for
 * them on the device, so the caller may launch at once.  Apply on an offloaded
 * handle returns EINVAL.  All three are no-ops in the target state.  Errors:
 * EINVAL (plan-only handle), ENOMEM (pinned host or device allocation; reload
 * then leaves the handle offloaded), EDEVICE. */
int h2dlp_offload(h2dlp_handle h);
int h2dlp_reload(h2dlp_handle h);
int h2dlp_reload_ex(h2dlp_handle h, void* stream);

/* Persistence (Section 6.1: the H2 matrix is computed once per geometry,
 * stored to a file and read back at later starts instead of being rebuilt).
 * h2dlp_save writes a built operator (an offloaded one too) to `path`: its
 * mesh, build options, the host state its recompression derived and every
 * device buffer, in host byte order.  EINVAL: the handle comes from
 * h2dlp_plan, or the file cannot be written; EDEVICE: a device copy failed.
 * h2dlp_load restores such a file on `device` (-1: the current device)
 * without building: the host structure is planned again from the stored mesh
 * and options (it is deterministic) and the device buffers are copied from the
 * file, so applies give the saved operator's results bit for bit.  *out
 * receives a handle like h2dlp_build_ex's (NULL on error).  EINVAL: path
 * missing or unreadable, not an operator file, truncated or inconsistent with
 * its own mesh; ENOTSUP: written by another version of this library, or the
 * device is not a gfx950; ENOMEM: device or pinned host memory ran out.  The
 * file is this library's own layout, not an exchange format. */
int h2dlp_save(h2dlp_handle h, const char* path);
int h2dlp_load(const char* path, int device, h2dlp_handle* out);

/* Finite-element solves either side of the boundary operator: one
 * evaluation of the magnetostatic field of a magnetised body (Section 2,
 * eqs. u1Poiss, u1Neumann, mainInt, u2diri):
 *     Delta u1 = div M in the body, du1/dn = M.n on its surface;
 *     u2 = (K + D) u1 on the surface (this library's operator);
 *     Delta u2 = 0 in the body with those values;  H = -grad (u1 + u2),
 *     E = -(1/2) int M.H  (units mu0 = 1; M in units of Ms).
 * Continuous P1 elements on tetrahedra, M constant per tetrahedron; u1 from
 * the weak form int grad u1 . grad v = int M . grad v with zero node sum;
 * both linear systems by Jacobi-preconditioned conjugate gradients in FP64
 * on the GPU (the paper names a GPU Krylov solver for large meshes).
 *
 * The volume: n_nodes x 3 FP64 coordinates and n_tets x 4 node indices
 * (0-based, either orientation, none degenerate), host memory. */
typedef struct {
    int64_t        n_nodes;
    const double*  xyz;
    int64_t        n_tets;
    const int32_t* tet;
} h2dlp_volume;

typedef struct h2dlp_fem_ctx* h2dlp_fem;

typedef struct {
    int32_t iters_u1, iters_u2;     /* CG iterations of the two solves */
    double  resid_u1, resid_u2;     /* final |r| / |r0| of the two solves */
    double  energy;                 /* -(1/2) sum_t vol_t M_t . H_t */
} h2dlp_fem_result;

/* Build: the surface (faces of one tetrahedron only, oriented outward), the
 * boundary operator on it with `opt` (order, leaf, eta, precision, coupling,
 * dense_far_max, recompress_eps, row_basis; device and stream as for h2dlp_build_ex),
 * the P1 stiffness matrix and the element geometry.  The volume is copied.
 * EINVAL for a bad volume (index out of range, degenerate tetrahedron, no
 * closed surface), else the errors of h2dlp_build_ex. */
int h2dlp_fem_build(const h2dlp_volume* vol, const h2dlp_options* opt, h2dlp_fem* out);
/* Sizes: boundary nodes, stiffness entries, device bytes of the FEM part,
 * and the boundary operator (owned by the handle: do not free it).  Any
 * pointer may be NULL. */
int h2dlp_fem_info(h2dlp_fem f, int64_t* n_boundary, int64_t* nnz, size_t* device_bytes,
                   h2dlp_handle* boundary_op);
/* The boundary nodes in the volume numbering, ascending (n_boundary values):
 * the boundary operator's node j is volume node nodes[j]. */
int h2dlp_fem_boundary_nodes(h2dlp_fem f, int64_t* nodes);
/* One field evaluation on `stream` (a hipStream_t, NULL = null stream).
 * m: n_tets x 3 FP64 device array (M per tetrahedron); h: n_tets x 3 FP64
 * device array, receives H; u1, u2: n_nodes FP64 device arrays for the two
 * potentials, or NULL.  Both solves are conjugate gradients in FP64, each
 * iteration preconditioned by six Chebyshev steps on D^-1 A (D the diagonal,
 * spectrum bounded by Gershgorin at build); each stops at |r| <= tol |r0| or
 * after max_iter iterations; *res (may be NULL) receives the iterations, residuals and the
 * energy.  Returns when the evaluation is done.  EINVAL for a NULL handle,
 * m or h, a pointer that is not device memory of the handle's GPU, tol <= 0
 * or max_iter < 1; EDEVICE when a HIP call fails. */
int h2dlp_fem_field(h2dlp_fem f, const double* m, double* h, double* u1, double* u2, double tol, int max_iter,
                    void* stream, h2dlp_fem_result* res);
void h2dlp_fem_free(h2dlp_fem f);

void h2dlp_free(h2dlp_handle h);

const char* h2dlp_last_error(void);

/* Kernel timing with hipEvents recorded around the launches of the apply, on
 * the stream each launch goes to.  Kinds: 0 permute, 1 leaf forward, 2 upward
 * transfer, 3 coupling, 4 downward transfer, 5 leaf backward V_t yhat_t (+
 * un-permute), 6 near field + diagonal.  The near field runs on a stream of
 * the handle's own, concurrently with kinds 3 and 4, so kind times overlap.  `enable` is a bit mask: bit q records kind q
 * (0 = off, H2DLP_PROFILE_ALL = every kind); record only the kinds you need,
 * since every event pair adds a little time to the stream.
 * h2dlp_profile_read synchronises the recorded events and returns the summed
 * milliseconds and launch counts per kind (n_kinds <= 7). */
#define H2DLP_NKINDS 7
#define H2DLP_PROFILE_ALL 0x7f
int h2dlp_profile(h2dlp_handle h, int enable);
int h2dlp_profile_read(h2dlp_handle h, double* ms, int64_t* launches, int n_kinds, int reset);

#ifdef __cplusplus
}
#endif

#endif /* H2DLP_H */
