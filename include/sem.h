/*
 * sem.h -- C ABI of an MI355X (gfx950) engine for the data-parallel hot path
 * of a spectral-element incompressible-flow solver: the matrix-free local
 * Poisson/Helmholtz operator on order-N hexahedra, the direct-stiffness
 * gather-scatter Q Q^T, and a Jacobi-preconditioned conjugate-gradient solve.
 *
 * Paper: "Strong Scaling of OpenACC enabled Nek5000 on several GPU based HPC
 * systems" (arXiv 2109.03592).  Section 2 defines the spectral element
 * discretisation (GLL tensor-product basis, global face exchange versus local
 * matrix-free work) and the pressure Poisson problem (Eq. 5); Algorithm 1
 * (axhelm) defines the local operator.
 *
 * Conventions for every entry point:
 *  - Returns SEM_OK (0) or a nonzero sem_status; sem_last_error() gives a
 *    thread-local message.  No C++ exception or abort crosses the ABI.
 *  - "E-vector" = one value per local node, layout [E][(N+1)^3] with the node
 *    index i + (N+1) j + (N+1)^2 k (i fastest), element e = ex + nx (ey + ny ez).
 *    This is Algorithm 1's u(lx1,ly1,lz1,e).
 *  - Pointers named "device" are HIP device pointers owned by the caller; the
 *    library never frees them.  "host" pointers are ordinary host memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Operators are
 *    enqueued asynchronously; entry points that return host data synchronise
 *    the stream first.
 *  - Everything runs in HIP kernels on the GPU; there is no CPU fallback.  A
 *    machine without a usable gfx950 device gets SEM_EHIP from sem_setup.
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int sem_status;
enum {
    SEM_OK = 0,
    SEM_EINVAL = 1,      /* bad argument or descriptor                        */
    SEM_ENOMEM = 2,      /* device or host allocation failed                  */
    SEM_EHIP = 3,        /* a HIP runtime call failed                         */
    SEM_ENOCONV = 4,     /* solve hit max_iter; x holds the last iterate      */
    SEM_EBREAKDOWN = 5,  /* CG breakdown: p.Ap <= 0 or not finite             */
    SEM_EBUDGET = 6,     /* request exceeds a memory budget or slot limit     */
    SEM_EUNSUPPORTED = 7 /* valid request the library was not built for       */
};

enum { SEM_MAP_BOX = 0, SEM_MAP_PIPE_SQ2DISK = 1 };
enum { SEM_FP64 = 0, SEM_FP32 = 1 };          /* element type of E-vectors       */
enum { SEM_PREC_FP64 = 0, SEM_PREC_MIXED = 1 }; /* solve precision               */
enum { SEM_WITH_FP32 = 1 };                   /* sem_mesh_desc.precision_flags  */
enum { SEM_MAX_ORDER = 17 };                  /* largest N with built kernels   */

typedef struct sem_mesh sem_mesh;

/* Mesh descriptor: an nel[0] x nel[1] x nel[2] lattice of hexahedra of order N.
 *  mapping SEM_MAP_BOX: each element is the trilinear image of its 8 vertices,
 *    taken from `vertices` when non-NULL ((nx+1)(ny+1)(nz+1) x 3 doubles, x
 *    fastest, host memory, read during sem_setup only) or else from the uniform
 *    lattice on [lo, hi].
 *  mapping SEM_MAP_PIPE_SQ2DISK: the square [lo0,hi0] x [lo1,hi1] (normally
 *    [-1,1]^2) is mapped to the unit disk by (X sqrt(1-Y^2/2), Y sqrt(1-X^2/2));
 *    z is uniform.  The map is singular where the square's corners are; the
 *    quadrature points there are dropped (geometric factors and mass set to 0).
 *  periodic[d]: identify the last node layer with the first along axis d.
 *  dirichlet_faces: bit 2d (2d+1) = homogeneous Dirichlet on the low (high)
 *    face of axis d; -1 = every non-periodic face.
 *  precision_flags: SEM_WITH_FP32 also builds FP32 copies of the geometric
 *    factors and the Jacobi diagonal (needed for SEM_FP32 operators and mixed
 *    solves). */
typedef struct {
    int N;
    int nel[3];
    int periodic[3];
    double lo[3], hi[3];
    int mapping;
    const double *vertices;
    int dirichlet_faces;
    int precision_flags;
} sem_mesh_desc;

typedef struct {
    int N;
    int64_t E;
    int64_t n_local;          /* E (N+1)^3                                   */
    int64_t n_global;         /* unique global nodes                          */
    int64_t n_shared_local;   /* local nodes whose global node has mult >= 2  */
    int64_t n_shared_global;  /* global nodes with mult >= 2                  */
    int64_t n_masked_global;  /* global nodes on Dirichlet faces              */
    int64_t n_unmasked_global;
    int64_t gs_plan_ids;      /* global ids the gather-scatter visits         */
    int64_t gs_plan_sum_ids;  /* the first gs_plan_sum_ids of them are summed, the
                                 rest (Dirichlet ids) are zeroed               */
    int64_t gs_plan_len;      /* local entries listed by the plan             */
    size_t device_bytes;      /* device memory held by the handle             */
} sem_mesh_info;

const char *sem_last_error(void);
const char *sem_version(void);

/* Build a mesh on the current HIP device (section 2: GLL rule, element
 * geometry, global numbering, gather-scatter plan, Jacobi diagonal) and
 * upload it.  The handle owns every device buffer it allocates.
 * Errors: SEM_EINVAL (N outside 1..SEM_MAX_ORDER, non-positive element counts,
 * degenerate geometry), SEM_ENOMEM, SEM_EHIP. */
sem_status sem_setup(const sem_mesh_desc *desc, void *stream, sem_mesh **out);
sem_status sem_free(sem_mesh *mesh);
sem_status sem_info(const sem_mesh *mesh, sem_mesh_info *info);

/* Host copies of set-up data, for checking.
 *  sem_export_gll: GLL nodes xi[N+1], weights w[N+1], D[(N+1)^2] with
 *    D[i*(N+1)+l] = derivative of the l-th Lagrange interpolant at xi_i.
 *  sem_export_maps: per local node (n_local entries each; NULL skips):
 *    glob_id (lexicographic: a + gx (b + gy c) with lattice indices
 *    a = ex N + i etc., reduced on periodic axes), mult (copies of that
 *    global node), mask (1 on Dirichlet faces).
 *  sem_export_geom: G[6][n_local] (g1..g6 = G_rr, G_ss, G_tt, G_rs, G_rt, G_st,
 *    Algorithm 1's factors with W det J folded in), B[n_local] (W det J),
 *    invdiag[n_local] (inverse assembled diagonal, 0 on masked nodes).
 *  sem_export_coords: xyz[3][n_local] node coordinates. */
sem_status sem_export_gll(int N, double *xi, double *w, double *D);
sem_status sem_export_maps(const sem_mesh *mesh, int64_t *glob_id, uint8_t *mult, uint8_t *mask);
sem_status sem_export_geom(const sem_mesh *mesh, double *G, double *B, double *invdiag);
sem_status sem_export_coords(const sem_mesh *mesh, double *xyz);

/* Host-only set-up, for checking on machines without a GPU: runs the host
 * part of sem_setup (GLL rule, coordinates, geometric factors, numbering,
 * gather-scatter plan, Jacobi diagonal) without touching any device, and
 * copies its products out.  info receives the sizes (device_bytes = 0).
 * Arrays as in the exports above; gs_off[gs_plan_ids + 1] and
 * gs_idx[gs_plan_len] receive the plan (global ids in ascending order, summed
 * ids first; each id's local copies in ascending local index).  Any array
 * pointer may be NULL. */
sem_status sem_host_setup(const sem_mesh_desc *desc, sem_mesh_info *info, int64_t *glob_id, uint8_t *mult,
                          uint8_t *mask, double *G, double *B, double *invdiag, int32_t *gs_off,
                          int32_t *gs_idx);

/* Replace the geometric factors and lumped mass of a mesh with caller-supplied
 * ones (host arrays in the sem_export_geom layout: G[6][n_local], B[n_local]),
 * e.g. factors computed by another code for the same element layout.  The
 * Jacobi diagonal and the FP32 copies are rebuilt; graphs stay valid.  A
 * Helmholtz form set by sem_set_helmholtz is dropped (its h2 B used the old B).
 * Errors: SEM_EINVAL (null pointers, non-positive assembled diagonal). */
sem_status sem_load_geometry(sem_mesh *mesh, const double *G, const double *B, void *stream);

/* Launch configuration of the local operator on this mesh: elements per
 * workgroup (1 <= epw, epw (N+1)^2 <= 512, its LDS -- 3 epw (N+1)^3 values,
 * or 3 epw (N+1)^2 for the plain and CG operators from order 8 on, which run
 * plane by plane -- within the device's per-workgroup limit, else the
 * operator calls fail with SEM_EHIP) and the number of persistent
 * workgroups (grid > 0; 0 keeps the default of 16 per compute unit).  Results
 * of sem_ax / sem_axgs do not depend on it; CG dot products do at rounding
 * level (their partial sums follow the workgroups).  Setting it applies to
 * the FP64 and FP32 operators, plain and CG; by default each precision has
 * its own count (the one that fills 64-lane waves best; for the FP64 plain
 * operator at N = 9 the measured best, five, while the CG operator keeps
 * one).  sem_get_operator_config reads the FP64 CG one. */
sem_status sem_set_operator_config(sem_mesh *mesh, int epw, int grid);
sem_status sem_get_operator_config(const sem_mesh *mesh, int *epw, int *grid);

/* Which kernel performs the gather-scatter QQ^T (section 2, the exchange and
 * summation of element face values) on this mesh, for sem_gs, sem_axgs,
 * sem_mass, every solve and the mesh's batched slots (the kind at admission):
 *   SEM_GS_AUTO (default): on the element lattice -- a global node's copies
 *     follow from its lattice position, so no plan is read -- whenever every
 *     periodic axis has at least two elements; else the plan.  On a single
 *     mesh of order 7 with at least 2048 element-row walks (the number of
 *     element rows along x times N - 1 interior planes per element layer) the
 *     nodes off the z-planes go through a kernel that streams whole element
 *     rows (same sums, same bits).
 *   SEM_GS_PLAN: the CSR plan sorted by global id.
 *   SEM_GS_STREAM: as SEM_GS_AUTO, with the row-streaming kernel at every
 *     order 2..7 whatever the mesh size (for checking it; it is slower than
 *     the per-node kernel on small meshes and at low orders).
 * Both sum a node's copies in ascending local index, from 0, and set
 * Dirichlet nodes to 0 at every copy: results are bit-identical.  Changing
 * the kind drops the captured CG iterations (re-captured on the next solve).
 * sem_get_gs_config returns the kind and whether the lattice kernel runs.
 * Errors: SEM_EINVAL (null mesh, unknown kind). */
enum { SEM_GS_AUTO = 0, SEM_GS_PLAN = 1, SEM_GS_STREAM = 2 };
sem_status sem_set_gs_config(sem_mesh *mesh, int kind);
sem_status sem_get_gs_config(const sem_mesh *mesh, int *kind, int *lattice_in_use);


/* Fused operator and gather-scatter (Algorithm 1 followed by section 2's
 * exchange of element face values, done in one launch for the faces a
 * workgroup holds).  A workgroup takes lines_per_wg consecutive x-lines of
 * elements (elements are numbered x fastest) and walks them in element order,
 * epw elements per tile.  A node on an interior t-plane (0 < k < N) whose
 * copies all lie in the workgroup -- across an x-face of one line, a y-face
 * between two of its lines, or the edge where both meet -- is summed in LDS
 * in ascending local index, the order of sem_gs, and written to every copy;
 * Dirichlet nodes are written as 0.  The remaining shared nodes (the t-planes
 * k = 0 and N, faces between workgroups, periodic x and y seams) are summed
 * by a gather-scatter launch over a residual plan.  The result is the same
 * bits as sem_ax followed by sem_gs.
 * Used by sem_axgs, the true residual of sem_pcg_solve and the Jacobi CG
 * iteration (FP64 and FP32) for orders 2..12; other settings (coarse term,
 * Schwarz, other orders) run the operator and the full gather-scatter as two
 * launches.
 * It is off by default: on the 48x48x96 pipe at N = 7 the fused apply
 * measured 1.95-1.98 ms against 1.92 ms for the two launches (the
 * line-ordered walk and the epilogue cost more than the gather-scatter
 * traffic they save).
 * sem_set_axgs_config: enable 0 (default) or 1; epw and lines_per_wg 0 pick
 * them automatically (the tile that keeps the most waves resident, then the
 * smallest line count that fills the device in one round).  It waits for the
 * device and drops cached CG graphs.  Errors: SEM_EINVAL (enable not 0/1,
 * negative counts, epw (N+1)^2 > 512, more workgroups than the partials
 * buffer holds); a tile whose LDS exceeds the device limit makes the fused
 * path unavailable (the two launches run).
 * sem_get_axgs_info: the shape in use for dtype (SEM_FP64 or SEM_FP32; built
 * on first use); enabled = 0 when the fused path does not apply. */
typedef struct {
    int enabled;              /* 1: the fused path runs for this precision     */
    int epw;                  /* elements per tile                             */
    int lines_per_wg;         /* x-lines per workgroup                         */
    int y_onchip;             /* 1: y-faces between a workgroup's lines in LDS */
    int64_t grid;             /* workgroups per launch                         */
    int64_t residual_ids;     /* global ids left to the residual launch        */
    int64_t residual_copies;  /* their local copies                            */
} sem_axgs_info;
sem_status sem_set_axgs_config(sem_mesh *mesh, int enable, int epw, int lines_per_wg);
sem_status sem_get_axgs_info(sem_mesh *mesh, int dtype, sem_axgs_info *info);
/* Host-only (for checking): the residual plan the fused path would use on the
 * mesh of desc with lines_per_wg x-lines per workgroup (y_onchip 0 or 1), in
 * the sem_host_setup plan format: *n_ids and *n_copies receive its sizes;
 * off[n_ids + 1] and idx[n_copies] (may be NULL) the ids' local copies.
 * Errors: SEM_EINVAL (null desc or sizes, lines_per_wg < 1, invalid mesh). */
sem_status sem_host_axgs_residual(const sem_mesh_desc *desc, int lines_per_wg, int y_onchip, int64_t *n_ids,
                                  int64_t *n_copies, int32_t *off, int32_t *idx);

/* Helmholtz form of the operator (Eq. 4 with the variable coefficient h1 of
 * Algorithm 1): afterwards sem_ax, sem_axgs and sem_pcg_solve apply
 *   A_L u = sum_q h1_q (grad phi)^T G_q (grad u) + h2 B u
 * i.e. the three products of the combine step are scaled by h1 at the point
 * and h2 B u is added, and the Jacobi preconditioner is rebuilt from that
 * operator's assembled diagonal.  h1, h2: device FP64 E-vectors (n_local) or
 * NULL (h1 = 1, h2 = 0); both NULL restores the Poisson operator.  The values
 * are copied (and FP32 copies made with SEM_WITH_FP32).  For CG the caller
 * keeps h1 > 0 and h2 >= 0.  Batched solves (sem_batch_*) take Poisson meshes
 * only.  Synchronises `stream`.  Errors: SEM_EINVAL, SEM_ENOMEM, SEM_EHIP. */
sem_status sem_set_helmholtz(sem_mesh *mesh, const double *h1, const double *h2, void *stream);

/* Local operator, Algorithm 1: w = A_L u element by element (no
 * gather-scatter).  u, w: device E-vectors of `dtype` (SEM_FP64 or SEM_FP32;
 * FP32 needs SEM_WITH_FP32).  opt_dot (device double, may be NULL) receives
 * sum_local u.w, which equals u^T A u when u is continuous.  u and w must not
 * overlap. */
sem_status sem_ax(sem_mesh *mesh, int dtype, const void *u, void *w, double *opt_dot, void *stream);

/* Direct-stiffness summation and Dirichlet mask, in place (section 2, the
 * global exchange of element face values): every copy of a global node gets
 * the sum of all its copies, summed in ascending local index; nodes on
 * Dirichlet faces get 0.  v: device E-vector of `dtype`. */
sem_status sem_gs(sem_mesh *mesh, int dtype, void *v, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sem_ax with
 * the dot product, w = A_L u and *dot = sum u.w, allocating nothing.  The
 * operator's per-workgroup dot partials go to a fixed array of 16384 doubles
 * (128 KiB) that each device holds until the process ends, instead of the
 * mesh's partials buffer; u, w (n_local entries of dtype) and dot (one
 * double) are caller-owned device memory.  Results are the same bits as
 * sem_ax(mesh, dtype, u, w, dot, stream).  All calls on one device share
 * that device's array, so calls that overlap in time on one device (other
 * streams, other threads) race; calls ordered on one stream do not.
 * Errors: SEM_EINVAL (null pointers, u == w, unknown dtype, a mesh of another
 * device, more operator workgroups than 16384 partials -- a larger grid set by
 * sem_set_operator_config), SEM_EHIP. */
sem_status sem_ax_noalloc(sem_mesh *mesh, int dtype, const void *u, void *w, double *dot, void *stream);

/* w = mask(Q Q^T A_L u): sem_ax followed by sem_gs. */
sem_status sem_axgs(sem_mesh *mesh, int dtype, const void *u, void *w, void *stream);

/* Weak-form right-hand side of the pressure Poisson problem (Eq. 5 on the
 * spectral-element discretisation of section 2): b = mask(Q Q^T (B f)), where
 * B is the diagonal mass matrix that Gauss-Lobatto-Legendre quadrature on
 * the tensor-product Lagrange basis gives, B_e(i,j,k) = w_i w_j w_k |J|(i,j,k),
 * and Q Q^T is the direct-stiffness summation of sem_gs.  f, b: device FP64
 * E-vectors (n_local, the element-major local layout of sem_ax), caller-owned;
 * f is read, b written (f == b is allowed: the scaling is pointwise).  Enqueued
 * on `stream`, no synchronisation.  Errors: SEM_EINVAL (null argument),
 * SEM_EHIP. */
sem_status sem_mass(sem_mesh *mesh, const double *f, double *b, void *stream);

/* u_local = mask(Q v): the scatter Q of section 2's split into global and
 * element-local work, the transpose of the gather Q^T that sums a global
 * node's copies.  It copies one value per global node to every local copy of
 * that node and sets the copies on Dirichlet faces to 0.  v_global: device
 * FP64, n_global entries indexed by the glob_id of sem_export_maps; u_local:
 * device FP64 E-vector (n_local); both caller-owned and not overlapping.
 * Enqueued on `stream`, no synchronisation.  Errors: SEM_EINVAL (null
 * argument), SEM_EHIP. */
sem_status sem_scatter(sem_mesh *mesh, const double *v_global, double *u_local, void *stream);

/* Solve options.  sem_solve_opts_default fills tol=1e-10, max_iter=5000,
 * precision=SEM_PREC_FP64, inner_tol=1e-4, inner_max_iter=max_iter,
 * poll_every=16, use_graph=1, fixed_iters=0, x0_given=0, profile=0. */
typedef struct {
    double tol;          /* stop when ||b - A x|| <= tol ||b|| (unique-dof 2-norm) */
    int max_iter;        /* limit on PCG iterations (inner ones for mixed)         */
    int precision;       /* SEM_PREC_FP64 or SEM_PREC_MIXED                        */
    double inner_tol;    /* mixed: relative tolerance of each FP32 inner solve
                            (loosened to 0.5 tol/rel when the FP64 relative
                            residual rel needs less reduction, at most 0.5)     */
    int inner_max_iter;  /* mixed: limit per inner solve                           */
    int poll_every;      /* iterations between host convergence checks            */
    int use_graph;       /* replay poll_every iterations as one hipGraph           */
    int fixed_iters;     /* > 0: run exactly this many FP64 iterations, no polling,
                            no final residual (throughput measurement)           */
    int x0_given;        /* 1: x holds the initial guess; 0: start from x = 0      */
    int profile;         /* 1: time each kernel class with HIP events recorded on
                            `stream` around every launch (iterations then run
                            without graphs); results in sem_solve_stats            */
} sem_solve_opts;

typedef struct {
    int status;               /* same value the call returns                  */
    int iterations;           /* PCG iterations (FP64, or FP32 inner total)    */
    int outer_iterations;     /* mixed: refinement steps; FP64: restarts + 1   */
    double rel_residual;      /* true ||b - A x|| / ||b|| at exit (FP64)        */
    double bnorm;             /* ||b||                                         */
    double seconds;           /* wall time of the call                         */
    /* with opts.profile: summed device time per kernel class over all CG
     * iterations, and the number of operator launches timed */
    double ms_operator;       /* local operator (with the fused p update)      */
    double ms_gather_scatter;
    double ms_update;         /* alpha, r update with dot products, beta      */
    int operator_launches;
} sem_solve_stats;

void sem_solve_opts_default(sem_solve_opts *opts);

/* Jacobi-PCG on the masked assembled system A x = b (section 2 Eq. 5 solved
 * by a preconditioned Krylov method; the preconditioner is the inverse
 * assembled diagonal, plus the coarse term of sem_set_coarse when set).  b: device FP64 E-vector, continuous (all copies of a
 * global node equal) and masked.  x: device FP64 E-vector, in/out.
 * FP64: dot products, alpha and beta stay on the device; the host reads the
 * residual every poll_every iterations.  When the recursive residual meets
 * tol the true residual b - A x is recomputed; if it does not, CG restarts
 * from x (at most 3 times).
 * SEM_PREC_MIXED: defect correction -- r = b - A x in FP64, an FP32 PCG solves
 * A d = r/||r|| to inner_tol, x += ||r|| d in FP64, until the FP64 true
 * residual meets tol.  Needs SEM_WITH_FP32.
 * Synchronises `stream` before returning.  Errors: SEM_ENOCONV (x holds the
 * last iterate), SEM_EBREAKDOWN, SEM_EINVAL, SEM_EHIP. */
sem_status sem_pcg_solve(sem_mesh *mesh, const double *b, double *x, const sem_solve_opts *opts,
                         sem_solve_stats *stats, void *stream);

/* ---------------------------------------------------------------------------
 * Two-level preconditioner (Eq. 6: a coarse term plus local solves; the local
 * solves here are single nodes, i.e. Jacobi).  With a coarse space set, CG
 * solves (sem_pcg_solve, sem_proj_solve; FP64, and the FP32 inner solves of
 * SEM_PREC_MIXED) use
 *   M^{-1} r = D^{-1} r + P C(A0) P^T r
 * where
 *   - P holds the trilinear hat functions of the element vertices at the
 *     GLL nodes (element reference coordinates), 0 at Dirichlet nodes;
 *     periodic images of a vertex are one vertex;
 *   - A0 = P^T A P (the masked assembled operator of the mesh's current form,
 *     Poisson or Helmholtz), assembled from element blocks P_e^T A_e P_e;
 *     vertices whose masked hat function is 0 are not coarse unknowns;
 *   - C(A0) is `chebyshev_steps` steps of Chebyshev iteration for
 *     D0^-1 A0 z = D0^-1 r0 from z = 0, D0 = diag(A0), on [a, b] with b the
 *     largest absolute row sum of D0^-1 A0 and a = fraction * b: a fixed
 *     polynomial, so M is symmetric positive definite.
 * The coarse term runs inside the CG iteration: restriction, Chebyshev and
 * the coarse part of <r, z> after the residual update, the prolongation in
 * the operator's prologue.  The coarse data and the Chebyshev solve stay FP64
 * in both precisions; an FP32 inner solve restricts its FP32 residual and adds
 * the rounded correction.  Batched solves (sem_batch_*): a slot of a mesh
 * with a coarse space takes the coarse term too, in its CG (FP64, or the
 * FP32 inner iterations of a mixed slot), with its own coarse vectors
 * (several slots may share the mesh) -- its restriction, Chebyshev solve
 * (FP64) and prolongation P z0 (rounded to the CG's precision) run per slot
 * after the batched update, and the batched operator adds P z0 in its p
 * update, so the preconditioner is the same M (prolongation summed in
 * another order: the same to rounding).  The coarse space must not change
 * (sem_set_coarse) while the mesh has slots in a batch.
 */
typedef struct {
    int64_t n_vertices;   /* element vertices (periodic images merged)          */
    int64_t n_coarse;     /* coarse unknowns (vertices with a non-zero hat)      */
    int64_t nnz;          /* stored entries of A0 (rows of coarse unknowns)      */
    int chebyshev_steps;  /* 0: no coarse space (Jacobi only)                   */
    double a, b;          /* Chebyshev interval of D0^-1 A0                      */
} sem_coarse_info;

/* Build (chebyshev_steps 1..1000, fraction in (0, 1)) or remove
 * (chebyshev_steps 0) the coarse space of `mesh`.  The build applies the
 * local operator to the 8 masked corner hat functions (FP64, on `stream`),
 * assembles A0 on the host in a fixed order and keeps it on the device;
 * sem_set_helmholtz and sem_load_geometry rebuild it for the new operator.
 * Device memory: about 130 bytes per element and 380 per vertex, plus two
 * temporary FP64 E-vectors during the build.  Synchronises `stream`.
 * Errors: SEM_EINVAL (steps or fraction out of range, a zero coarse
 * operator), SEM_EUNSUPPORTED (N > 12, or 8 E >= 2^31), SEM_ENOMEM, SEM_EHIP. */
sem_status sem_set_coarse(sem_mesh *mesh, int chebyshev_steps, double fraction, void *stream);
sem_status sem_get_coarse_info(const sem_mesh *mesh, sem_coarse_info *info);

/* z = M^{-1} r with the mesh's FP64 preconditioner (Jacobi or the Schwarz
 * local solves of sem_set_schwarz, plus the coarse term when set).  r, z: distinct device FP64 E-vectors, r continuous; z is
 * continuous and masked.  Asynchronous on `stream`. */
sem_status sem_precond_apply(sem_mesh *mesh, const double *r, double *z, void *stream);

/* ---------------------------------------------------------------------------
 * Overlapping Schwarz local solves (Eq. 6, the sum over local subdomains),
 * in place of Jacobi as the local part of the FP64 preconditioner:
 *   z = sum_k R_k^T A_k^{-1} R_k r   (+ the coarse term when set)
 * where
 *   - subdomain k is element k extended by one node layer into every
 *     neighbour that exists (also across periodic faces); nodes beyond a
 *     non-periodic face do not exist and nodes on Dirichlet faces are not
 *     unknowns;
 *   - A_k is the separable (fast-diagonalisation) form on a box with the
 *     element's mean edge lengths:
 *       A_k = B_t x B_s x A_r + B_t x A_s x B_r + A_t x B_s x B_r
 *     with A_d, B_d the 1-D GLL stiffness and lumped mass of the element and
 *     of an equal copy on each side that has a neighbour, restricted to the
 *     subdomain's nodes; it is inverted through the 1-D generalised
 *     eigenvectors (six 1-D contractions per element);
 *   - the local solutions are added without weights into every node they
 *     cover.
 * A_k uses the Poisson form also when sem_set_helmholtz is set (the
 * preconditioner stays symmetric positive definite).  Mixed-precision and
 * batched solves fail with SEM_EUNSUPPORTED while it is set.
 */
/* enable 1: build the 1-D factors on the host (from the element corner
 * coordinates; factors shared by elements with equal length and sides) and
 * the device buffers (an extended E-vector of (N+3)^3 values per element and
 * one E-vector); 0: remove.  Synchronises `stream`.
 * Errors: SEM_EUNSUPPORTED (N = 1: the one-node overlap reaches the far faces
 * of the neighbours and an interior subdomain's local problem is singular;
 * N > 12; E >= 2^31),
 * SEM_EINVAL (degenerate element), SEM_ENOMEM, SEM_EHIP. */
sem_status sem_set_schwarz(sem_mesh *mesh, int enable, void *stream);
/* enabled: 1 when set; n_factors: distinct 1-D factor sets (either may be NULL). */
sem_status sem_get_schwarz_info(const sem_mesh *mesh, int *enabled, int64_t *n_factors);
/* Host only (no device): the 1-D factors of one direction of an extended
 * element of length ell with side kinds left/right (0 a neighbour, 1
 * Dirichlet, 2 a free end): S (count x count, row-major, row = kept extended
 * index lo + row, column = mode) with S^T B S = I and S^T A S = diag(lam).
 * S holds (N+3)^2 and lam N+3 doubles.  Errors: SEM_EINVAL. */
sem_status sem_host_fdm_1d(int N, double ell, int left, int right, double *S, double *lam, int *lo, int *count);

/* ---------------------------------------------------------------------------
 * Projection onto previous solutions (section 2: successive solves of a time
 * step are accelerated by projecting onto the span of earlier solutions,
 * after Fischer).  A projection space keeps an A-orthonormal basis
 * x_1..x_l of earlier solutions of one mesh's current operator (A-inner
 * product x^T A y = unique-dof sum of x and the assembled A y), together with
 * A x_i.  For a right-hand side b the guess
 *   xbar = sum_i (x_i . b) x_i
 * is the element of the span closest to the solution in the A-norm.
 *
 * Ownership: the space owns 2 max_vectors device E-vectors (FP64) and keeps
 * the mesh pointer: free the space before the mesh.  When the mesh's operator
 * changes (sem_set_helmholtz, sem_load_geometry) the basis is emptied.
 */
typedef struct sem_proj sem_proj;

/* max_vectors: 1..32.  Errors: SEM_EINVAL, SEM_ENOMEM. */
sem_status sem_proj_create(sem_mesh *mesh, int max_vectors, sem_proj **out);
sem_status sem_proj_free(sem_proj *proj);
/* Forget the basis. */
sem_status sem_proj_reset(sem_proj *proj);
/* Number of basis vectors held. */
sem_status sem_proj_size(sem_proj *proj, int *n);
/* x = sum_i (x_i . b) x_i (x = 0 for an empty basis).  b, x: device FP64
 * E-vectors, b continuous and masked; asynchronous on `stream`. */
sem_status sem_proj_project(sem_proj *proj, const double *b, double *x, void *stream);
/* Add a solution x (device FP64 E-vector, continuous, masked): one operator
 * apply, two passes of A-Gram-Schmidt against the basis, A-normalisation.  A
 * remainder whose A-norm is below 1e-8 of x's is dropped (*added = 0, may be
 * NULL); a full basis restarts from x alone.  Synchronises `stream`. */
sem_status sem_proj_add(sem_proj *proj, const double *x, int *added, void *stream);
/* sem_pcg_solve started from the projection (opts->x0_given is forced), then
 * the solution joins the basis when the solve succeeded.  Same arguments,
 * statistics and errors as sem_pcg_solve. */
sem_status sem_proj_solve(sem_proj *proj, const double *b, double *x, const sem_solve_opts *opts,
                          sem_solve_stats *stats, void *stream);

/* ---------------------------------------------------------------------------
 * Batched and continuous solves.  A batch holds up to max_slots concurrent
 * solves ("slots"), each on any mesh (orders 2..10, any size) with its own
 * right-hand side, solution and precision.  Every CG phase of all slots runs
 * as one persistent launch over a table of (slot, element tile) work items
 * (the operator: one launch per order present) -- the paper moves loops of
 * small kernels inside the kernel (section 3) -- and poll_every iterations
 * are replayed as one hipGraph.  Each slot's dot
 * products are summed from its own items in a fixed order, so a slot's result
 * does not depend on which other slots share the launches.  The
 * preconditioner is Jacobi, plus the coarse term of Eq. 6 for the slots of
 * a mesh with a coarse space (sem_set_coarse; its per-slot phases are
 * launched slot by slot); meshes with the Helmholtz form or the Schwarz local
 * solves are refused (SEM_EUNSUPPORTED).
 *
 * Ownership: the batch owns its slot vectors (allocated within
 * device_budget bytes, 0 = unlimited, reused after retirement); meshes, b and
 * x stay the caller's and must outlive the slots that use them.
 */
typedef struct sem_batch sem_batch;

sem_status sem_batch_create(int max_slots, size_t device_budget, void *stream, sem_batch **out);
sem_status sem_batch_free(sem_batch *batch);

/* Autotuner: for every order among `meshes` and each precision they carry,
 * time the batched CG operator for each candidate elements-per-workgroup and
 * keep the fastest.  The batch must have no admitted slots. */
sem_status sem_batch_tune(sem_batch *batch, sem_mesh *const *meshes, int n, void *stream);
/* Elements per operator workgroup for order N (epw (N+1)^2 <= 512; 0 restores
 * the default), for the FP64 and the FP32 operator alike (the autotuner picks
 * each precision's own).  The batch must have no admitted slots (SEM_EINVAL).
 * sem_batch_get_epw reads the count in use for `precision` (SEM_FP64 or
 * SEM_FP32). */
sem_status sem_batch_set_epw(sem_batch *batch, int N, int epw);
sem_status sem_batch_get_epw(const sem_batch *batch, int N, int precision, int *epw);
/* Workgroups of the batched launches: ax_grid for each order's operator,
 * vec_grid for the gather-scatter and vector kernels (> 0; 0 restores the
 * default of 16 per compute unit).  Each persistent workgroup walks the work
 * table from its index in steps of the grid, so a small grid makes every
 * workgroup take many (slot, tile) items in turn; results do not depend on it
 * (each slot's partial sums follow its own items).  The batch must have no
 * admitted slots (SEM_EINVAL); cached graphs are dropped. */
sem_status sem_batch_set_grid(sem_batch *batch, int ax_grid, int vec_grid);
sem_status sem_batch_get_grid(const sem_batch *batch, int *ax_grid, int *vec_grid);

/* One-shot: solve A_i x_i = b_i for i < n together (b_i, x_i device FP64
 * E-vectors of mesh i; opts as for sem_pcg_solve, shared by all; stats: n
 * entries or NULL).  Returns SEM_OK when every system converged, else the
 * first failing status. */
sem_status sem_batch_solve(sem_batch *batch, sem_mesh *const *meshes, int n, const double *const *b,
                           double *const *x, const sem_solve_opts *opts, sem_solve_stats *stats, void *stream);

/* Continuous batching: admit a solve into a free slot (SEM_EBUDGET when no
 * slot or no memory within the budget is left), advance all admitted slots by
 * `iterations` CG iterations (serving phase changes -- residual checks,
 * restarts, mixed-precision refinement steps -- at the step boundary), list
 * finished slots, and retire a slot (its stats; the slot becomes free). */
sem_status sem_batch_admit(sem_batch *batch, sem_mesh *mesh, const double *b, double *x,
                           const sem_solve_opts *opts, int *slot, void *stream);
sem_status sem_batch_step(sem_batch *batch, int iterations, int use_graph, void *stream, int *n_active);
sem_status sem_batch_finished(const sem_batch *batch, int *slots, int capacity, int *n);
sem_status sem_batch_retire(sem_batch *batch, int slot, sem_solve_stats *stats);

/* Host-only (for checking): the byte layout of one slot's vector buffer for a
 * mesh of n_local local points.  offsets[0..2] receive the offsets of the
 * FP64 r, p, w; with precision SEM_PREC_MIXED offsets[3..6] those of the FP32
 * x, r, p, w (otherwise 0).  Each vector starts on a 256-byte boundary;
 * *bytes receives the size the batch allocates for the slot, which holds
 * every vector.  SEM_EINVAL on a null pointer, n_local < 1 or an unknown
 * precision. */
sem_status sem_batch_slot_layout(int64_t n_local, int precision, size_t *offsets, size_t *bytes);

#ifdef __cplusplus
}
#endif
#endif /* SEM_H */
