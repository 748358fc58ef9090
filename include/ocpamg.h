/*
 * ocpamg -- AMG-preconditioned CG for the P1 finite element system of the
 * reduced optimality equation of elliptic optimal control with energy
 * regularization, on one MI355X (gfx950).
 *
 * The problem (Section 1, eq. (5)): find u with  -rho*Lap(u) + u = ubar  in
 * Omega and u = 0 on Gamma, for a regularization parameter rho > 0 and a
 * target ubar in L2(Omega).  Its Galerkin discretization with continuous
 * piecewise-linear elements on a tetrahedral mesh (Section 2: the discrete
 * variational problem and system (linsys)) is the sparse SPD system
 *
 *     (rho*K + M) u = f,   K_ij = int grad(phi_j).grad(phi_i),
 *                          M_ij = int phi_j phi_i,   f_i = int ubar phi_i,
 *
 * over the interior vertices.  It is solved by preconditioned CG (Section 4)
 * with an algebraic multigrid V(1,1)-cycle as preconditioner (Section 3.1).
 *
 * Conventions for every entry point below:
 *   - Every function returns an int status: 0 success, negative on error
 *     (OCP_ERR_*), pcg_solve may also return OCP_MAXIT (+1).  No exception
 *     crosses this interface.  ocp_last_error() gives a message.
 *   - Pointers documented as "device" point to memory on the context's GPU;
 *     "host" pointers are ordinary CPU memory.  Arrays are dense, C order.
 *   - All work is enqueued on the context's HIP stream.  Calls that return a
 *     size or a status computed on the GPU synchronize that stream.
 *   - Library-owned device memory comes from the allocator given to
 *     ocp_ctx_create (or hipMalloc/hipFree when none is given).
 *   - A context is used by one host thread at a time.  Solves only read
 *     systems and hierarchies (each solve owns its vectors, scalars and
 *     reduction partials; data a first solve derives, such as the Jacobi
 *     diagonal or a block panel width, is published under a lock or by
 *     compare-and-swap once complete), so several contexts on several
 *     streams may solve with the same system and hierarchy at once.
 *     Calls that change a system (fe_set_rho) or free it must not overlap
 *     solves that use it.
 */
#ifndef OCPAMG_H
#define OCPAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define OCP_OK 0
#define OCP_MAXIT 1              /* pcg_solve: iteration cap reached (not an error) */
#define OCP_ERR_INVALID_ARG (-1) /* NULL pointer, size <= 0, rho <= 0 or not finite, ... */
#define OCP_ERR_BAD_MESH (-2)    /* vertex index out of range, degenerate tet, no interior vertex */
#define OCP_ERR_OOM (-3)         /* the allocator returned NULL */
#define OCP_ERR_BREAKDOWN (-4)   /* CG breakdown: p^T A p <= 0, r^T z <= 0, or non-finite */
#define OCP_ERR_HIP (-5)         /* a HIP runtime call failed */
#define OCP_ERR_UNSUPPORTED (-6) /* a size limit of the implementation was exceeded */

/* --------------------------------------------------------------- context */
typedef struct ocp_ctx ocp_ctx;
typedef struct ocp_system ocp_system;
typedef struct ocp_hierarchy ocp_hierarchy;

/* Device allocator callbacks: alloc returns a device pointer of at least
 * `bytes` bytes (256-byte aligned) or NULL; free releases it.  `user` is
 * passed through.  Both may be NULL: then hipMalloc / hipFree are used. */
typedef void *(*ocp_alloc_fn)(size_t bytes, void *user);
typedef void (*ocp_free_fn)(void *ptr, void *user);

/* Create a context bound to the current HIP device and to `stream`
 * (a hipStream_t; NULL = the default stream).  The caller keeps ownership of
 * the stream.  *out is freed by ocp_ctx_destroy. */
int ocp_ctx_create(void *stream, ocp_alloc_fn alloc, ocp_free_fn free_fn, void *user,
                   ocp_ctx **out);
void ocp_ctx_destroy(ocp_ctx *ctx);
/* Message of the last failed call on this context ("" if none).  Owned by the
 * context; valid until the next call on it. */
const char *ocp_last_error(const ocp_ctx *ctx);
/* Library version string (static storage). */
const char *ocp_version(void);

/* ------------------------------------------------------------------ mesh */
/* A tetrahedral mesh of Omega (Section 2: an admissible, shape-regular
 * simplicial decomposition).  All arrays are device memory, borrowed for the
 * duration of the call that receives the mesh. */
typedef struct {
    int32_t n_vertices;
    int32_t n_tets;
    const double *xyz;        /* device [n_vertices][3] vertex coordinates */
    const int32_t *tets;      /* device [n_tets][4] vertex ids, any orientation */
    const uint8_t *dirichlet; /* device [n_vertices], 1 = vertex on Gamma (u = 0) */
} ocp_mesh;

/* ---------------------------------------------------------------- target */
#define OCP_TARGET_SINE_MODES 0 /* ubar = offset + sum_m amp[m] prod_d sin(k[m][d] pi x_d) */
#define OCP_TARGET_BOX 1        /* ubar = 1 on the open box (lo, hi), 0 elsewhere */
#define OCP_TARGET_NODAL 2      /* ubar = sum_v nodal[v] phi_v (P1 interpolant) */

/* Target function ubar (Section 1).  Mode tables are host memory, copied by
 * the call; `nodal` is device memory [n_vertices], borrowed for the call. */
typedef struct {
    int32_t kind;
    int32_t n_modes;       /* SINE_MODES: number of modes, 1..4096 */
    const int32_t *k;      /* host [n_modes][3], wave numbers 1..1024 */
    const double *amp;     /* host [n_modes] */
    double offset;
    double lo[3], hi[3];   /* BOX */
    const double *nodal;   /* NODAL: device [n_vertices] */
} ocp_target;

/* -------------------------------------------------------------- assembly */
#define OCP_KEEP_KM 1 /* keep K and M values separately so fe_set_rho can re-weight */
#define OCP_NO_LOAD 2 /* assemble A only: f is set to zero and target may be NULL; the load
                       * vector then comes from fe_load, which may run on another context
                       * while amg_setup works on this system */

/* Assemble A = rho*K + M and f (Section 2, system (linsys)) on the interior
 * vertices of `mesh` into CSR on the device.  Element matrices are exact; f
 * uses the 4-point degree-2 rule on each tetrahedron (with OCP_NO_LOAD in
 * flags, f is zero and target is not read).  The assembly is
 * row-owned (one owner per row, no atomics on values) and bitwise
 * deterministic.  Unknowns are the interior vertices in increasing vertex id.
 * Errors: INVALID_ARG (NULL, counts <= 0, rho <= 0 or not finite, bad target),
 * BAD_MESH (index out of range, |det| <= 1e-12 * longest edge^3, no interior
 * vertex), UNSUPPORTED (a vertex with more than 255 incident tets or a row
 * with more than 128 entries), OOM, HIP.  *out is freed by ocp_system_destroy. */
int fe_assemble(ocp_ctx *ctx, const ocp_mesh *mesh, double rho, const ocp_target *target,
                int32_t flags, ocp_system **out);
void ocp_system_destroy(ocp_system *sys);

/* Replace rho: A = rho*K + M (needs OCP_KEEP_KM at assembly).  The system's
 * values change in place, so no solve may use it while this runs.  Every
 * hierarchy built on this system before the call is stale afterwards (its
 * smoother diagonal, eigenvalue bound and coarse operators belong to the old
 * matrix): the solves and amg_vcycle refuse it with INVALID_ARG until it is
 * rebuilt with amg_setup. */
int fe_set_rho(ocp_ctx *ctx, ocp_system *sys, double rho);

/* A new system on the same mesh with A = rho*K + M, from the K and M values
 * that `base` stored (base assembled with OCP_KEEP_KM): the pattern, maps
 * and f are copied, no element is recomputed.  The result has no K/M of its
 * own and is freed by ocp_system_destroy; the mesh must stay alive as for
 * base.  Errors: INVALID_ARG (NULL, rho <= 0, base without K/M), OOM, HIP. */
int fe_derive(ocp_ctx *ctx, const ocp_system *base, double rho, ocp_system **out);

/* Load vector of another target on the system's mesh (Section 2: f_i =
 * int ubar phi_i, by the rule of fe_assemble): f_dev (device [n_dofs],
 * caller-owned) receives it.  The system borrows the mesh given to
 * fe_assemble (for fe_derive: the base's), whose device arrays must still be
 * alive.  Errors: INVALID_ARG (NULL, bad target), OOM, HIP. */
int fe_load(ocp_ctx *ctx, const ocp_system *sys, const ocp_target *target, double *f_dev);

/* Load vectors of k targets on the same mesh in one block: F (device
 * [n_dofs][k], row-major, caller-owned) receives F[i*k + j] = int ubar_j phi_i
 * for target j (the same rule as fe_assemble).  This is the right-hand side
 * block of pcg_solve_multi.  Errors as fe_load; INVALID_ARG if k < 1. */
int fe_load_multi(ocp_ctx *ctx, const ocp_system *sys, int32_t k, const ocp_target *targets, double *F);

/* Read-only view of an assembled system (device pointers owned by `sys`). */
typedef struct {
    int32_t n_vertices;
    int32_t n_dofs;             /* interior unknowns */
    int64_t nnz;
    double rho;
    const int32_t *row_ptr;     /* device [n_dofs+1] */
    const int32_t *col;         /* device [nnz], sorted within each row */
    const double *val;          /* device [nnz] */
    const double *f;            /* device [n_dofs] */
    const int32_t *dof_of_vertex; /* device [n_vertices], -1 on Gamma */
    const int32_t *vertex_of_dof; /* device [n_dofs] */
    int32_t sell_coded;         /* 1: the solve-phase sliced-ELL copy reads 4-bit column codes
                                   (every 64-row slice has <= 16 distinct col - row offsets) */
    int64_t sell_entries;       /* stored entries of that copy (64-row slices padded to their
                                   longest row) */
} ocp_system_view;
int ocp_system_get_view(const ocp_system *sys, ocp_system_view *view);

/* y = A x for device vectors x, y of length n_dofs (the CSR SpMV kernel of
 * the CG iteration). */
int ocp_spmv(ocp_ctx *ctx, const ocp_system *sys, const double *x, double *y);

/* ------------------------------------------------------------ AMG setup */
#define OCP_PREC_FP64 0  /* hierarchy values and V-cycle in double */
#define OCP_PREC_MIXED 1 /* hierarchy values and V-cycle in float, CG in double */

#define OCP_SMOOTH_L1JACOBI 0
#define OCP_SMOOTH_CHEBYSHEV 1

/* The AMG method of the hierarchy:
 *   OCP_AMG_AGGREGATION  smoothed aggregation (default): distance-2
 *       independent-set aggregates, smoothed prolongator, polynomial
 *       (Chebyshev or L1-Jacobi) smoother; this build's design for the GPU.
 *   OCP_AMG_REDBLACK     the method of Section 3.1: red-black colouring
 *       coarsening (an unmarked dof turns black = coarse, its unmarked
 *       neighbours red = fine, until every dof is marked; visited here in a
 *       fixed hash order of the dofs), interpolation of a fine dof by the
 *       average of its coarse neighbours, Galerkin A_c = P^T A P, and one
 *       symmetric Gauss-Seidel sweep (forward before, backward after the
 *       coarse correction), the dofs swept colour by colour in a colouring of
 *       A's graph.  smoother, degree, omega and cheb_ratio are ignored. */
#define OCP_AMG_AGGREGATION 0
#define OCP_AMG_REDBLACK 1

typedef struct {
    int32_t precision;   /* OCP_PREC_* */
    int32_t smoother;    /* OCP_SMOOTH_* */
    int32_t degree;      /* Chebyshev degree, 1 or 2; L1-Jacobi uses 1 */
    int32_t coarse_max;  /* stop coarsening at n <= coarse_max (dense solve there), <= 2048 */
    int32_t max_levels;  /* 1..16 */
    double theta;        /* strength threshold: |a_ij| >= theta sqrt(a_ii a_jj) */
    double omega;        /* prolongator smoothing: omega/lambda_max(D^-1 A), 1.9 default */
    double cheb_ratio;   /* Chebyshev interval [lambda/cheb_ratio, lambda], lambda = Gershgorin bound */
    int32_t method;      /* OCP_AMG_AGGREGATION (default) or OCP_AMG_REDBLACK */
} ocp_amg_params;

/* Fill `p` with the defaults (smoothed aggregation, FP64, Chebyshev degree 2
 * on [lambda/10, lambda], coarse_max 512, 10 levels, theta 0, omega 1.9). */
void amg_default_params(ocp_amg_params *p);

/* Build a smoothed-aggregation hierarchy for the system's A (Section 3.1:
 * coarse spaces from a coarsening of the matrix graph, interpolation P, and
 * Galerkin coarse operators A_c = P^T A P, applied recursively).  NULL params
 * means defaults.  The hierarchy must not outlive `sys`.
 * Errors: INVALID_ARG, UNSUPPORTED (SpGEMM row too long), OOM, HIP. */
int amg_setup(ocp_ctx *ctx, const ocp_system *sys, const ocp_amg_params *params,
              ocp_hierarchy **out);
void ocp_hierarchy_destroy(ocp_hierarchy *h);

/* Read-only view of one level (device pointers owned by the hierarchy).
 * Level 0 is the fine level (A is the system's matrix). P, R and agg are
 * NULL on the last level; dense_inv is non-NULL only there. */
typedef struct {
    int32_t n_levels;
    int32_t level;
    int32_t n;                 /* rows of A on this level */
    int32_t n_coarse;          /* columns of P (rows of the next level) */
    int64_t nnz_A, nnz_P;
    const int32_t *A_row_ptr, *A_col;
    const double *A_val;
    const int32_t *P_row_ptr, *P_col;
    const double *P_val;
    const int32_t *R_row_ptr, *R_col;
    const double *R_val;
    const int32_t *agg;        /* device [n], aggregate of each row */
    const double *dense_inv;   /* device [n][n] inverse of A on the last level */
    double lambda_max;         /* Gershgorin bound of D^-1 A used for omega */
} ocp_level_view;
int ocp_hierarchy_get_level(const ocp_hierarchy *h, int32_t level, ocp_level_view *view);

/* z = B r: one V-cycle with zero initial guess (Section 3.1, two-grid
 * operator applied recursively), the same polynomial smoother before and
 * after the coarse correction so that B is symmetric.  r, z: device [n_dofs]. */
int amg_vcycle(ocp_ctx *ctx, const ocp_hierarchy *h, const double *r, double *z);

/* ---------------------------------------------------------------- solve */
#define OCP_STOP_L2 0      /* stop when ||r_k||_2 <= rtol ||f||_2 (default) */
#define OCP_STOP_PRECOND 1 /* stop when sqrt(r_k^T z_k) <= rtol sqrt(r_0^T z_0) */
#define OCP_FLEXIBLE 2     /* flexible (Polak-Ribiere) beta = r'.(z' - z) / (r.z), for a preconditioner
                              symmetric only to rounding (FP32 V-cycle); pcg_solve and the step API
                              with a hierarchy; ignored by the batch and block solves */

typedef struct {
    int32_t iterations;
    int32_t status;         /* same value pcg_solve returns */
    double rel_res_l2;      /* ||r_k|| / ||f|| of the CG recurrence */
    double rel_res_precond; /* sqrt(r_k^T z_k / r_0^T z_0) */
    double true_rel_res;    /* ||f - A u|| / ||f|| recomputed in double at exit */
    double setup_ms;        /* wall time amg_setup took to build the hierarchy used (0: Jacobi) */
    double solve_ms;        /* GPU time of the solve (events on the context stream) */
} ocp_solve_info;

/* Preconditioned CG from u = 0 (Section 4: PCG, one V(1,1)-cycle per
 * iteration as preconditioner; tolerance 1e-8 in the paper).
 *   h      hierarchy from amg_setup, or NULL for Jacobi preconditioning.  It may
 *          belong to another system on the same mesh with the same pattern
 *          (another rho): the V-cycle is then the one built for that
 *          system, still a fixed SPD preconditioner, while CG and the stop
 *          test use this system (the serving loop shares hierarchies across
 *          nearby rho this way)
 *   f      device [n_dofs] right-hand side, or NULL for the system's f
 *   u      device [n_vertices] output, caller-owned; Dirichlet entries set 0
 *   rtol   > 0;  maxit >= 1;  flags: OCP_STOP_L2 or OCP_STOP_PRECOND, | OCP_FLEXIBLE
 * Blocks until converged or capped.  Returns 0 (converged), OCP_MAXIT (u holds
 * the last iterate), OCP_ERR_BREAKDOWN, or another error. */
int pcg_solve(ocp_ctx *ctx, const ocp_system *sys, const ocp_hierarchy *h, const double *f,
              double *u, double rtol, int32_t maxit, int32_t flags, ocp_solve_info *info);

/* pcg_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same solve, same arguments, same kernels and the same bits as
 * pcg_solve, with every work vector (CG vectors, V-cycle vectors, device
 * scalars, reduction partials) carved from one fixed scratch array of
 * OCP_NOALLOC_SCRATCH_BYTES that the library holds per GPU from its first use
 * on that GPU until the process ends.  The call makes no device allocation
 * or free (nor does any allocator callback run).  The caller still passes f
 * and u.  A solve whose work memory exceeds the scratch size (about 80-110
 * bytes per unknown: n up to roughly 6e5 with an FP64 hierarchy, 8e5 mixed)
 * is refused with OCP_ERR_UNSUPPORTED before any work is enqueued.  Every
 * call on one GPU shares that GPU's scratch array and leaves its contents
 * behind: calls that overlap on one GPU (several contexts, streams or host
 * threads at once) race and must be serialized by the caller.  Kernel
 * timing (ocp_profile_enable) is not recorded during the call.  Returns as
 * pcg_solve. */
#define OCP_NOALLOC_SCRATCH_BYTES (64u << 20)
int pcg_solve_noalloc(ocp_ctx *ctx, const ocp_system *sys, const ocp_hierarchy *h, const double *f,
                      double *u, double rtol, int32_t maxit, int32_t flags, ocp_solve_info *info);

/* Block PCG for k right-hand sides that share A and the hierarchy (the PCG
 * of Section 4 run as k independent recurrences in one pass over the
 * matrix per iteration).  Every column has its own alpha, beta and stop
 * test; a column that has converged, broken down or reached maxit is frozen
 * while the others continue.  The V-cycle is the one of pcg_solve (same
 * coefficients, the hierarchy's precision); CG is double.
 *   k      1..64 columns
 *   F      device [n_dofs][k] row-major (entry (i,j) at i*k + j), or NULL:
 *          every column solves with the system's f
 *   U      device [n_vertices][k] output, caller-owned; Dirichlet rows 0
 *   infos  host [k] per-column results (may be NULL)
 *   flags  OCP_STOP_L2 or OCP_STOP_PRECOND, optionally | OCP_BLOCK_TILE(kb)
 * The block kernels cut the k columns into panels of kb columns (8, 16, 32
 * or 64); unless forced with OCP_BLOCK_TILE the width is chosen by timing
 * the candidates on the first solve of each (system or hierarchy, k) and
 * then kept, so repeated solves run the same kernels and give the same bits.
 * Blocks until every column has stopped.  Returns the worst column's status:
 * OCP_ERR_BREAKDOWN if any column broke down, else OCP_MAXIT if any column
 * reached the cap, else 0; or another error (then no column result). */
#define OCP_BLOCK_TILE(kb) ((int32_t)(kb) << 8)
int pcg_solve_multi(ocp_ctx *ctx, const ocp_system *sys, const ocp_hierarchy *h, int32_t k,
                    const double *F, double *U, double rtol, int32_t maxit, int32_t flags,
                    ocp_solve_info *infos);

/* Many independent solves packed together (each one the PCG of pcg_solve
 * on its own system, hierarchy and right-hand side).  Problems of at most
 * 2^18 unknowns run in one persistent launch, one workgroup per solve doing
 * the whole iteration (every V-cycle pass, the stop test) on the device:
 * some thirty kernel dispatches per iteration per problem, each only
 * microseconds of work at these sizes, become one dispatch for the batch.
 * Their results equal pcg_solve's to rounding (dot products are summed in
 * another order), bit for bit from one batch call to the next.  Larger
 * problems (or all, with OCP_BATCH_GRAPH) are packed into one HIP graph that
 * holds one iteration of every solve and is replayed until all have
 * stopped; those give the same bits as pcg_solve alone.
 *   m             1..4096 solves
 *   systems[m]    systems (may repeat); hierarchies[m] or NULL (Jacobi), an
 *                 entry may be NULL; f[m] device right-hand sides or NULL
 *                 (system f), an entry may be NULL; u[m] device outputs
 *                 [n_vertices of system i]
 *   infos         host [m] or NULL; solve_ms is the whole batch's time
 * Returns the worst status (BREAKDOWN, then MAXIT) or an error. */
#define OCP_BATCH_GRAPH (1 << 16) /* pcg_solve_batch: use the graph path for every solve */
int pcg_solve_batch(ocp_ctx *ctx, int32_t m, const ocp_system *const *systems,
                    const ocp_hierarchy *const *hierarchies, const double *const *f, double *const *u,
                    double rtol, int32_t maxit, int32_t flags, ocp_solve_info *infos);

/* Step interface of pcg_solve for callers that interleave several solves
 * (the serving loop): the same iteration, enqueued in pieces without
 * blocking.  A context runs one such solve at a time, and while it is
 * active every other call on that context is refused (INVALID_ARG); use one
 * context (stream) per concurrent solve.  The hierarchy and system are only
 * read, so several contexts may solve with the same ones at once.
 *   pcg_begin    enqueues u = 0, r = f, the first V-cycle; *out owns the
 *                work vectors.  Arguments as pcg_solve.
 *   pcg_advance  enqueues `iters` more iterations (those after the stop
 *                return at once on the device) and a copy of the scalars.
 *   pcg_poll     does not block: 2 while the last advance is still on the
 *                GPU (info untouched), 1 when it has finished and the stop
 *                test has not fired (advance again), 0 once the solve has
 *                stopped (info->status holds 0, OCP_MAXIT or BREAKDOWN), <0
 *                on a runtime error.  true_rel_res and solve_ms are 0 here.
 *   pcg_end      recomputes the true residual, writes u (device
 *                [n_vertices]), fills info, frees the handle; returns the
 *                status as pcg_solve (OCP_MAXIT if ended before the stop). */
typedef struct ocp_solve_handle ocp_solve_handle;
int pcg_begin(ocp_ctx *ctx, const ocp_system *sys, const ocp_hierarchy *h, const double *f, double rtol,
              int32_t maxit, int32_t flags, ocp_solve_handle **out);
int pcg_advance(ocp_solve_handle *hd, int32_t iters);
int pcg_poll(ocp_solve_handle *hd, ocp_solve_info *info);
int pcg_end(ocp_solve_handle *hd, double *u, ocp_solve_info *info);

/* ------------------------------------------- control, adjoint, errors */
/* Adjoint and control from a computed state (Section 1: the gradient
 * equation (4) gives p = -rho u; the state equation (2) with the reduced
 * equation (5) gives z = -Lap u = (ubar - u) / rho), at every vertex of the
 * system's mesh: p[v] = -rho u[v], z[v] = (ubar(x_v) - u[v]) / rho, with
 * ubar evaluated at the vertex (its nodal value for a NODAL target; on the
 * box faces an indicator is 0), rho the system's.
 *   u      device [n_vertices] state (as written by pcg_solve)
 *   p, z   device [n_vertices] outputs, caller-owned; either may be NULL
 * The system's mesh must still be alive.  Errors: INVALID_ARG (NULL system
 * or u, bad target when z is asked for), OOM, HIP. */
int fe_recover(ocp_ctx *ctx, const ocp_system *sys, const ocp_target *target, const double *u, double *p,
               double *z);

/* Errors of a P1 state u (device [n_vertices]) measured in Section 4.1
 * (Tables 1-3), integrated element by element over the system's mesh with
 * a degree-7 rule (125 points per tetrahedron):
 *   out[0] = ||u_rho - u||_L2,  out[1] = ||grad(u_rho - u)||_L2, where u_rho
 *            is the exact solution of eq. (5) for a target made of Dirichlet
 *            eigenfunctions: a SINE_MODES target with offset 0 gives
 *            u_rho = sum_m amp[m] / (1 + rho pi^2 |k_m|^2) prod_d sin(k_md pi x_d);
 *            NaN for any other target (no closed form)
 *   out[2] = ||ubar - u||_L2 (the distance to the target; a NODAL target is
 *            its P1 interpolant)
 * out is host memory [3].  Synchronizes the stream.  Errors: INVALID_ARG,
 * OOM, HIP. */
int fe_error_norms(ocp_ctx *ctx, const ocp_system *sys, const ocp_target *target, const double *u, double *out);

/* Residual error indicator of a P1 state u (device [n_vertices]) for the
 * adaptive refinement of Sections 4.2 and 4.3 (the paper names a
 * residual-based indicator; this is the robust one for reaction-diffusion
 * equations): per tetrahedron T of the system's mesh
 *   eta2[T] = a_T^2 ||ubar - u||^2_T
 *           + 1/2 sum over interior faces F of T of rho^(-1/2) a_F |F| (rho [grad u . n_F])^2,
 *   a_S = min(1, h_S / sqrt(rho)), h_S the longest edge of S,
 * the first term by the 4-point rule of the load vector.  eta2 is device
 * [n_tets], caller-owned.  Errors: INVALID_ARG, OOM, HIP. */
int fe_error_indicator(ocp_ctx *ctx, const ocp_system *sys, const ocp_target *target, const double *u,
                       double *eta2);

/* --------------------------------------------------- adaptive refinement */
/* A tetrahedral mesh refined by bisection in host memory (Sections 4.2, 4.3:
 * meshes refined adaptively by a residual-based indicator).  Tetrahedron
 * (x0, x1, x2, x3) with tag d is bisected at the midpoint of edge (x0, x_d)
 * into (x0..x_{d-1}, z, x_{d+1}..x3) and (x1..x_d, z, x_{d+1}..x3), tag d-1
 * (3 after 1); every tetrahedron that has a bisected edge is bisected in
 * turn until none has (conforming result).  The initial tetrahedra start
 * with tag 3 and must list their vertices along lattice paths as the Kuhn
 * split does (cube corner, +e_i, +e_i+e_j, opposite corner); other meshes
 * may not stay conforming.  All arrays are host memory.
 *   create  copies the mesh (n_vertices, xyz [n][3], n_tets, tets [n][4]).
 *   refine  marks by Doerfler's bulk criterion (largest eta2 first until
 *           their sum reaches theta * total, 0 < theta <= 1; eta2 host
 *           [n_tets] of the current mesh), bisects; *n_marked (may be NULL)
 *           receives the number marked.
 *   sizes / get  the current mesh: xyz [n_vertices][3], tets [n_tets][4]
 *           and dirichlet [n_vertices] (1 on faces of one tetrahedron only);
 *           any output pointer may be NULL.
 * Errors: INVALID_ARG, BAD_MESH (index out of range; a closure that does
 * not end), UNSUPPORTED (more than 2^31 entries). */
typedef struct ocp_refiner ocp_refiner;
int ocp_refiner_create(const double *xyz, int32_t n_vertices, const int32_t *tets, int32_t n_tets,
                       ocp_refiner **out);
void ocp_refiner_destroy(ocp_refiner *r);
int ocp_refiner_refine(ocp_refiner *r, const double *eta2, double theta, int32_t *n_marked);
int ocp_refiner_sizes(const ocp_refiner *r, int32_t *n_vertices, int32_t *n_tets);
int ocp_refiner_get(const ocp_refiner *r, double *xyz, int32_t *tets, uint8_t *dirichlet);

/* ------------------------------------------------------- kernel timing */
#define OCP_KERNEL_CG_SPMV 0      /* q = A p with p.q, FP64 CSR (the CG iteration's SpMV) */
#define OCP_KERNEL_VC_PRE0 1      /* fine-level first smoothing step fused with the residual */
#define OCP_KERNEL_VC_POST0 2     /* fine-level last post-smoothing pass with r.z */
#define OCP_KERNEL_VC_RESTRICT0 3 /* fine-level restriction R r */
#define OCP_KERNEL_VC_PROLONG0 4  /* fine-level prolongation D^-1 (...) + P e */
#define OCP_KERNEL_VC_PRE0_B 5    /* fine-level second pre-smoothing pass (degree 2) */
#define OCP_KERNEL_VC_POST0_A 6   /* fine-level first post-smoothing residual (degree 2) */
#define OCP_KERNEL_BLK_SPMM 7     /* Q = A P with per-column p.q, FP64 CSR (pcg_solve_multi) */

/* Live timing of selected kernels with HIP events on the context stream.
 * ocp_profile_enable(ctx, 1) clears the counters and brackets every launch of
 * the kernels above inside pcg_solve (pcg_solve_multi for BLK_SPMM) with an event pair; launches of the
 * solve's final iteration (which may return early after convergence) and of
 * the initial preconditioner application (before iteration 1) are not
 * counted.  ocp_profile_read returns the number of counted launches and their
 * summed duration in milliseconds. */
int ocp_profile_enable(ocp_ctx *ctx, int32_t on);
int ocp_profile_read(ocp_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* OCPAMG_H */
