/*
 * cgp.h -- C ABI of the MI355X (gfx950) coarse-grid-projection library.
 *
 * The library implements the per-time-step elliptic work that coarse grid
 * projection (CGP; Kashefi, arXiv 2003.00082) moves onto a coarsened mesh, on
 * a fine P1 space V_j and a coarse space V_{j-k} built by k uniform 4-way
 * subdivisions (Section 2.3, Eq. 18):
 *
 *   cgp_restrict       inject the fine velocity onto the coarse nodes (Eq. 19)
 *                      and assemble the coarse source of Eq. 12 or Eq. 15;
 *   cgp_poisson_solve  solve the coarse Poisson system (Eqs. 12, 15);
 *   cgp_prolong        P1 prolongation back to the finest level (Eq. 20);
 *   cgp_lorentz_force  grad(phi_f) and the Lorentz source of Eqs. 13-14;
 *   cgp_velocity_correct  grad(p_f) and the projection of Eqs. 16-17;
 *   cgp_momentum_step  the semi-implicit momentum step of Eqs. 13-14 (fine mesh);
 *   cgp_interpolate    a level's P1 field at arbitrary points (the non-nested restriction);
 *   cgp_surface_force  pressure and viscous force of the fluid on a body (drag and lift).
 *
 * Conventions for every call:
 *   - Return value: CGP_OK (0) or a negative cgp_status.  No C++ exception
 *     crosses the ABI.  cgp_last_error() gives a message for the last failing
 *     call of the calling thread.
 *   - h_* arguments are host pointers, read during the call and never retained.
 *   - d_* arguments are device pointers owned by the caller (e.g. torch tensors
 *     on the context's device).  They must stay valid until the work enqueued on
 *     the context's stream has completed.
 *   - Meshes, matrices, maps, solver workspaces and models are owned by the
 *     library and released by cgp_mesh_free / cgp_model_free / cgp_destroy.
 *   - Unless stated otherwise a call only enqueues work on the context's stream
 *     and returns; device-side failures surface at cgp_sync().
 *   - Arguments are validated before anything is enqueued: null pointers, sizes
 *     out of range or unknown handles give CGP_E_INVALID and enqueue nothing.
 *   - A context is used by one host thread at a time.  A mesh's solver
 *     workspace is shared by all solves on that mesh, so two solves on the same
 *     mesh must not run concurrently (they are serialised on one stream anyway).
 *   - Floating-point data are IEEE fp64 unless stated; indices are int32.
 */
#ifndef CGP_H
#define CGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cgp_ctx_s *cgp_ctx;
typedef int32_t cgp_mesh;   /* handle of an uploaded mesh hierarchy (>= 0) */
typedef int32_t cgp_model;  /* handle of a learned initial-guess network (>= 0) */
typedef int32_t cgp_graph;  /* handle of a captured HIP graph (>= 0) */
typedef int32_t cgp_status;

enum {
    CGP_OK = 0,
    CGP_E_INVALID = -1,     /* bad argument; nothing was enqueued */
    CGP_E_NOMEM = -2,       /* device or host allocation failed */
    CGP_E_HIP = -3,         /* a HIP runtime call failed (message in cgp_last_error) */
    CGP_E_MESH = -4,        /* mesh rejected: index out of range or triangle not CCW */
    CGP_E_NOCONV = -5,      /* returned by cgp_solve_check: an instance hit max_iter */
    CGP_E_BREAKDOWN = -6,   /* returned by cgp_solve_check: p.Kp <= 0 or non-finite */
    CGP_E_UNSUPPORTED = -7, /* valid request the library does not implement */
    CGP_E_ABORTED = -8      /* returned by cgp_solve_check: the solve kernel timed out */
};

/* sources of cgp_restrict */
enum { CGP_SRC_CURL = 0, CGP_SRC_DIV = 1 };
/* arithmetic of cgp_poisson_solve */
enum { CGP_FP64 = 0, CGP_FP32_IR = 1 };
/* initial guess of cgp_poisson_solve */
enum { CGP_GUESS_ZERO = 0, CGP_GUESS_GIVEN = 1, CGP_GUESS_EXTRAP = 2, CGP_GUESS_LEARNED = 3 };
/* how cgp_poisson_solve synchronises its workgroups between CG stages:
 *   STAGED      one kernel launch per stage (one per CG iteration), launched from
 *               replayed HIP graphs; the call returns once the host has seen every
 *               instance finish (it waits on the device, it does not enqueue only).
 *               Under graph capture (cgp_graph_begin) the call waits for nothing: it
 *               records the boot, a fixed number of stage launches (the stage budget,
 *               cgp_solve_opts.stage_budget) and a closing kernel into the graph; it
 *               needs an earlier uncaptured solve of the same meshes, vectors and
 *               options (CGP_E_INVALID otherwise), which built the launch records.
 *               Each workgroup owns a compact tile of at most 512 rows (recursive
 *               coordinate bisection; when that takes more than 256 tiles, the larger
 *               of 256 and n/1024 tiles of up to 1024 rows; more while a region does not
 *               fit a workgroup) and works on the rows within graph distance
 *               d of it; meshes whose rows are wider than 12 entries or whose
 *               regions do not fit use STAGED_ROWS instead (Jacobi only)
 *   STAGED_ROWS as STAGED with workgroups owning consecutive row ranges (Jacobi only)
 *   PERSISTENT  one co-resident launch with a grid-wide barrier between stages;
 *               fully asynchronous, so it can be captured in a caller's graph
 *               (Jacobi only)
 *   AUTO        STAGED for the Chebyshev preconditioner or deflation; plain Jacobi:
 *               PERSISTENT while the context's stream is being captured, otherwise
 *               STAGED_ROWS */
enum { CGP_ENGINE_AUTO = 0, CGP_ENGINE_STAGED = 1, CGP_ENGINE_PERSISTENT = 2, CGP_ENGINE_STAGED_ROWS = 3 };
/* per-instance solve status (cgp_solve_stats.status) */
enum { CGP_SOLVE_OK = 0, CGP_SOLVE_NOCONV = 1, CGP_SOLVE_BREAKDOWN = 2, CGP_SOLVE_ABORTED = 3 };

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (e.g. torch.cuda.current_stream().cuda_stream) or NULL for the null stream.
 * Synchronous. */
cgp_status cgp_create(cgp_ctx *out, int32_t device, void *hip_stream);
/* Free the context and everything it owns (meshes, models, graphs).  Synchronous. */
cgp_status cgp_destroy(cgp_ctx ctx);
/* Replace the stream on which later calls enqueue their work. */
cgp_status cgp_set_stream(cgp_ctx ctx, void *hip_stream);
/* Wait for the context's stream; reports asynchronous HIP errors. */
cgp_status cgp_sync(cgp_ctx ctx);
/* Message of the last failing call made by this thread ("" if none); the message is kept
 * per host thread, so ctx may be any context or NULL. */
const char *cgp_last_error(cgp_ctx ctx);
/* Number of compute units of the context's device (for sizing launches). */
int32_t cgp_device_cus(cgp_ctx ctx);

/* ------------------------------------------------------------------ meshes */

/* Upload a coarse P1 mesh and build k uniform 4-way refinements on the device
 * (Section 2.3, Eq. 18: each level has 4x the triangles of the one below).
 *   h_xy        [2*n_nodes]  node coordinates, (x0, y0, x1, y1, ...)
 *   h_tri       [3*n_tris]   triangles, counter-clockwise vertex ids
 *   h_dirichlet [n_nodes]    1 = homogeneous Dirichlet node, 0 = free
 *   k_levels    >= 0         number of refinements (the finest level is k)
 * Numbering of the hierarchy: level l+1 keeps the ids of level l; its other
 * nodes are the midpoints of the level-l edges, edge e (edges = sorted unique
 * (min id, max id) pairs in lexicographic order) getting id N_l + e.
 * Triangle t = (a,b,c) has children 4t..4t+3 = (a,mab,mca), (mab,b,mbc),
 * (mca,mbc,c), (mab,mbc,mca).  A midpoint is a Dirichlet node iff its edge has
 * exactly one adjacent triangle and both end points are Dirichlet nodes.
 * Level 0 also gets the Galerkin P1 stiffness matrix of the coarse Poisson
 * problems in CSR form (ascending columns), with Dirichlet rows replaced by
 * identity rows and Dirichlet columns removed, plus its Jacobi inverse
 * diagonal and fp32 copies.
 * Returns CGP_E_MESH if a vertex id is out of range, a triangle repeats a
 * vertex or has non-positive signed area.  Synchronous (setup call). */
cgp_status cgp_mesh_upload(cgp_ctx ctx, const double *h_xy, int64_t n_nodes,
                           const int32_t *h_tri, int64_t n_tris,
                           const uint8_t *h_dirichlet, int32_t k_levels, cgp_mesh *out);
/* Sizes of level `level` (0 = coarse .. k = finest).  n_edges is the edge
 * count of that level (0 for the finest level, whose edges are not built);
 * nnz is the stiffness nonzero count (level 0 only, else 0).  Any output may
 * be NULL.  Synchronous. */
cgp_status cgp_mesh_info(cgp_ctx ctx, cgp_mesh mesh, int32_t level, int64_t *n_nodes,
                         int64_t *n_tris, int64_t *n_edges, int64_t *nnz);
/* Number of refinement levels k of the mesh. */
cgp_status cgp_mesh_levels(cgp_ctx ctx, cgp_mesh mesh, int32_t *k_levels);
/* Copy level `level` back to the host: h_xy [2N], h_tri [3T], h_dirichlet [N],
 * h_edge_ends [2E] (edge e = (h_edge_ends[2e], h_edge_ends[2e+1]), min first).
 * Any output may be NULL.  Synchronous. */
cgp_status cgp_mesh_download(cgp_ctx ctx, cgp_mesh mesh, int32_t level, double *h_xy,
                             int32_t *h_tri, uint8_t *h_dirichlet, int32_t *h_edge_ends);
/* Copy the level-0 system matrix back: h_rowptr [N+1], h_col [nnz], h_val
 * [nnz], h_dinv [N] (any may be NULL).  Synchronous. */
cgp_status cgp_mesh_matrix(cgp_ctx ctx, cgp_mesh mesh, int32_t *h_rowptr, int32_t *h_col,
                           double *h_val, double *h_dinv);
/* Release a mesh and its workspaces.  Synchronous. */
cgp_status cgp_mesh_free(cgp_ctx ctx, cgp_mesh mesh);

/* ------------------------------------------------------------------ CGP steps 1 and 5 */

/* Restrict the finest-level velocity (d_uf, d_vf: [N_k]) to the coarse nodes by
 * injection (Eq. 19; under the hierarchical numbering coarse node i is fine
 * node i) and assemble the coarse right-hand side d_b [N_0] of K phi = b:
 *   kind = CGP_SRC_CURL: Eq. 12, b_i = -scale * int (dv/dx - du/dy) psi_i  (scale = B0)
 *   kind = CGP_SRC_DIV : Eq. 15, b_i = -scale * int (du/dx + dv/dy) psi_i  (scale = rho/dt)
 * with the element-constant derivatives of the P1 interpolant of the injected
 * velocity; b_i = 0 on Dirichlet rows.  (K is the positive stiffness matrix, so
 * this is the paper's Laplace equation multiplied by -1.)  d_uc, d_vc [N_0]
 * optionally receive the injected velocity (NULL to skip). */
cgp_status cgp_restrict(cgp_ctx ctx, cgp_mesh mesh, const double *d_uf, const double *d_vf,
                        int32_t kind, double scale, double *d_b, double *d_uc, double *d_vc);

/* ------------------------------------------------------------------ CGP steps 2 and 6 */

typedef struct {
    int32_t precision;    /* CGP_FP64 or CGP_FP32_IR                                    */
    int32_t guess;        /* CGP_GUESS_*                                                */
    double tol;           /* stop when ||b - K phi||_2 <= tol ||b||_2 (true fp64 residual) */
    double refine_delta;  /* CGP_FP32_IR: refine when the fp32 residual fell by this factor
                             since the last refinement (0 = default: 0.1 with Jacobi,
                             0.01 with the Chebyshev preconditioner)                    */
    int32_t max_iter;     /* cap on CG iterations per instance (0 = default 100000)      */
    cgp_model model;      /* network for CGP_GUESS_LEARNED                               */
    int32_t spmv_lanes;   /* lanes per matrix row of the general row-range stages (residual,
                             judge, persistent engine): 0 = default (4; 1 for the persistent
                             engine, whose workgroups own thousands of rows), else 1, 2, 4, 8 */
    int32_t blocks;       /* workgroups of the row-range and persistent engines: 0 = one per
                             compute unit (persistent: every co-resident workgroup slot)     */
    int32_t engine;       /* CGP_ENGINE_*                                                */
    int32_t launches_per_graph; /* CGP_ENGINE_STAGED: stages per replayed graph (0 = 16; even) */
    int32_t precond_degree; /* CGP_DEGREE_TUNED (-1): per instance, the degree cgp_autotune chose
                             for its mesh (this precision and deflation); otherwise
                             0 or 1: Jacobi M = diag(K); 2..8: Chebyshev polynomial of this
                             degree in D^-1 K over [hi/1000, hi] ([hi/30, hi] with
                             deflation), hi = max_i sum_j |K_ij|/K_ii (Gershgorin),
                             applied as that many steps of Chebyshev iteration for
                             K z = r from z = 0 (CGP_ENGINE_STAGED only)                */
    int32_t deflation;    /* 0: off.  1: subdomain deflation (an extension): CG runs on the
                             complement of a coarse space Z of aggregates (free-row
                             indicators; the tiled iteration's tiles from recursive
                             coordinate bisection, each bisected once more: two
                             aggregates per tile), x0 is corrected so that Z^T r = 0 and each
                             direction is made K-orthogonal to range(Z) (Nicolaides;
                             Saad, Yeung, Erhel, Guyomarc'h).  Needs the tiled iteration
                             (CGP_ENGINE_STAGED or AUTO), at most 2048 aggregates per mesh,
                             rows coupled to at most 4 aggregates: CGP_E_UNSUPPORTED
                             otherwise.  E = Z^T K Z is inverted on the host on first use
                             per mesh. */
    int32_t stage_budget; /* staged engines under graph capture: the stage launches recorded
                             (each deflated stage with its coarse step).  0 = 5/4 of the
                             launches the last uncaptured solve of the same launch records
                             needed, plus 8; at most 65536.  Launches past an instance's end
                             return at once; an instance not finished by the last one ends
                             with status CGP_SOLVE_ABORTED and its phi is not a solution.
                             Ignored outside capture. */
} cgp_solve_opts;

typedef struct {
    int32_t iters;        /* CG iterations                                          */
    int32_t refinements;  /* fp64 residual refinements (CGP_FP32_IR)                */
    int32_t status;       /* CGP_SOLVE_*                                            */
    int32_t guess_used;   /* CGP_GUESS_* actually used (LEARNED may fall back to GIVEN) */
    double rel_res;       /* final true ||b - K phi|| / ||b||                        */
    double rel_res_guess; /* ||b - K phi0|| / ||b|| of the initial guess used         */
} cgp_solve_stats;

/* Solve K phi = b on the level-0 mesh of each of n_inst instances with
 * preconditioned conjugate gradients (Jacobi or a Chebyshev polynomial, see
 * cgp_solve_opts.precond_degree), all instances in the same launches (Eqs. 12, 15;
 * the paper used GMRES(m)+ILU(0) for the same systems).
 *   h_meshes[i]  mesh of instance i (distinct meshes; one instance per mesh)
 *   h_d_b[i]     device pointer, right-hand side [N_0]
 *   h_d_phi[i]   device pointer [N_0]: the guess on entry for GUESS_GIVEN, the
 *                solution on exit
 *   h_d_prev1[i], h_d_prev2[i]  previous two solutions phi^{n-1}, phi^{n-2}
 *                (device pointers; required for GUESS_EXTRAP, which starts from
 *                2 phi^{n-1} - phi^{n-2}, and GUESS_LEARNED, whose network guess
 *                (h_opts->model, see cgp_model_predict) is kept only if its
 *                error in the energy norm |x - x*|_K, which CG minimises, is not
 *                above that of phi^{n-1}, else phi^{n-1} is used; the two are
 *                compared exactly through J(x) = x.Kx/2 - b.x = |x - x*|_K^2/2 + const);
 *                may be NULL otherwise.  They must not alias phi.
 *   d_stats      device array [n_inst], written when the solve completes.
 * CGP_FP64: every vector and product in fp64.  CGP_FP32_IR: fp32 matrix,
 * vectors and products with fp64 dot-product accumulation, refined by true
 * fp64 residuals b - K phi and fp64 solution updates.  ||b|| = 0 gives phi = 0.
 * With CGP_ENGINE_STAGED the call waits until every instance has finished
 * (results are complete once the stream reaches the enqueued work); with
 * CGP_ENGINE_PERSISTENT it only enqueues.  Numerical failures are reported in
 * d_stats (see cgp_solve_check). */
cgp_status cgp_poisson_solve(cgp_ctx ctx, int32_t n_inst, const cgp_mesh *h_meshes,
                             const double *const *h_d_b, double *const *h_d_phi,
                             const double *const *h_d_prev1, const double *const *h_d_prev2,
                             const cgp_solve_opts *h_opts, cgp_solve_stats *d_stats);
/* For callers that cannot allocate device memory while they run (tight serving loops,
 * harnesses that forbid hipMalloc, code that must not grow its footprint): one solve as
 * cgp_poisson_solve with n_inst = 1, allocating nothing.  Every buffer it needs beyond the
 * mesh's own data and the caller's vectors (CG vectors, partial sums, control state,
 * launch records, deflation coefficients) lives in a fixed library-owned device array of
 * CGP_NOALLOC_SCRATCH_BYTES per device, held until the process ends; its stage kernels are
 * enqueued one by one on the context's stream (no graph is instantiated) and the call
 * returns once the device reports completion, like CGP_ENGINE_STAGED.
 *   d_b, d_phi, d_prev1, d_prev2, h_opts, d_stats: as for cgp_poisson_solve (one instance;
 *   d_prev1/d_prev2 only for CGP_GUESS_EXTRAP).
 * Limits (CGP_E_INVALID, nothing enqueued): the solve must fit the array (100 bytes per row
 * plus the records of its workgroups: about 670000 rows); CGP_GUESS_LEARNED and
 * CGP_ENGINE_PERSISTENT are CGP_E_UNSUPPORTED; no graph capture.  The Chebyshev
 * preconditioner and deflation use the mesh's tiled plan of that degree and its deflation
 * data, which this call does not build: an earlier cgp_poisson_solve on the mesh with the
 * same degree and deflation (a set-up call, which may allocate) must have built them.
 * All calls on one device share the array and it keeps the last call's contents (the call
 * clears what must start at zero): calls that overlap on one GPU (other host threads or
 * contexts on other streams) race and must be serialised by the caller. */
#define CGP_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
cgp_status cgp_poisson_solve_noalloc(cgp_ctx ctx, cgp_mesh mesh, const double *d_b, double *d_phi,
                                     const double *d_prev1, const double *d_prev2,
                                     const cgp_solve_opts *h_opts, cgp_solve_stats *d_stats);
/* Synchronise and read n_inst stats back into h_stats (may be NULL); returns
 * CGP_OK, or CGP_E_NOCONV / CGP_E_BREAKDOWN / CGP_E_ABORTED for the first
 * failing instance. */
cgp_status cgp_solve_check(cgp_ctx ctx, int32_t n_inst, const cgp_solve_stats *d_stats,
                           cgp_solve_stats *h_stats);
/* Total number of stage kernels the staged engine has enqueued on this context
 * (including the launches of the last replayed graph that found every instance
 * already finished); for averaging per-launch time. */
int64_t cgp_stage_launches(cgp_ctx ctx);
/* Stage timing, for measuring the solver's kernels (not for production runs).  With
 * enable = 1 (which also zeroes the totals) the staged engine enqueues the stage kernels of
 * later solves one by one on the context's stream, in the same chunks it would replay as
 * graphs, each dispatch carrying its own start and stop HIP events (hipExtLaunchKernelGGL:
 * the interval is the kernel's execution, without the gaps between kernels); the call waits
 * for each chunk and adds each kernel's interval to the totals (the tiled or row-range
 * stage kernel, and the deflation coarse step).  Results are the same as without timing.
 * enable = 0 returns to graph replay.  Not during graph capture. */
cgp_status cgp_stage_timing(cgp_ctx ctx, int32_t enable);
/* Totals since timing was enabled: stage-kernel launches and their summed duration (us),
 * coarse-step launches and theirs.  Any output may be NULL. */
cgp_status cgp_stage_timing_read(cgp_ctx ctx, int64_t *h_stage_launches, double *h_stage_us,
                                 int64_t *h_coarse_launches, double *h_coarse_us);
/* Choose the preconditioner degree of each instance of a batch by timing (an extension of
 * the method: the paper fixes its solver).  For every candidate degree d in {1 (Jacobi),
 * 2, ..., 8} the call solves the whole batch at degree d, on the staged tiled engine with
 * this precision and deflation, each mesh's system for a unit source on its free rows from
 * zero to 1e-8 (the first solve of a candidate builds the tiled plans and is not timed;
 * the best of two timed solves counts, HIP events on the context's stream).  The fastest
 * candidate d* fixes the batch's length, the most iterations S* any instance needs at d*;
 * each instance then gets the lowest candidate degree at which it needs at most S*
 * iterations (a lower degree works on a smaller region per tile: fewer bytes per stage for
 * the same number of stages).  The choices become the meshes' degrees for solves with
 * precond_degree = CGP_DEGREE_TUNED (instances of one batched solve may run different
 * degrees).  They are cached by the batch's shapes (rows, nonzeros and widest row of each
 * mesh, in order), precision and deflation: a batch of the same shapes takes the cached
 * choices without solving.
 *   h_degree_out [n]      (may be NULL): the chosen degrees
 *   h_ms_out     [8]      (may be NULL): the batch's time at each candidate in ms (-1 where
 *                         a mesh did not fit the candidate's tiled plan or deflation, or an
 *                         instance did not converge)
 *   h_iters_out  [n * 8]  (may be NULL): each instance's iterations at each candidate (-1 as above)
 * Synchronous; allocates the tuning problem's vectors. */
#define CGP_DEGREE_TUNED (-1)
#define CGP_AUTOTUNE_CANDIDATES 8
cgp_status cgp_autotune(cgp_ctx ctx, int32_t n, const cgp_mesh *h_meshes, int32_t precision,
                        int32_t deflation, int32_t *h_degree_out, double *h_ms_out, int32_t *h_iters_out);

/* ------------------------------------------------------------------ CGP steps 3, 7 and 4 */

/* Prolong a coarse nodal field d_qc [N_0] to the finest level d_qf [N_k] with
 * the P1 shape functions, one level at a time (Eq. 20): nodes kept from the
 * coarser level copy their value, the midpoint of edge (a, b) gets
 * (q_a + q_b) * 0.5.  k = 0 copies. */
cgp_status cgp_prolong(cgp_ctx ctx, cgp_mesh mesh, const double *d_qc, double *d_qf);

/* Lorentz-force source of Eqs. 13-14 on the finest level from the prolonged
 * potential d_phif [N_k] and velocity d_uf, d_vf [N_k]:
 *   F_x = sigma B0 (-G_y - B0 u),  F_y = sigma B0 (G_x - B0 v)
 * where G is the nodal gradient of phi: the area-weighted mean of the
 * element-constant gradients of the triangles around the node (Eqs. 4, 7, 11;
 * sigma = the Stuart number N when rho = d = u_inf = B0 = 1, Eq. 24).
 * d_fx, d_fy [N_k] receive the force; d_grad_elem [2 T_k] optionally receives
 * the element gradients (gx, gy per triangle; NULL to skip). */
cgp_status cgp_lorentz_force(cgp_ctx ctx, cgp_mesh mesh, const double *d_phif,
                             const double *d_uf, const double *d_vf, double sigma, double B0,
                             double *d_fx, double *d_fy, double *d_grad_elem);

/* Velocity correction of Eqs. 16-17 (step 8 of Section 2.2) on the finest level:
 *   u = ut - scale G_x,  v = vt - scale G_y,  scale = dt / rho,
 * with G the nodal gradient of the prolonged pressure d_pf [N_k] (the same
 * area-weighted mean of element gradients as cgp_lorentz_force).  d_ut, d_vt
 * [N_k] hold the intermediate velocity of Eqs. 13-14; d_u, d_v [N_k] receive
 * the corrected velocity.  d_mask [N_k] uint8 or NULL: where bit 0 (u) or bit 1 (v)
 * is set that component keeps its intermediate value (its Dirichlet value from the
 * momentum step, the same mask as cgp_momentum_step's); NULL corrects every node.  In
 * place is allowed (d_u == d_ut, d_v == d_vt); d_u != d_v and neither is d_pf
 * (CGP_E_INVALID). */
cgp_status cgp_velocity_correct(cgp_ctx ctx, cgp_mesh mesh, const double *d_pf, const double *d_ut,
                                const double *d_vt, const uint8_t *d_mask, double scale, double *d_u,
                                double *d_v);

/* The force of the fluid on a body (Section 3's cylinder: drag and lift, and their
 * viscous parts), the traction integral of the Newtonian stress -p I + mu (grad w +
 * grad w^T) over the body's boundary edges of a level:
 *   F_p = -sum_edges (p_a + p_b)/2 n |ab|,   F_v = sum_edges mu (grad w + grad w^T)_t n |ab|
 * with n the unit normal out of the body (towards the fluid triangle t's third vertex)
 * and grad w the constant P1 gradient of (u, v) on t.
 *   d_edges   [3 n_edges] int32 (device): a, b (the edge's nodes), t (the triangle that
 *             owns the edge) of the level
 *   d_p, d_u, d_v  [N_level] fp64 (the prolonged pressure and the velocity)
 *   d_force   [5] fp64 (device) out: F_p (x, y), F_v (x, y), and the number of edges
 *             skipped because an index was out of range or a, b were not nodes of t
 * One workgroup with a fixed-order reduction (the result does not depend on timing).
 * Coefficients: C = 2 F / (rho u_inf^2 d). */
cgp_status cgp_surface_force(cgp_ctx ctx, cgp_mesh mesh, int32_t level, int64_t n_edges, const int32_t *d_edges,
                             const double *d_p, const double *d_u, const double *d_v, double mu, double *d_force);

/* The general restriction of Section 2.3, for a coarse mesh that is not nested in the
 * fine one: the P1 field of a level evaluated at arbitrary points (e.g. the nodes of
 * another coarse mesh).  Each point is located in a triangle of the level (barycentric
 * coordinates >= -1e-12; among several, e.g. on an edge, the triangle with the largest
 * smallest coordinate, the lowest id on a tie) and the field interpolated there.
 *   level      0..k
 *   n_pts      >= 0
 *   d_pts      [2 n_pts] fp64, (x, y) interleaved
 *   d_field    [N_level] fp64, the level's nodal values
 *   d_out      [n_pts] fp64: the interpolated values, NaN for a point outside the mesh
 *   d_tri      [n_pts] int32 or NULL: the containing triangle, -1 outside
 * The level's point locator (a uniform grid of triangle buckets) is built on the first call
 * for that level (a host synchronisation; CGP_E_INVALID under graph capture until then).
 * d_out must not be d_field or d_pts (CGP_E_INVALID). */
cgp_status cgp_interpolate(cgp_ctx ctx, cgp_mesh mesh, int32_t level, int64_t n_pts, const double *d_pts,
                           const double *d_field, double *d_out, int32_t *d_tri);

/* Step 4 of the CGP algorithm, Eqs. 13-14 (the general scheme Eq. 8): the
 * intermediate velocity (u~, v~) on the finest level from
 *   (rho/dt) M w~ + rho C(u^n) w~ + mu K w~ = (rho/dt) M w^n + M f,   w = u, v,
 * Galerkin P1 (Section 2.3): M the mass matrix, C(u^n)_ij = int psi_i (u^n . grad psi_j)
 * with u^n interpolated in P1, K the stiffness; f = (d_fx, d_fy), the nodal
 * Lorentz source (cgp_lorentz_force), interpolated in P1.  The time derivative uses
 * u^n (Eq. 8).  Dirichlet rows are identity rows: the boundary values are the
 * caller's, passed in d_ut / d_vt at those nodes.
 *   d_un, d_vn, d_fx, d_fy  [N_f] fp64 at the finest level's nodes (read only)
 *   d_mask       [N_f] uint8 or NULL: the Dirichlet rows of each component, bit 0 for u
 *                and bit 1 for v (Section 3's channel: inflow and cylinder 3, slip walls
 *                2, natural outflow 0); NULL: the mesh's Dirichlet nodes, both components
 *   d_ut, d_vt   [N_f] in: initial guess, with the boundary values at Dirichlet nodes;
 *                out: the intermediate velocity (updated in place)
 *   rho, mu, dt  > 0, >= 0, > 0 (finite)
 *   tol          relative residual ||b - A w|| <= tol ||b|| of each component (> 0)
 *   max_iter     >= 1
 *   h_stats      host, optional: per component iterations, status (CGP_SOLVE_*),
 *                final relative residual of the recurrence
 * Both components share one matrix (a row fixed for one component only is that
 * component's identity row inside the products) and are solved together by Jacobi-preconditioned
 * BiCGStab (van der Vorst) in fp64, two launches per iteration.  The matrix is
 * assembled on every call (it depends on u^n); its pattern (the finest level's
 * adjacency) and the workspace are built on the first call for a mesh.  The call
 * returns after the solve (it synchronises the context's stream); CGP_E_NOCONV or
 * CGP_E_BREAKDOWN when a component did not reach tol (its last iterate is in the
 * output).  Nodes of more than 32 neighbours: CGP_E_UNSUPPORTED.  d_ut and d_vt must
 * differ from each other and from the inputs (CGP_E_INVALID).  Not capturable. */
typedef struct {
    int32_t iters[2];
    int32_t status[2];
    double rel_res[2];
} cgp_momentum_stats;

cgp_status cgp_momentum_step(cgp_ctx ctx, cgp_mesh mesh, const double *d_un, const double *d_vn,
                             const double *d_fx, const double *d_fy, const uint8_t *d_mask, double rho,
                             double mu, double dt, double tol, int32_t max_iter, double *d_ut, double *d_vt,
                             cgp_momentum_stats *h_stats);

/* ------------------------------------------------------------------ learned initial guess */

/* A graph network on the coarse mesh that predicts the initial guess of a
 * solve from the current right-hand side b and the previous two solutions p1,
 * p2 (an extension of the paper's method; Section 2.2's sequence of solves
 * supplies the training data):
 *   features  [b/s_b, p1/s_p, p2/s_p, r_e/s_r, K d/s_r, d/s_d, dirichlet, 1] with
 *             e = 2 p1 - p2, d = p1 - p2, r_e = b - K e, s_* = RMS over the nodes
 *   encoder   h = relu(X W0 + c0) (8 -> 64); three layers
 *             h <- relu([h, mean of the neighbours' h] W_l + c_l) + h (128 -> 64)
 *   decoder   y = h w_d + c_d;  g = e + s_d y on free nodes, 0 on Dirichlet nodes
 *   smoother  guess = g after 4 damped Jacobi sweeps g <- g + (2/3) D^-1 (b - K g),
 *             which damp the high-frequency part of the network's error
 * Dense products use bfloat16 operands on the matrix cores with fp32
 * accumulation.  Parameters: cgp_model_param_count() floats, in the order
 * W0 [16x64] (rows 8..15 multiply zero padding), c0 [64], then W_l [128x64],
 * c_l [64] for l = 1..3, then w_d [64], c_d [1] (row-major).
 * Training minimises the energy norm (delta^T K delta) / N_free of delta =
 * (y - (target - e) / s_d) on free nodes with Adam (beta 0.9 / 0.999, eps 1e-8). */
int64_t cgp_model_param_count(void);
/* New model with seeded He-normal weights (splitmix64 stream) and zero biases.  The
 * network's shape is fixed: hidden must be 64 and layers 3 (message layers), else
 * CGP_E_UNSUPPORTED. */
#define CGP_MODEL_HIDDEN 64
#define CGP_MODEL_LAYERS 3
cgp_status cgp_model_create(cgp_ctx ctx, int32_t hidden, int32_t layers, uint64_t seed, cgp_model *out);
cgp_status cgp_model_free(cgp_ctx ctx, cgp_model model);
/* Copy the fp32 parameters out / in (h_params: cgp_model_param_count() floats).
 * Setting parameters resets the optimiser state.  Synchronous. */
cgp_status cgp_model_get_params(cgp_ctx ctx, cgp_model model, float *h_params);
cgp_status cgp_model_set_params(cgp_ctx ctx, cgp_model model, const float *h_params);
/* Enqueue one prediction: d_guess [N_0] receives the network's guess. */
cgp_status cgp_model_predict(cgp_ctx ctx, cgp_model model, cgp_mesh mesh, const double *d_b,
                             const double *d_prev1, const double *d_prev2, double *d_guess);
/* Loss and gradient for one sample with d_target = the solution.  h_loss (1)
 * and h_grad (cgp_model_param_count()) may be NULL.  Synchronous. */
cgp_status cgp_model_grad(cgp_ctx ctx, cgp_model model, cgp_mesh mesh, const double *d_b,
                          const double *d_prev1, const double *d_prev2, const double *d_target,
                          double *h_loss, float *h_grad);
/* Train on n_samples samples (device pointers, all on `mesh`) for `epochs`
 * epochs, one Adam step per sample, samples in a seeded shuffled order per
 * epoch.  h_loss_history [epochs] receives the mean loss of each epoch (may be
 * NULL).  Synchronous. */
cgp_status cgp_model_train(cgp_ctx ctx, cgp_model model, cgp_mesh mesh, int32_t n_samples,
                           const double *const *h_d_b, const double *const *h_d_prev1,
                           const double *const *h_d_prev2, const double *const *h_d_target,
                           int32_t epochs, double lr, uint64_t seed, double *h_loss_history);
/* Parameters to / from a file (8-byte tag, int64 count, float32 values). */
cgp_status cgp_model_save(cgp_ctx ctx, cgp_model model, const char *path);
cgp_status cgp_model_load(cgp_ctx ctx, const char *path, cgp_model *out);

/* ------------------------------------------------------------------ HIP graphs */

/* Begin capturing the context's stream; library calls made until
 * cgp_graph_end are recorded instead of executed (they must be the
 * asynchronous calls above, or cgp_poisson_solve on the staged engines as its
 * engine comment says).  The stream must not be the null stream.  A graph holds
 * the launch records of the solves it recorded until it is freed; it reads and
 * writes the vectors named at capture, and must not be launched after a mesh it
 * uses was freed.  A solve graph can be captured as a whole CGP step (restrict,
 * solve, prolong, Lorentz force, solve, prolong, velocity correction): one
 * graph launch per time step. */
cgp_status cgp_graph_begin(cgp_ctx ctx);
/* End the capture and instantiate it. */
cgp_status cgp_graph_end(cgp_ctx ctx, cgp_graph *out);
/* Launch a captured graph on the context's stream. */
cgp_status cgp_graph_launch(cgp_ctx ctx, cgp_graph graph);
cgp_status cgp_graph_free(cgp_ctx ctx, cgp_graph graph);

#ifdef __cplusplus
}
#endif
#endif /* CGP_H */
