/*
 * arb.h -- C ABI of the articulated-body Stokes solver hot path on gfx950.
 *
 * The library solves the constrained mobility problem of Balboa Usabiaga &
 * Delmotte, "A numerical method for suspensions of articulated bodies in
 * viscous flows" (arXiv:2107.10800), Sec. 2.3 Eq. linear_system:
 *
 *     [ M   -K   0  ] [lambda]   [ u_s ]
 *     [-K^T  0  C^T ] [  U   ] = [ -F  ]
 *     [ 0    C   0  ] [ phi  ]   [  B  ]
 *
 * for N blobs of radius a on M rigid bodies, with velocity constraints C U = B,
 * using the block-diagonal preconditioner of Sec. 3.1 inside restarted GMRES.
 *
 * Conventions (all entry points):
 *  - Floating point is IEEE double unless stated.  Vectors are AoS:
 *    positions / lambda / blob velocities as x0 y0 z0 x1 ...; per body
 *    U_p = (u, w), F_p = (f, tau) with the torque about the tracking point q_p;
 *    quaternions theta_p = (s, p1, p2, p3), scalar first, unit norm.
 *  - Blobs of one body are contiguous: body p owns blobs
 *    blob_offset[p] .. blob_offset[p+1]-1.
 *  - Host pointers are read during the call and never retained; the caller
 *    owns them.  `_dev` entry points take device pointers (hipMalloc'ed or
 *    torch tensors' data_ptr) and a hipStream_t (NULL = the context's stream);
 *    they are asynchronous with respect to the host and allocate nothing on
 *    the caller's behalf (the context's own workspace may grow on the first
 *    call at a larger size).
 *  - Return value: 0 success, > 0 warning (result usable), < 0 error (result
 *    undefined).  arb_last_error() gives the message of the last non-zero code.
 *  - One context per host thread; calls on one context are not thread safe.
 */
#ifndef ARB_H
#define ARB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define ARB_OK                 0
#define ARB_W_NOT_CONVERGED    1   /* GMRES hit max_iter; best iterate returned   */
#define ARB_W_PINV_USED        2   /* a pseudo-inverse replaced an inverse (Sec. 3.1) */
#define ARB_W_LEARNED_FALLBACK 3   /* learned body mobility rejected; exact used */
#define ARB_E_ARG             -1   /* bad argument / size / state not set        */
#define ARB_E_NOT_SPD         -2   /* blob mobility block not positive definite  */
#define ARB_E_BELOW_WALL      -3   /* a blob at z <= a with the wall on          */
#define ARB_E_DEVICE          -4   /* HIP runtime error                          */
#define ARB_E_NAN             -5   /* non-finite value met                       */
#define ARB_E_HOST            -6   /* host-side failure (memory allocation, a   */
                                   /* worker thread); no C++ exception leaves   */
                                   /* an entry point                            */

/* precision of the blob-blob mobility product (the Krylov solver is always FP64) */
#define ARB_FP64   0   /* pair sum in double                                   */
#define ARB_FP32C  1   /* pair sum in float: hi/lo split positions, float sums */
                       /* per 256-source tile, double sums across tiles        */
/* preconditioners */
#define ARB_PC_NONE    0
#define ARB_PC_BLOCK   1   /* Sec. 3.1, Eq. precond                          */
#define ARB_PC_LEARNED 2   /* body mobility N~_p from the learned network    */
#define ARB_PC_BODYFRAME 3 /* free-space blocks of each body type rotated into
                              each body (no per-solve factorisation; ignores the
                              wall inside the blocks)                         */

/* pair kernel choice (arb_options.pair_kernel) */
#define ARB_PAIR_AUTO      0  /* autotuned (wall RPY) / by size (single-blob bodies) */
#define ARB_PAIR_TARGET    1  /* target-parallel: ordered sums, bitwise reproducible */
#define ARB_PAIR_SYMMETRIC 2  /* each unordered pair once, FP64 atomic sums           */
#define ARB_PAIR_FMM       3  /* fast product for large N: Chebyshev-interpolation     */
                              /* multipole method (fmm_* options); an approximation   */
                              /* of every blob mobility product, FP32 arithmetic      */

/* body models */
#define ARB_MODEL_MULTIBLOB   0  /* rigid multiblob bodies, Eq. linear_system (Sec. 2.3) */
#define ARB_MODEL_SINGLE_BLOB 1  /* every body one blob at its tracking point with the
                                    generalised RPY tensor (Sec. 2.4), unknowns
                                    y = [U (6M); phi (Nc)] of Eq. linear_system_general,
                                    rows [U - N C^T phi; C U] = [N F; B]; unbounded,
                                    preconditioner NONE or BLOCK only; ARB_FP32C
                                    sums the tensor in float (units of a, float runs
                                    promoted to double) inside FP64 refinement  */

typedef struct arb_ctx arb_ctx;

typedef struct {
    int    device;     /* HIP device ordinal                                   */
    int    precision;  /* ARB_FP64 | ARB_FP32C                                 */
    int    wall;       /* 0 unbounded, 1 no-slip plane z = 0 (Sec. 2.3)        */
    double eta;        /* viscosity                                            */
    double a;          /* blob radius                                          */
    double tol;        /* GMRES relative residual ||b - A y|| / ||b||          */
    int    restart;    /* GMRES restart length (<= 256)                        */
    int    max_iter;   /* GMRES iteration cap (all cycles)                     */
    int    precond;    /* ARB_PC_*                                             */
    int    slices;     /* source slices of the pair kernel; 0 = autotune       */
                       /* (systems of at most 1,024 blobs sum over runs of 16  */
                       /* sources per workgroup instead, unless pair_kernel =  */
                       /* ARB_PAIR_SYMMETRIC)                                  */
    int    pair_kernel; /* 0 = autotuned choice, 1 = target-parallel kernel   */
                        /* (ordered reduction: bitwise reproducible),          */
                        /* 2 = symmetric kernel (each unordered pair once,     */
                        /* M_ji = M_ij^T; FP64 atomic sums, reproducible to    */
                        /* rounding only)                                      */
    int    graphs;     /* 0 = the GMRES iteration is captured once per Arnoldi */
                       /* index in HIP graphs and replayed (default),          */
                       /* 1 = plain launches                                   */
    int    model;      /* ARB_MODEL_MULTIBLOB (default) or ARB_MODEL_SINGLE_BLOB */
    /* ARB_PAIR_FMM only.  For single-blob bodies the generalised tensor of Sec. 2.4
     * is interpolated with force and torque channels.  The octree's root cube spans
     * the blobs; cells of a level are adjacent when their integer coordinates
     * differ by at most 1.  Pairs in adjacent leaves are summed directly; the
     * tensor between well-separated cells is replaced by its tensor-product
     * Chebyshev interpolant (fmm_order points per direction) in both
     * arguments (a listed cell with fewer blobs than proxies enters with its
     * blobs).  The error falls geometrically with fmm_order (max error
     * relative to the largest entry about 1e-4 at 5, 1e-5 at 6 for dense
     * suspensions).  The tree is rebuilt on the host whenever the state
     * changes (one device-to-host copy of the positions and a sort, on up to
     * 16 host threads; the tree does not depend on their number).  Products
     * are deterministic: the same positions and forces give the same result
     * bit for bit.                                                          */
    int    fmm_order;  /* Chebyshev points per direction, 2..8 (0 = 6)          */
    int    fmm_levels; /* leaf level L; 0 = chosen: with fmm_leaf > 0 the       */
                       /* shallowest level whose mean occupancy is <= fmm_leaf, */
                       /* else the level with the fewest pair evaluations per   */
                       /* product (direct pairs + M2L pairs, arb_fmm_stats),    */
                       /* going deeper from level 2 while they fall; never      */
                       /* deeper than the deepest level with a cell             */
                       /* side >= 2a; L <= 1 gives the direct sum               */
    int    fmm_leaf;   /* mean blobs per leaf aimed at (0 = see fmm_levels)     */
    int    left_precond; /* 0 = right preconditioning A P^-1 (default): the     */
                       /* Krylov residual is the true residual; 1 = left       */
                       /* preconditioning P^-1 A, the form Sec. 3.1 names: the */
                       /* Givens recursion tracks ||P^-1 (b - A y)||, a cycle  */
                       /* stops when that has fallen by the factor the true    */
                       /* residual still has to fall, and the stopping test is */
                       /* always on the true residual ||b - A y|| <= tol ||b|| */
    int    small_cycle; /* 0 = a small system (multiblob, FP64, block         */
                       /* preconditioner, right preconditioning, at most 128   */
                       /* blobs and 4,096 unknowns, assemblies of at most 64   */
                       /* rows) runs each GMRES restart cycle in one launch of */
                       /* one workgroup, with the stopping test on the device  */
                       /* (default); 1 = one kernel per operation, a host      */
                       /* stopping test per step                               */
    int    refine_final; /* ARB_FP32C refinement: 0 = once one correction has  */
                       /* been checked with the FP64 pair sum, a later one is  */
                       /* accepted without that product when its inner GMRES   */
                       /* residual plus 10x the FP32 error the checked one     */
                       /* showed (scaled to the current residual) is within    */
                       /* tol (default; arb_solve_info.residual_bounded = 1);  */
                       /* 1 = every solve ends with the FP64 residual of the   */
                       /* returned iterate                                     */
} arb_options;

typedef struct {
    int    iterations;      /* Arnoldi steps over all cycles                   */
    int    restarts;        /* completed cycles                                */
    double rel_residual;    /* ||b - A y|| / ||b|| of the returned iterate with
                               the FP64 pair sum (the stopping test), or the
                               bound on it when residual_bounded = 1          */
    double rel_residual_fp64; /* the same number (kept for callers that read it) */
    double t_build_ms;      /* preconditioner build                            */
    double t_solve_ms;      /* Krylov iterations incl. final residual          */
    int    pinv_used;       /* number of blocks inverted by pseudo-inverse     */
    int    history_len;     /* entries written to history                      */
    double history[1024];   /* relative residual estimate per iteration        */
    int    products_fp64;   /* blob mobility products with the FP64 pair sum   */
    int    products_fp32;   /* ... with the FP32 pair sum                      */
    int    precond_applies; /* preconditioner applications                     */
    int    one_launch_cycles; /* restart cycles run in one launch (small systems, */
                            /* arb_options.small_cycle)                         */
    int    residual_bounded; /* 1: ARB_FP32C, the last correction was accepted  */
                            /* on the bound of arb_options.refine_final = 0     */
                            /* (rel_residual is that bound, not an FP64 sum)    */
} arb_solve_info;

/* Work of the fast product's current tree (ARB_PAIR_FMM), filled by
 * arb_fmm_get_stats after a product has built it. */
typedef struct {
    int       levels;       /* leaf level L (0: one cell, the direct sum)        */
    int       order;        /* Chebyshev points per direction n                  */
    int       cells;        /* cells of all levels                               */
    int       leaves;       /* non-empty leaves                                  */
    long long near_pairs;   /* ordered blob pairs summed directly per product    */
    long long interactions; /* interaction-list entries (cell pairs)             */
    long long m2l_pairs;    /* M2L pairs evaluated per product: n^3 per proxy of */
                            /* each listed cell, or per blob when it holds fewer */
                            /* blobs than proxies                                */
    double    build_ms;     /* host time of the last tree build (incl. copies)   */
    unsigned long long plan_hash; /* arb_fmm_plan only: FNV-1a hash of the plan's */
                            /* index arrays (blob order, cells, lists, work      */
                            /* items, tables); equal plans give equal hashes     */
} arb_fmm_stats;

/* -------------------------------------------------------------- lifetime */
/* Create a context on opt->device.  Returns ARB_E_ARG for bad options. */
int  arb_create(arb_ctx **out, const arb_options *opt);
void arb_destroy(arb_ctx *ctx);
const char *arb_last_error(const arb_ctx *ctx);
/* Pair-kernel launch shape actually used (after autotuning): > 0 source
 * slices of the target-parallel kernel, < 0 the symmetric kernel with -value
 * source tiles per work item. */
int  arb_get_slices(const arb_ctx *ctx, int n_blobs);

/* -------------------------------------------------------------- bodies
 * Body partition and body-frame blob positions (Sec. 2.3: blobs r_i of body
 * p, r_i = q_p + R(theta_p) r_i^ref).  blob_offset: M+1 int32, nondecreasing,
 * blob_offset[0] = 0, blob_offset[M] = N.  r_ref: 3N body-frame positions.
 * body_type: M int32 (>= 0) used by ARB_PC_LEARNED, may be NULL. */
int arb_set_bodies(arb_ctx *ctx, int M, const int32_t *blob_offset,
                   const double *r_ref, const int32_t *body_type);

/* Body state x_p = {q_p, theta_p} (Sec. 2.1): q 3M, theta 4M (unit, scalar
 * first).  Recomputes blob positions (a GPU kernel) and the constraint rows. */
int arb_set_state(arb_ctx *ctx, const double *q, const double *theta);

/* Lab-frame blob positions r_i = q_p + R(theta_p) r_i^ref, 3N (Sec. 2.3). */
int arb_blob_positions(arb_ctx *ctx, double *r_out);

/* -------------------------------------------------------------- constraints
 * Links (Sec. 2.2, Eq. constraint / Eq. dg): link n joins body pq[2n] (+ end)
 * and body pq[2n+1] (- end; -1 = a fixed lab point dl_q).  dl_p, dl_q: 3P
 * body-frame arms; dldot_p, dldot_q: their time derivatives (NULL = passive,
 * B = 0).  nproj: P counts in 1..3 (NULL = 3); proj: 9P, the first nproj[n]
 * rows of proj[9n..] are body-p-frame directions d onto which the link's
 * velocity constraint is projected (NULL = e_x, e_y, e_z).  Each kept row
 * reads d.(u_p + w_p x l_p - u_q - w_q x l_q) = d.B_n, l = R dl (App. A).
 * Replaces previously set links.  ARB_E_ARG if links and rows together give
 * one articulated body more than 2048 constraint rows (the per-assembly
 * blocks of the preconditioner and the correction are sized for that). */
int arb_set_links(arb_ctx *ctx, int P, const int32_t *pq, const double *dl_p,
                  const double *dl_q, const double *dldot_p, const double *dldot_q,
                  const int32_t *nproj, const double *proj);

/* General rows (Sec. 2.2: a constraint may act on single components or on
 * one body): row k couples bodies pq[2k] and pq[2k+1] (-1 = none) with
 * body-frame (of body pq[2k]) coefficients coef[12k..] = (c_u_p, c_w_p,
 * c_u_q, c_w_q); it reads c.U = rhs[k].  Rows follow the link rows in phi.
 * Replaces previously set rows. */
int arb_set_rows(arb_ctx *ctx, int R, const int32_t *pq, const double *coef,
                 const double *rhs);

/* Number of constraint rows N_c and of unknowns n = 3N + 6M + N_c (6M + N_c
 * in the single-blob model). */
int arb_sizes(const arb_ctx *ctx, int *N, int *M, int *Nc, int64_t *n);

/* Statistics of the fast product's tree (ARB_PAIR_FMM).  ARB_E_ARG when the
 * context does not use the fast product or no product has built a tree yet. */
int arb_fmm_get_stats(const arb_ctx *ctx, arb_fmm_stats *out);

/* The fast product's octree for N blobs at pos (3N doubles, xyz per blob, host
 * memory, units of length), planned on the host with no device and no
 * context: the leaf level and work counts a product over these positions
 * would use (a = blob radius; order, levels, leaf as the fmm_* options, 0 for
 * their defaults); build_ms is the host time of the planning, plan_hash a
 * digest of the whole plan.  The planning runs on up to 16 host threads (one
 * per 65,536 blobs); the environment variable ARB_HOST_THREADS (1..16) caps
 * them, here and in the products' tree builds; the plan does not depend on the
 * count.  Returns ARB_E_ARG for bad sizes or options, ARB_E_NAN for a
 * non-finite position, ARB_E_HOST when host memory or a thread fails. */
int arb_fmm_plan(int N, const double *pos, double a, int order, int levels, int leaf,
                 arb_fmm_stats *out);

/* -------------------------------------------------------------- operators
 * u = M lambda over the context's blobs (Sec. 2.3 Eq. no-slip / Eq. RPY):
 * u_i = sum_j M_ij lambda_j over all j including i; 3N in, 3N out. */
int arb_mobility_apply(arb_ctx *ctx, const double *lambda, double *u);
int arb_mobility_apply_dev(arb_ctx *ctx, const double *lambda_dev, double *u_dev,
                           void *stream);

/* Stateless pair sum for loose blobs: pos 3N, lambda 3N, u 3N (device
 * pointers), using ctx's a, eta, wall and precision.  Blobs below the wall are
 * not checked here (use arb_check_wall). */
int arb_rpy_apply_dev(arb_ctx *ctx, int N, const double *pos_dev,
                      const double *lambda_dev, double *u_dev, void *stream);
/* Host-pointer version of arb_rpy_apply_dev; checks z > a when the wall is on. */
int arb_rpy_apply(arb_ctx *ctx, int N, const double *pos, const double *lambda,
                  double *u);

/* Allocation-free version of arb_rpy_apply_dev, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops, hosts
 * that forbid hipMalloc).  Same arguments and result; it always runs the
 * target-parallel kernel (ctx's slices, else a heuristic count, at most what
 * the scratch holds: 4 slices at the maximum size), so with
 * pair_kernel = ARB_PAIR_TARGET and the same slices it matches
 * arb_rpy_apply_dev bit for bit.  Every intermediate lives in one static
 * device array of 10 MiB per device, held until the process ends: N may not
 * exceed ARB_NOALLOC_MAX_BLOBS (ARB_E_ARG with a message otherwise), and the
 * fast product is refused (ARB_E_ARG).  Calls on one device share that array:
 * calls that overlap in time on one device (other host threads, other
 * streams) race and give undefined results.  No device memory is allocated
 * or freed. */
#define ARB_NOALLOC_MAX_BLOBS 65536
int arb_rpy_apply_noalloc_dev(arb_ctx *ctx, int N, const double *pos_dev,
                              const double *lambda_dev, double *u_dev, void *stream);

/* Body mobility of single-blob bodies (Sec. 2.4; ARB_MODEL_SINGLE_BLOB only):
 * UW = N FT with N the unbounded generalised RPY tensor (all ordered body
 * pairs, self blocks included) at the context's state.  FT: 6M (f, tau per
 * body), UW: 6M (u, w per body).  ARB_E_ARG in the multiblob model. */
int arb_body_mobility_apply(arb_ctx *ctx, const double *FT, double *UW);
/* Device-pointer version on stream (NULL = the context's stream). */
int arb_body_mobility_apply_dev(arb_ctx *ctx, const double *FT_dev, double *UW_dev,
                                void *stream);

/* out = A y for y = [lambda; U; phi] (Eq. linear_system); n doubles each.  In
 * the single-blob model y = [U; phi] and out = [U - N C^T phi; C U]. */
int arb_system_apply(arb_ctx *ctx, const double *y, double *out);
/* K U (3N) and K^T lambda (6M) (Eq. no-slip / Eq. balance). */
int arb_K_apply(arb_ctx *ctx, const double *U, double *out);
int arb_KT_apply(arb_ctx *ctx, const double *lambda, double *out);
/* Dense constraint rows in the lab frame: coef 12 Nc (c_u_p, c_w_p, c_u_q,
 * c_w_q), body pair 2 Nc, and B (Nc). */
int arb_constraint_rows(arb_ctx *ctx, double *coef, int32_t *pq, double *B);

/* -------------------------------------------------------------- preconditioner
 * Build the block-diagonal preconditioner of Sec. 3.1 for the current state
 * (per-body M_pp, batched Cholesky, N~_p, per-assembly G~_a).  Returns
 * ARB_W_PINV_USED if a pseudo-inverse was needed, ARB_E_NOT_SPD if some
 * M_pp is not positive definite. */
int arb_precond_build(arb_ctx *ctx);
/* z = P^-1 r (Eq. precond solved exactly), n doubles each. */
int arb_precond_apply(arb_ctx *ctx, const double *r, double *z);
/* Lower Cholesky factor of body p's blob mobility (3n_p x 3n_p row-major,
 * upper part zero), and N~_p (36, row-major); either may be NULL.  (When no
 * body has more than 256 rows the build forms M_pp^-1 without a factor and
 * this call factors the kept M_pp on the host.)  The
 * per-type preconditioners (ARB_PC_LEARNED, ARB_PC_BODYFRAME) have no per-body
 * factor: L must be NULL there (ARB_E_ARG otherwise). */
int arb_precond_block(arb_ctx *ctx, int p, double *L, double *Ntilde);

/* -------------------------------------------------------------- solve
 * Solve A y = b with b = [u_s; -F; B] (Eq. linear_system) by restarted
 * GMRES (right-preconditioned, or left with opt.left_precond) to
 * ||b - A y|| <= tol ||b|| in FP64.  With
 * ARB_FP32C the solve is GMRES iterative refinement: inner GMRES with the FP32
 * pair sum on the correction equation, residuals formed in FP64.  F: 6M;
 * u_slip: 3N or NULL (zero); y0: n or NULL (zero initial guess, Sec. 3.2.1
 * warm start otherwise).  Outputs (may be NULL): U 6M, phi N_c, lambda 3N.
 * info may be NULL. */
int arb_solve(arb_ctx *ctx, const double *F, const double *u_slip, const double *y0,
              double *U, double *phi, double *lambda, arb_solve_info *info);
/* Device-pointer version: F_dev 6M, u_slip_dev 3N or NULL, y_dev n (in: the
 * initial guess if warm != 0, out: the solution). */
int arb_solve_dev(arb_ctx *ctx, const double *F_dev, const double *u_slip_dev,
                  double *y_dev, int warm, arb_solve_info *info, void *stream);

/* -------------------------------------------------------------- time step
 * Explicit Euler update of every body (Sec. 4.3 step 3, applied per body):
 * q_p += dt u_p, theta_p <- theta_{w_p dt} . theta_p.  U: 6M.  The new state
 * becomes the context's state; q/theta (3M/4M, may be NULL) receive it. */
int arb_euler_update(arb_ctx *ctx, const double *U, double dt, double *q, double *theta);

/* Reconstruction of articulated bodies (Sec. 4.1, Eq. Pq_eq_z, Eq.
 * pseudo-inv-sol, Eq. reconst-up-COM).  An articulated body is a set of
 * bodies joined by links; for each, at the context's orientations and link
 * arms, the link equations read P q = -z with row block n of P q equal to
 * q_p - q_q and z_n = R(theta_p) dl_np - R(theta_q) dl_nq.  The tracking
 * points are replaced by q~ + q_COM, q~ = -P^+ z (the zero-mean minimum-norm
 * solution) and q_COM the mean of the current tracking points of that
 * articulated body.  An articulated body with a link to a fixed lab point
 * has no translational freedom: q = -P^+ z.  Bodies without links keep their
 * positions.  Loop-free articulated bodies then obey every link exactly;
 * with loops the links hold in the least-squares sense.  The result becomes
 * the context's state.  q (3M, may be NULL) receives it; g_inf (may be NULL)
 * the largest |component| of g_n over all links afterwards, g2 (may be NULL)
 * the sum of g_n . g_n.  ARB_E_ARG if an articulated body has more than 2048
 * bodies. */
int arb_reconstruct(arb_ctx *ctx, double *q, double *g_inf, double *g2);

/* Link residual g_n (Eq. constraint) at the context's state: g_inf and g2 as
 * for arb_reconstruct (either may be NULL).  The state is not changed. */
int arb_link_residual(arb_ctx *ctx, double *g_inf, double *g2);

typedef struct {
    int    solve_status;     /* return code of the step's solve (0 or a warning) */
    int    iterations;       /* its GMRES iterations                             */
    double rel_residual;     /* its FP64 relative residual                       */
    double t_build_ms;       /* its preconditioner build                         */
    double t_solve_ms;       /* its Krylov iterations                            */
    double g_inf_star;       /* max |g_n component| after the reconstruction     */
    double g2_star;          /* sum of g_n . g_n after the reconstruction        */
    int    corrected;        /* 1 if the correction ran                          */
    int    corr_iterations;  /* its largest step count over articulated bodies   */
    double corr_residual;    /* its largest final ||F||_2                        */
    double g_inf;            /* max |g_n component| at the end of the step       */
} arb_step_info;

/* One explicit Euler step with reconstruction and correction (Sec. 4.3):
 *  1. solve Eq. linear_system at the context's state (forces F, 6M; slip
 *     u_slip, 3N or NULL) for U; with warm != 0 GMRES starts from the last
 *     solution this context computed (by arb_solve or arb_step_euler) when its
 *     length matches, otherwise from zero;
 *  2.-3. every body moves by q_p += dt u_p, theta_p <- theta_{w_p dt} . theta_p,
 *     so each articulated body's mean tracking point moves by dt u_COM (Eq. ucom);
 *  4. every articulated body is rebuilt as in arb_reconstruct;
 *  5. if sum g_n . g_n >= delta, the correction of arb_correct_positions runs
 *     with tolerance corr_tol (> 0) and at most corr_max_iter (>= 0) steps.
 * The new state becomes the context's state; q (3M), theta (4M) and U (6M,
 * the velocities of step 1) receive it when not NULL; info (may be NULL) the
 * figures of the step.  Links are those set on the context (for arms that
 * change in time the caller sets them before each step).  Returns the solve's
 * code (a warning > 0 still completes the step) or an error. */
int arb_step_euler(arb_ctx *ctx, const double *F, const double *u_slip, double dt, double delta,
                   double corr_tol, int corr_max_iter, int warm, double *q, double *theta,
                   double *U, arb_step_info *info);

/* One explicit midpoint (RK2) step with reconstruction and correction (App. C):
 * U^k at the context's state (warm as for arb_step_euler); steps 2-5 of
 * arb_step_euler over dt/2 to the midpoint state; U^(k+1/2) there (GMRES
 * warm-started from U^k's solution); steps 2-5 over dt from the initial state
 * with U^(k+1/2).  Arguments as for arb_step_euler; U receives U^(k+1/2).
 * info: iterations summed over the two solves, rel_residual the larger, the
 * constraint figures of the full step (corrected = 1 if either stage
 * corrected, corr_iterations the larger).  Returns ARB_W_NOT_CONVERGED if
 * either solve did not converge, else the first warning of the two, or an
 * error. */
int arb_step_midpoint(arb_ctx *ctx, const double *F, const double *u_slip, double dt,
                      double delta, double corr_tol, int corr_max_iter, int warm, double *q,
                      double *theta, double *U, arb_step_info *info);

/* Link arms at one instant, for time steps whose arms change in time (Sec. 2.2:
 * arms dl(t) and their rates enter the link velocity rows; Sec. 5.1: the sliding
 * plates of the colonies): dl_p, dl_q (3P each, in the body frames of p and q),
 * dldot_p, dldot_q (3P each, their time derivatives; NULL = zero) and proj (9P,
 * the row projections as in arb_set_links, for rows that follow the arms; NULL
 * = keep the context's).  Link pairs and row counts stay those of the last
 * arb_set_links. */
typedef struct {
    const double *dl_p, *dl_q, *dldot_p, *dldot_q, *proj;
} arb_arms;

/* arb_step_euler for arms that change in time: the solve of step 1 uses the arms
 * set on the context (time t); once the bodies have moved the arms become `end`
 * (time t + dt), with which the rebuild, the check and the correction run and
 * which the context keeps.  ARB_E_ARG if end (or its dl_p, dl_q with links) is
 * NULL, ARB_E_NAN if it is not finite; the step is not started then. */
int arb_step_euler_arms(arb_ctx *ctx, const double *F, const double *u_slip, double dt,
                        double delta, double corr_tol, int corr_max_iter, int warm,
                        const arb_arms *end, double *q, double *theta, double *U,
                        arb_step_info *info);
/* arb_step_midpoint for arms that change in time (App. C with Sec. 2.2): U^k with
 * the context's arms (t); the half step's rebuild, check and correction and
 * U^(k+1/2) with `mid` (t + dt/2); the full step's with `end` (t + dt), which the
 * context keeps.  Errors as for arb_step_euler_arms. */
int arb_step_midpoint_arms(arb_ctx *ctx, const double *F, const double *u_slip, double dt,
                           double delta, double corr_tol, int corr_max_iter, int warm,
                           const arb_arms *mid, const arb_arms *end, double *q, double *theta,
                           double *U, arb_step_info *info);

/* Position/orientation correction (Sec. 4.2, Eq. min_probl, App. B): per
 * assembly, Levenberg-Marquardt on the link residuals g_n plus
 * ||dtheta_p||^2 - 1, exact Jacobian, mu = ||F||^2, until ||F||_2 <= tol or
 * max_iter steps.  Applies q <- q + dq, theta <- dtheta . theta to the
 * context state and writes it to q/theta (may be NULL).  iters (may be NULL)
 * receives the largest step count over assemblies; resid the largest final
 * link residual ||g||_2 per assembly. */
int arb_correct_positions(arb_ctx *ctx, double tol, int max_iter, double *q,
                          double *theta, int *iters, double *resid);

/* -------------------------------------------------------------- learned body mobility
 * A 7 -> 128 -> 128 -> 21 network (SiLU hidden layers, linear output, BF16
 * operands with FP32 accumulation on the matrix cores, FP32 master weights)
 * maps features x = [h/a, theta with s >= 0, onehot(type 0), onehot(type 1)]
 * of one body to y, the row-major lower triangle of L (diagonal entries as
 * log L_ii), L the Cholesky factor of D N~_p D with
 * D = diag(sqrt(6 pi eta a) I3, sqrt(8 pi eta a^3) I3); N~_p is
 * the body mobility [K_p^T (M^(pp))^-1 K_p]^-1 of the block preconditioner
 * (Sec. 3.1).  Parameters: 20,245 floats, flat [W1 (128x7), b1, W2 (128x128),
 * b2, W3 (21x128), b3], W row-major (out x in).  With ARB_PC_LEARNED the solve
 * takes N~_w = N~_p from the network; each body's blob block is the unbounded
 * body-frame mobility of its type (all bodies of one type must share r_ref),
 * rotated, with a rank-6 correction that makes the block solve exact for
 * N~_w: M~^-1 = A + Z_f D Z_f^T, D = N~_f N~_w^-1 N~_f - N~_f (A, Z_f, N~_f the
 * rotated unbounded blocks), so K^T M~^-1 K = N~_w^-1.  A non-finite
 * prediction (or |y| >= 80), or an N~_w or N~_f that is not positive definite,
 * makes the build fall back to the exact one (ARB_W_LEARNED_FALLBACK).  Inputs and outputs are standardised:
 * the network sees (x - in_mu)/in_sd and y = out_mu + out_sd * output. */
/* Standardisation constants (7, 7, 21, 21 floats; sd > 0); identity by default. */
int arb_mlp_set_scaling(arb_ctx *ctx, const float *in_mu, const float *in_sd,
                        const float *out_mu, const float *out_sd);
/* Load parameters (n = 20245) and reset the Adam state. */
int arb_mlp_set_params(arb_ctx *ctx, int n, const float *params);
int arb_mlp_get_params(arb_ctx *ctx, int n, float *params);
/* Y (B x 21) = network(X (B x 7)) with both standardisations applied, host arrays. */
int arb_mlp_forward(arb_ctx *ctx, int B, const float *X, float *Y);
/* Gradient (n = 20245 floats, parameter layout) of the mean squared error of
 * the standardised outputs, (T - out_mu)/out_sd, over the B x 21 outputs at
 * the current parameters; loss may be NULL. */
int arb_mlp_grad(arb_ctx *ctx, int B, const float *X, const float *T, float *grad,
                 double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on a batch in device
 * memory (X_dev B x 7, T_dev B x 21 floats).  loss (host, may be NULL) is the
 * batch loss before the step; passing it synchronises the stream. */
int arb_mlp_train_step_dev(arb_ctx *ctx, int B, const float *X_dev, const float *T_dev,
                           float lr, double *loss, void *stream);
/* Features of every body of the current state, M x 7 floats. */
int arb_mlp_features(arb_ctx *ctx, float *X);
/* Exact body mobilities of the current state from the block build (Sec. 3.1):
 * Nt (36 M doubles, row-major, may be NULL) and the network's training labels
 * target (21 M floats: lower triangle of chol(D N~_p D), log on the
 * diagonal, may be NULL). */
int arb_body_mobility(arb_ctx *ctx, double *Nt, float *target);

/* -------------------------------------------------------------- timing
 * When enabled, HIP events are recorded on the launching stream around every
 * launch of the blob-pair kernel (the dominant kernel).  arb_profile_read
 * waits for the recorded events, returns the summed kernel time (ms) and the
 * launch count since the last read, and clears them. */
int arb_profile(arb_ctx *ctx, int enable);
int arb_profile_read(arb_ctx *ctx, double *pair_ms, int *pair_launches);

#ifdef __cplusplus
}
#endif
#endif /* ARB_H */
