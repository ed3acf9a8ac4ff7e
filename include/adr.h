/*
 * adr.h -- C ABI of the MI355X ADR-amplitude solver.
 *
 * Solves the point-source Helmholtz equation in the factored form of Treister & Haber,
 * arXiv:1712.06091:
 *   u = a exp(-i w tau)                                    (Sec. 1, eq. new_u)
 *   Lap a - 2 i w grad(tau).grad(a) - i w (Lap tau) a
 *        - w^2 (|grad tau|^2 - kappa^2) a - i w gamma kappa^2 a = q exp(i w tau)
 *                                                          (Sec. 1, eq. ADR, plus the
 *                                                           absorbing term of Sec. 1)
 * discretized with the second-order upwind scheme H_2up (Sec. 2.2, eq. londUpwindDiff),
 * the averaging mass for the Lap(tau) term (Sec. 2.3) and the boundary condition
 * eq. BCADR, and solved by flexible GMRES(m) (Sec. 4.2) preconditioned by a multigrid
 * V-cycle on (1-beta) H_2up + beta H_1up (eq. precADRup) with Galerkin coarse
 * operators (eq. coarseGridMatrix).  Options select the paper's other systems on the same
 * kernels: the Krylov cycle (Alg. KrylovCycle), the central-advection system H_cen and
 * its two-stage solve (Alg. ADRlong), and the standard Helmholtz system (tau = NULL) with
 * the shifted-Laplacian preconditioner (eq. shift).
 *
 * Conventions (every entry point):
 *  - Grids are nodal with n[k] nodes along axis k (k = 0 is x, the fastest-varying
 *    index), spacing h on every axis, node j at position j*h.  Arrays are dense,
 *    row-major with x fastest: index = x + n[0]*(y + n[1]*z).
 *  - Complex arrays are interleaved (re, im): "c128" = 2 doubles per node, "c64" = 2
 *    floats per node (the storage of torch.complex128 / torch.complex64).
 *  - Unless stated otherwise, array pointers are DEVICE pointers on the current HIP
 *    device, owned by the caller; the library never frees them and keeps no reference
 *    to them after the call returns (adr_setup copies what it needs).
 *  - Calls return an adr_status and never throw.  On error nothing is half-written
 *    unless stated; adr_last_error() gives a message.
 *  - A context is bound to the stream given at setup; all work is enqueued on it.  A
 *    context is not thread-safe; use one per stream.
 */
#ifndef ADR_H_
#define ADR_H_

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ADR_OK = 0,
  ADR_EINVAL = 1,    /* bad argument: null pointer, bad size, source too close to a face */
  ADR_ENOMEM = 2,    /* device or host allocation failed                                 */
  ADR_EHIP = 3,      /* a HIP runtime call failed                                        */
  ADR_ENOCONV = 4,   /* solver hit maxit before tol; the best iterate is still written   */
  ADR_ENUMERIC = 5,  /* NaN/Inf in a residual norm                                       */
  ADR_ENOTSUP = 6    /* option combination not supported                                */
} adr_status;

typedef enum {
  ADR_PREC_FP64 = 0,   /* every step in complex FP64                                      */
  ADR_PREC_MIXED = 1   /* V-cycle in complex FP32; outer GMRES, residuals, coarsest FP64  */
} adr_precision;

typedef enum {
  ADR_RELAX_JACOBI = 0,  /* damped Jacobi sweeps (Sec. 3.1)                                */
  ADR_RELAX_GMRES = 1    /* Jacobi-preconditioned GMRES steps (Sec. 4.2)                   */
} adr_relax;

/* The discrete problem (Sec. 2).  kappa2, tau and gamma are DEVICE pointers to n
 * doubles each; gamma may be NULL (no absorption).  src[k] is the source node index
 * along axis k; it must be at least 2 nodes from every face.  With src[0] < 0 the
 * travel-time derivatives are plain differences of tau (no factoring, no near-source
 * rule).  tau may be NULL: tau = 0 everywhere, src is ignored, and the operator is the
 * standard second-order Helmholtz matrix H of eq. HelmholtzLinSystem (with the
 * absorbing term of Sec. 1); u = a.  Requires ndim in {2,3}, n[k] >= 5, h > 0,
 * omega > 0. */
typedef struct {
  int ndim;
  int n[3];
  double h;
  double omega;
  const double *kappa2;
  const double *tau;
  const double *gamma;
  int src[3];
} adr_problem;

/* Multigrid cycle used as the preconditioner. */
typedef enum {
  ADR_CYCLE_V = 0,   /* two-grid cycle applied recursively (Alg. TwoCycle)               */
  ADR_CYCLE_K = 1    /* Krylov cycle (Sec. 3.1, Alg. KrylovCycle): every coarse level    */
                     /* that is not the coarsest is solved by flexible GMRES(2) from     */
                     /* zero, preconditioned by the cycle one level down                 */
} adr_cycle;

/* Reaction term of the ADR operator.  Sec. 1 notes that a travel time solving the
 * eikonal equation |grad tau|^2 = kappa^2 removes -w^2 (|grad tau|^2 - kappa^2) a from
 * eq. ADR; a numerical tau satisfies it only approximately (and not across the kinks of
 * a first-arrival tau).  Both add the absorbing term -i w gamma kappa^2 of Sec. 1. */
typedef enum {
  ADR_REACTION_NUMERICAL = 0,  /* c = w^2 (kappa^2 - |g|^2) - i w gamma kappa^2 with the     */
                               /* numerical g = grad tau: kappa^2 enters the operator here   */
  ADR_REACTION_EIKONAL = 1     /* c = -i w gamma kappa^2: the term is dropped, as Sec. 1     */
                               /* does; requires tau (ADR_EINVAL with tau = NULL, where the  */
                               /* w^2 kappa^2 term is the Helmholtz operator's own)          */
} adr_reaction;

/* Advection scheme of the ADR operator (Sec. 2.2). */
typedef enum {
  ADR_ADV_UPWIND = 0,   /* second-order upwind, eq. londUpwindDiff (H_2up; blended with   */
                        /* first-order upwind by beta in the preconditioner)              */
  ADR_ADV_CENTRAL = 1   /* central, eq. londDiff (H_cen of eq. ADRLinSystemCentral); face */
                        /* nodes of an axis use the upwind operators there (Sec. 2.2.1)   */
} adr_advection;

/* Solver options; adr_default_options() fills the defaults named below. */
typedef struct {
  adr_precision prec;   /* default ADR_PREC_MIXED                                        */
  int levels;           /* multigrid levels; 0 = automatic: halve while (n-1) is even,    */
                        /* coarse n >= 5 and the grid has more than coarsest_max nodes   */
  int coarsest_max;     /* default 729                                                    */
  int nu[8];            /* relaxations per level (pre = post); default l+2 for 0-based    */
                        /* level l, i.e. 2 on the finest, 3 on the next (Sec. 4.2)        */
  adr_relax relax[8];   /* default JACOBI on level 0, GMRES on coarser levels (which    */
                        /* must relax by GMRES); GMRES on level 0 is the paper's choice  */
                        /* (Sec. 4.2), not with adjoint solves or rescaled cycles        */
  double jacobi_weight; /* default 0.8                                                    */
  double beta;          /* preconditioner blend of eq. precADRup; default 0.25 (Sec. 4.2) */
  int restart;          /* FGMRES restart length m; default 5 (Sec. 4.2); max 8           */
  int use_graph;        /* capture each V-cycle in a hipGraph; default 1                 */
  adr_cycle cycle;      /* default ADR_CYCLE_V                                            */
  double kcycle_threshold; /* Krylov cycle: keep only the first coarse GMRES step when its */
                        /* residual is <= this times the initial one; default 0.1       */
                        /* (Sec. 4.2.2); 0 always takes both steps                       */
  int coarse_split;     /* Galerkin-stencil apply on coarse levels: 1 = one lane per     */
                        /* node, 4 = four wavefronts per 64 nodes, 8 = LDS z-marching    */
                        /* tiles (3D levels with rows of <= 129 nodes and >= 8 planes    */
                        /* per slab; one lane elsewhere), 0 (default) = the              */
                        /* fastest per level, timed at setup and cached per grid shape   */
                        /* and precision for the process                                 */
  int tail_max_nodes;   /* V-cycle: coarse levels from the first one with at most this   */
                        /* many nodes down to the coarsest in one single-workgroup       */
                        /* kernel.  Disabled: must be 0 (the default); any other value   */
                        /* makes adr_setup return ADR_ENOTSUP                            */
  int full_cycles;      /* 1: every FGMRES restart cycle takes `restart` steps, the      */
                        /* convergence test only at cycle ends (batched solves always    */
                        /* run this way); default 0: stop inside a cycle once the        */
                        /* residual estimate reaches tol                                 */
  double shift_alpha;   /* alpha >= 0: the multigrid cycle works on the shifted operator */
                        /* A_beta - i alpha w^2 diag(kappa^2) (Sec. 3.1, eq. shift; the  */
                        /* paper's Helmholtz runs use 0.2 with tau = NULL) while FGMRES  */
                        /* solves the unshifted system; default 0 (no shift)             */
  adr_advection advection; /* default ADR_ADV_UPWIND; applies to the solved operator and */
                        /* to the preconditioner                                          */
  double outer_beta;    /* blend of the operator FGMRES solves: 0 (default) = H_2up,      */
                        /* 1 = H_1up (eq. 1up, the first stage of Alg. ADRlong)          */
  int rescaled;         /* 1: the cycle preconditions M A M^{-1} (M = diag(exp(-i w tau)), */
                        /* eq. ADRcenRescaled): its fine level is the phase-rescaled      */
                        /* operator and its coarse levels the Galerkin products of that   */
                        /* (the second stage of Alg. ADRlong); the solve stays in a, which */
                        /* gives the same iterates since M is unitary.  Not with the      */
                        /* adjoint or batch calls (ADR_ENOTSUP).  Default 0               */
  int pipeline_max_nodes; /* coarse levels with at most this many nodes relax by the    */
                        /* pipelined GMRES step (one launch per Arnoldi step: the        */
                        /* orthogonalization of step k-1 and the apply of step k share   */
                        /* it, the apply formed by linearity from stored products).  Same */
                        /* result up to rounding.  Default 2^31 - 1 (every coarse        */
                        /* level); 0 = the two-launch steps everywhere                   */
  adr_reaction reaction; /* default ADR_REACTION_NUMERICAL                                */
  int kcycle_levels;    /* Krylov cycle: the flexible-GMRES coarse solve on coarse levels */
                        /* 1..kcycle_levels only, the plain recursion of the V-cycle     */
                        /* below (a Krylov acceleration of the top of the hierarchy);    */
                        /* default 0 = every level                                        */
  int fine_tiles;       /* 1 (default): on 3D complex-FP32 finest levels with rows of at  */
                        /* most 257 nodes and at least 16 planes, the Jacobi sweeps and  */
                        /* the residual stage the iterate in LDS z-marching tiles (the   */
                        /* same arithmetic) if a setup-time timing finds them at least   */
                        /* 1% faster; 2: wherever they apply; 0: one lane per node       */
  int batch_merge;      /* adr_setup_batch: 1 = one group for problems of different grid  */
                        /* shapes when they nest under the largest (no more levels, no    */
                        /* more nodes on any level): every launch covers all problems,    */
                        /* each on its own grid (LDS tiles off; see adr_setup_batch);     */
                        /* 0 (default) = one group per grid shape                        */
} adr_options;

typedef struct {
  int outer_iters;      /* FGMRES iterations (= preconditioner applications)             */
  int restarts;
  double relres;        /* final true relative residual ||q_hat - A a|| / ||q_hat||, A    */
                        /* the solved operator (H_2up, or as set by outer_beta/advection) */
  double setup_ms;      /* wall time of the setup that built the context                 */
  double solve_ms;      /* adr_solve wall time                                           */
} adr_stats;

typedef struct adr_ctx adr_ctx;

/* Host: fill *o with the defaults above. */
void adr_default_options(adr_options *o);

/* Build the context: ADR coefficients from tau (Sec. 2.1, eq. travel_time_coeff), the
 * fine operator data, the Galerkin hierarchy of A_beta and the coarsest inverse.
 * `stream` is a hipStream_t (NULL = default stream).  The caller's arrays may be freed
 * after return.  *out is NULL on error. */
adr_status adr_setup(const adr_problem *prob, const adr_options *opt, void *stream, adr_ctx **out);

/* Free everything the context owns.  NULL is a no-op. */
void adr_destroy(adr_ctx *ctx);

/* y = A_beta x on the fine grid in FP64: the context's ADR operator with advection blend
 * beta (0 = H_2up, 1 = H_1up; with central advection H_cen, beta only acting on face
 * nodes; the Helmholtz H when tau was NULL), never shifted.  x and y c128 of n nodes,
 * distinct buffers.  Enqueued on the context stream. */
adr_status adr_apply(adr_ctx *ctx, double beta, const void *x_c128, void *y_c128);

/* One preconditioner application z = M^{-1} r: the configured cycle (a V-cycle, Alg.
 * TwoCycle applied recursively, or a Krylov cycle, Alg. KrylovCycle) on A_beta (shifted
 * when shift_alpha > 0, on the rescaled operator when `rescaled`) from a zero guess, in
 * the context's precision; r and z c128, distinct.  The Krylov cycle is
 * not linear in r (it is homogeneous: scaling r scales z).
 * Enqueued on the context stream; no host synchronization. */
adr_status adr_vcycle(adr_ctx *ctx, const void *r_c128, void *z_c128);

/* Solve A a = q exp(i w tau) by FGMRES(m) preconditioned by the configured cycle
 * (Sec. 4.2); A = H_2up by default, H_1up with outer_beta = 1, H_cen with central
 * advection, the Helmholtz H (and a = u) when tau was NULL.  q: c128 right-hand
 * side of the Helmholtz equation (a point source is e_src / h^ndim).  a: c128, in =
 * initial guess when use_initial_guess != 0 (else ignored and zero is used), out =
 * amplitude.  Stops when the true relative residual is <= tol or after maxit FGMRES
 * iterations (ADR_ENOCONV, best iterate written).  Synchronizes the stream.  stats may
 * be NULL. */
adr_status adr_solve(adr_ctx *ctx, const void *q_c128, void *a_c128, double tol, int maxit,
                     int use_initial_guess, adr_stats *stats);

/* Adjoint solve (not in the paper; the gradient of a receiver misfit needs it):
 * A^H lam = s exp(i w tau), A the operator adr_solve solves (H_2up by default; not with a
 * rescaled cycle: ADR_ENOTSUP), with the conjugate-transposed fine operator and the
 * conjugate-transposed multigrid hierarchy ((P^T A P)^H = P^T A^H P, P real), built on
 * the first call.  For J = 1/2 ||R u - d||^2, u = a exp(-i w tau), the right-hand side is
 * s = R^T (R u - d) (see adr_adjoint_source); then dJ/dkappa2 = adr_grad_kappa2(a, lam).
 * Same arguments, precision and stopping rule as adr_solve.  Synchronizes the stream. */
adr_status adr_solve_adjoint(adr_ctx *ctx, const void *s_c128, void *lam_c128, double tol, int maxit,
                             int use_initial_guess, adr_stats *stats);

/* y = A^H x in FP64, A the operator adr_solve solves (conjugate transpose of adr_apply
 * with beta = outer_beta); x, y c128, distinct.  Enqueued. */
adr_status adr_apply_adjoint(adr_ctx *ctx, const void *x_c128, void *y_c128);

/* grad[i] += -Re(conj(lam_i) c'_i a_i): the kappa^2 derivative of the misfit at fixed
 * travel time, dH_2up/dkappa2_i = c'_i e_i e_i^T through the reaction term, with
 * c'_i = w^2 - i w gamma_i (ADR_REACTION_NUMERICAL) or -i w gamma_i (ADR_REACTION_EIKONAL).
 * a, lam c128; grad FP64 device array of n nodes, accumulated into.  Enqueued. */
adr_status adr_grad_kappa2(adr_ctx *ctx, const void *a_c128, const void *lam_c128, double *grad);

/* Receivers: r_k = u[idx_k] - d_k for k < nrec (idx: device int32 linear node indices;
 * d, r: c128 device arrays of nrec).  If misfit != NULL (host), *misfit = 1/2 sum |r_k|^2
 * and the stream is synchronized; otherwise enqueued only. */
adr_status adr_receiver_residual(adr_ctx *ctx, const void *u_c128, const int *idx, const void *d_c128, int nrec,
                                 void *r_c128, double *misfit);

/* For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): adr_receiver_residual without a
 * context.  r_k = u[idx_k] - d_k for k < nrec, enqueued on `stream` (a hipStream_t; NULL =
 * the default stream).  If misfit != NULL (host), *misfit = 1/2 sum |r_k|^2, summed in the
 * same order as adr_receiver_residual (same value bit for bit), and the stream is
 * synchronized.  The misfit's partial sums live in a fixed device array inside the
 * library (512 doubles, 4 KiB, one copy per GPU, held until the process ends); nothing
 * is allocated.  Every call on a GPU shares that array, which keeps the last call's
 * partials: calls that overlap on one GPU (other threads, other streams) race.
 * ADR_EINVAL for a NULL array pointer or nrec outside [1, ADR_NOALLOC_MAX_REC];
 * adr_last_error(NULL) gives the message. */
#define ADR_NOALLOC_MAX_REC (1 << 26)
adr_status adr_receiver_residual_noalloc(const void *u_c128, const int *idx, const void *d_c128, int nrec,
                                         void *r_c128, double *misfit, void *stream);

/* Adjoint source s = R^T r: s = 0, then s[idx_k] += r_k for k in order (repeated indices
 * accumulate).  s: c128 of n nodes.  Enqueued. */
adr_status adr_adjoint_source(adr_ctx *ctx, const int *idx, const void *r_c128, int nrec, void *s_c128);

/* u = a exp(-i w tau) (eq. new_u); a, u c128 (may alias).  Enqueued, no sync. */
adr_status adr_wavefield(adr_ctx *ctx, const void *a_c128, void *u_c128);

/* Copy the fine-level coefficients out (FP64 device arrays of n nodes each):
 * g (ndim planes, axis k at g + k*n: d tau / d x_k), L (Lap tau), c (c128 reaction
 * w^2 (kappa^2 - |g|^2) - i w gamma kappa^2).  Any pointer may be NULL. */
adr_status adr_get_coefficients(adr_ctx *ctx, double *g, double *L, void *c_c128);

/* Multigrid level information (host out-params).  level 0 = finest.  nodes[k] = grid
 * size along axis k; *stencil_points = stored stencil size (0 for the matrix-free fine
 * level, 21 in 2D / 81 in 3D on Galerkin levels). */
adr_status adr_level_info(adr_ctx *ctx, int level, int *nodes, int *stencil_points);

/* Galerkin-apply variant in use on coarse level `level`, 1 <= level <= levels - 2 (host
 * out-param): 1 = one lane per node, 4 = four wavefronts per 64 nodes, 8 = LDS tiles
 * (adr_options.coarse_split, or the setup-time timing when that is 0).  ADR_EINVAL for
 * the fine level, the coarsest level (solved by its dense inverse), a level out of range
 * or a NULL pointer. */
adr_status adr_level_split(adr_ctx *ctx, int level, int *split);
int adr_num_levels(const adr_ctx *ctx);

/* The setup-time autotuner's table (process-wide): for every coarse-level shape and
 * precision timed so far, the Galerkin-apply variant (1, 4, 8) and, for the LDS tiles,
 * the z-slab count of the launch, with the measured time of 8 launches.
 * adr_tuning_table_write writes it as text to `path` (host string; one line per entry:
 * ndim nx ny nz real_bytes variant slabs ms) and returns the number of entries, -1 if
 * the file cannot be written.  adr_tuning_table_read loads such a file into the table
 * (later setups on those shapes take the entries instead of timing) and returns the
 * number of entries read, -1 if the file cannot be opened or holds a malformed entry.
 * Not thread-safe against concurrent adr_setup calls. */
int adr_tuning_table_write(const char *path);
int adr_tuning_table_read(const char *path);

/* Copy a Galerkin level's stencil (level >= 1) out as c128: stencil_points planes of
 * that level's node count, plane p holding the coefficient of neighbour offset
 * offsets[3p..3p+2] = (dx, dy, dz); offsets is a HOST int array of 3*stencil_points
 * (may be NULL).  Entries that point outside the grid are zero. */
adr_status adr_get_level_stencil(adr_ctx *ctx, int level, void *planes_c128, int *offsets);

/* Batched shots: `count` independent problems (own source, medium, tau and omega each;
 * any mix of grid sizes) solved together, the batched point sources of Sec. 4.2 (one
 * solve per source).  adr_setup_batch groups the problems by grid shape; each group's
 * contexts live in one device arena at a constant stride, so every kernel of a group
 * runs once for all its problems (one launch per phase), on one of `nstreams` (1..64)
 * non-blocking streams of default priority (group g on stream g % nstreams).
 * adr_solve_batch runs one FGMRES per problem with full restart cycles (see
 * adr_options.full_cycles; the options' own value is ignored) so that the problems of a
 * group stay in lockstep; converged problems are masked off on the device, and groups
 * advance independently.  Per problem the result equals adr_solve with full_cycles = 1
 * bit for bit.  With batch_merge = 1 (and nesting shapes) all problems form one group:
 * the arena holds one slot per problem in a common layout sized for the largest, each
 * launch covers every problem on its own grid of the launch's level (a problem whose
 * hierarchy ends above that level is skipped; one whose coarsest level it is applies its
 * coarsest inverse there), with the largest problem's variants and block counts; results
 * then match adr_solve up to rounding (different reduction partitions), not bit for bit.  q[i], a[i]: per-problem c128 device arrays as in adr_solve (zero initial
 * guess; a[i] is written when problem i finishes).  stats: host array of count entries,
 * or NULL.  Returns ADR_OK if every problem converged, else the first
 * non-convergence/error status; every a[i] holds its best iterate. */
typedef struct adr_batch adr_batch;
adr_status adr_setup_batch(int count, const adr_problem *probs, const adr_options *opt, int nstreams,
                           adr_batch **out);
adr_status adr_solve_batch(adr_batch *b, const void *const *q_c128, void *const *a_c128, double tol, int maxit,
                           adr_stats *stats);
int adr_batch_size(const adr_batch *b);
int adr_batch_groups(const adr_batch *b);          /* launch groups (1 when merged); 0 for NULL */
adr_ctx *adr_batch_context(adr_batch *b, int i);   /* borrowed; owned by the batch */
void adr_destroy_batch(adr_batch *b);               /* NULL is a no-op */

/* First-arrival travel time for the ADR coefficients, on the GPU: the factored eikonal
 * equation |tau0 grad tau1 + tau1 grad tau0|^2 = kappa^2, tau = tau0 tau1, tau0 = |x - x0|
 * (Sec. 1, eq. factoredEikonal), discretized with first-order one-sided differences of
 * tau1 towards the upwind neighbour of each axis and solved by fixed-point sweeps (the
 * parallel counterpart of the paper's factored fast marching): every sweep recomputes all
 * nodes from the previous sweep's values and keeps the smaller value, until a sweep
 * changes nothing.  Each node's candidate uses the largest set of axes with a causal
 * root, is held to tau_i <= tau_j + 1.1 h max(kappa_i, kappa_j) over its neighbours, and
 * falls back to the unfactored first-order Godunov update where that fails.
 * n[k], src[k]: HOST int arrays, axis 0 = x (as in adr_problem); kappa2: DEVICE, N
 * doubles (N = product of n); tau: DEVICE output, N doubles (tau(src) = 0); work: DEVICE
 * scratch of N + 1 doubles owned by the caller; max_sweeps >= 1; *sweeps (host, may be
 * NULL) = the number of sweeps that changed a value.  Enqueued on `stream` (hipStream_t,
 * NULL = default); synchronizes it every 32 sweeps.  ADR_ENOCONV if max_sweeps sweeps
 * all changed something (tau holds the last iterate); ADR_EINVAL for bad sizes or a
 * source outside the grid (message in adr_last_error(NULL)). */
adr_status adr_eikonal(int ndim, const int *n, double h, const double *kappa2, const int *src, double *tau,
                       double *work, int max_sweeps, int *sweeps, void *stream);

/* Kernel classes that adr_timer_start can time. */
typedef enum {
  ADR_TIMER_FINE_JACOBI = 0,    /* damped Jacobi sweep on the matrix-free finest level    */
  ADR_TIMER_FINE_RESIDUAL = 1,  /* V-cycle residual on the finest level                   */
  ADR_TIMER_COARSE_APPLY = 2,   /* Galerkin-stencil apply (GMRES relaxation and residual) */
  ADR_TIMER_COARSE_ORTH = 3,    /* GMRES-relaxation orthogonalization step               */
  ADR_TIMER_TRANSFER = 4,       /* restriction and prolongation                           */
  ADR_TIMER_OUTER_MATVEC = 5,   /* FP64 H_2up apply with fused Arnoldi dots (FGMRES)      */
  ADR_TIMER_OUTER_ORTH = 6,     /* FP64 Gram-Schmidt passes of the outer FGMRES           */
  ADR_TIMER_COARSE_TAIL = 7,    /* single-workgroup coarse tail of the V-cycle            */
  ADR_TIMER_FINE_GMRES = 8      /* matrix-free apply of the finest level's GMRES relaxation */
} adr_timer_kind;

/* Benchmark instrumentation.  adr_timer_start(ctx, kind, level) makes every later launch
 * of that kernel class (on `level`, or on any level if level < 0) record a pair of HIP
 * events on the context stream, up to 65536 launches (later ones go untimed).  adr_timer_stop synchronizes the
 * stream and returns (host out-params, any may be NULL) the summed kernel time in ms,
 * the number of timed launches and their algorithmic bytes: every array the kernel reads
 * or writes counted once per node (stencil neighbours of a vector count once).  Timing
 * adds an event record before and after each timed launch and nothing else. */
adr_status adr_timer_start(adr_ctx *ctx, int kind, int level);
adr_status adr_timer_stop(adr_ctx *ctx, double *ms, int *launches, double *bytes);

/* Two-stage solve of H_cen a = q_hat (Sec. 3.2, Alg. ADRlong).  `first` and `second`
 * are contexts on the same problem: adr_two_stage_options fills their options as in
 * Sec. 4.2 (first: H_1up solved and preconditioned, beta = outer_beta = 1, Krylov
 * cycle; second: central advection, beta = 0, shift_alpha = 0.2, rescaled, Krylov
 * cycle), starting from the defaults and keeping `prec` of *first on entry.
 * adr_solve_two_stage runs the first stage from zero to tol_first or maxit_first
 * iterations (5 and 1e-2 in the paper; not converging there is not an error), then the
 * second from that iterate to tol.  q, a as in adr_solve; st_first/st_second may be
 * NULL.  Returns the second stage's status (the first stage's on a failure there). */
void adr_two_stage_options(adr_options *first, adr_options *second);
adr_status adr_solve_two_stage(adr_ctx *first, adr_ctx *second, const void *q_c128, void *a_c128, double tol_first,
                               int maxit_first, double tol, int maxit, adr_stats *st_first, adr_stats *st_second);

const char *adr_strerror(adr_status s);
const char *adr_last_error(const adr_ctx *ctx);   /* NULL ctx: last setup error */

#ifdef __cplusplus
}
#endif
#endif /* ADR_H_ */
