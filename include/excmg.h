/*
 * excmg.h - C ABI of the MI355X (gfx950) EXCMG solver for the 3D biharmonic equation
 *
 *     Delta^2 u = f on (0,1)^3,
 *     u = g1 and du/dn = g2 on the boundary       (first kind,  bc_kind = 1), or
 *     u = g1 and d2u/dn2 = g2 on the boundary     (second kind, bc_kind = 2),
 *
 * discretised by the 25-point scheme and solved by the extrapolation cascadic multigrid
 * method (Pan, He & Ni, arXiv:1901.05118: problem statement eqs. bvp, BC, BC2 in Sec. 1;
 * scheme and boundary treatment in Sec. 2; cascade in Sec. 4.1, Algorithm 1; extrapolation
 * and interpolation in Sec. 4.2; Bi-CG in Sec. 5, Algorithm 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * All arrays are FP64.  A "node array" on a grid of N cells per axis holds (N+1)^3 values,
 *    node (i,j,k) at x = i/N, y = j/N, z = k/N stored at index (k*(N+1) + j)*(N+1) + i.
 *    An "interior vector" holds the (N-1)^3 unknowns (nodes 1..N-1 on every axis) in the same
 *    x-fastest order.
 *  * g1: read on every boundary node (faces, edges and corners).  g2: read on face-interior
 *    nodes only; first kind = outward normal derivative, so on the face x = 0 it is -du/dx
 *    and on x = 1 it is +du/dx; second kind = d2u/dx2 on x faces (likewise y, z).
 *    f: read on interior nodes only.
 *  * Pointers may be device (HBM) or host memory; the library detects which with
 *    hipPointerGetAttributes and stages host arrays through device memory.  The caller owns
 *    every array it passes; the library keeps no pointer after a call returns.
 *  * Work is issued on the stream set with excmg_set_stream (default: the null stream) and
 *    every entry point returns after its results are complete.
 *  * The library holds one context per process (levels, workspace, cached factors).  Calls
 *    are not thread-safe.
 *  * Return codes: EXCMG_OK (0) or a negative code; excmg_last_error() describes the last
 *    failure.  On EXCMG_ENOCONV the outputs hold the last iterate (the per-level records say
 *    whether a cap or the FP64 residual floor stopped it).  Calls that act on the current
 *    context (levels, workspace) return EXCMG_ENOCTX when there is none.
 *
 * Levels: a cascade of n_levels grids with N_l = N_0 * 2^l cells, l = 0 .. n_levels-1, where
 * N_0 = n_finest / 2^(n_levels-1) >= 2 (n_finest must be divisible by 2^(n_levels-1)),
 * n_levels >= 3.  Levels 0 and 1 are solved directly (DSOLVE); level l >= 2 is the paper's
 * i = l-1 of L = n_levels-2 and stops at the relative-residual tolerance
 * eps_i = tol * 10^(i-L).  Coarse-level data are the finest arrays sampled at every
 * 2^(n_levels-1-l)-th node.
 */
#ifndef EXCMG_H
#define EXCMG_H

#ifdef __cplusplus
extern "C" {
#endif

#define EXCMG_OK 0
#define EXCMG_EINVAL (-1)     /* bad size, level count, bc kind, NULL pointer              */
#define EXCMG_ENOMEM (-2)     /* device allocation failed                                 */
#define EXCMG_ENOCONV (-3)    /* iteration cap reached before the tolerance               */
#define EXCMG_EBREAKDOWN (-4) /* Bi-CG denominator zero or non-finite (Algorithm 2)        */
#define EXCMG_EHIP (-5)       /* a HIP runtime call failed                                */
#define EXCMG_ENOCTX (-6)     /* the call needs a context (excmg_setup / a solve) and none */
                              /* exists                                                    */

/* Precision of the Bi-CG vectors and stencil storage. */
#define EXCMG_FP64 0          /* everything in FP64                                        */
#define EXCMG_MIXED 1         /* FP32 Bi-CG inside an FP64 iterative-refinement loop       */

/* How the mixed path refines (excmg_opts.refine). */
#define EXCMG_RELIABLE 0      /* one FP32 Bi-CG run per level; whenever its recurrence       */
                              /* residual has dropped by inner_tol, the FP64 residual         */
                              /* b - A u replaces it and the run goes on with the same        */
                              /* search directions (residual replacement)                     */
#define EXCMG_RESTART 1       /* classic refinement: each step solves A e = r from e = 0 to  */
                              /* the relative tolerance inner_tol, then u += e               */

/* Level solver. */
#define EXCMG_BICG 0          /* Algorithm 2 as printed: both A p and A^T p* every iteration */
#define EXCMG_CG 1            /* its symmetric specialisation: A_h = A_h^T and r*_0 = r_0 make */
                              /* the shadow vectors equal to the primal ones, so one product  */
                              /* and half the vector traffic give bit-identical iterates      */

/* Preconditioner M of Algorithm 2 in solves (excmg_opts.precond). */
#define EXCMG_PRECOND_NONE 0   /* M = I                                                      */
#define EXCMG_PRECOND_JACOBI 1 /* M = diag(A_h) (FP64 Bi-CG only)                            */

#define EXCMG_MAX_LEVELS 16

/* Options of excmg_solve_ex.  Zero-initialise and set what you need. */
typedef struct excmg_opts {
    int n_finest;       /* cells per axis on the finest grid                               */
    int n_levels;       /* number of grids, >= 3                                            */
    int bc_kind;        /* 1 or 2                                                           */
    int precision;      /* EXCMG_FP64 or EXCMG_MIXED                                        */
    double tol;         /* relative-residual tolerance eps of the finest level (> 0)       */
    int max_iters;      /* Bi-CG iterations per run (0: 100000)                             */
    int max_runs;       /* Bi-CG runs per level in Algorithm 1's while loop (0: 5)          */
    double inner_tol;   /* mixed precision: residual reduction per refinement step        */
                        /* (0: 0.1 with EXCMG_RELIABLE, 1e-4 with EXCMG_RESTART, 1e-5 with  */
                        /* EXCMG_RESTART in excmg_solve_batch)                              */
    int max_outer;      /* mixed precision: refinement steps per level (0: 60)             */
    int batch_mode;     /* excmg_solve_batch: 0 = four graph-captured phase launches per    */
                        /* Bi-CG step, 1 = one persistent work-queue launch per step        */
    int method;         /* EXCMG_BICG (default) or EXCMG_CG (excmg_solve_ex only)           */
    int refine;         /* mixed precision: EXCMG_RELIABLE (default) or EXCMG_RESTART      */
    int precond;        /* EXCMG_PRECOND_NONE (default) or EXCMG_PRECOND_JACOBI (solve_ex) */
    int fp32_min_unknowns; /* mixed precision: levels with fewer unknowns run FP64 Bi-CG    */
                        /* (launch-latency bound, so FP32 vectors gain nothing there);       */
                        /* 0: 262144 (2^18) with EXCMG_RELIABLE and in excmg_solve_batch,    */
                        /* every level FP32 with EXCMG_RESTART; 1: FP32 on every level      */
    int row_pad;        /* mixed precision, 3D: 1 stores the rows of the FP32 Bi-CG vectors */
                        /* (and of the FP64 iterate and right-hand side they are solved     */
                        /* with) on a 128-byte multiple plus 128 bytes, so no cache line is */
                        /* split between two stencil tiles; the level's b and u are copied  */
                        /* in and out.  2: the same on the levels that take the recomputing */
                        /* form (recompute_min_unknowns), whose two sweeps then process two */
                        /* adjacent points per lane (8-byte accesses, 128-wide tiles).      */
                        /* 0 (default): contiguous rows.  Same results bit for bit; in the  */
                        /* 512^3 solve 1 and 2 are 2-4% slower than 0 on MI355X             */
    int recompute_min_unknowns; /* 3D Bi-CG (FP64 and mixed): levels with at least this many */
                        /* unknowns form q = A p and q* = A^T p* again in the update sweep   */
                        /* instead of storing them, and update x once per two iterations    */
                        /* (mixed 58 instead of 72 bytes per unknown and iteration, FP64    */
                        /* 106 instead of 136; a second stencil pass); 0: 2^22 with FP32    */
                        /* vectors, 2^20 with FP64 ones; 1: every level.  Same results bit  */
                        /* for bit                                                          */
} excmg_opts;

/* Why a Bi-CG level stopped (excmg_level_stats.exit).  Algorithm 1 repeats Bi-CG on a level
 * until the true relative residual meets the level's tolerance; in FP64 arithmetic that
 * residual cannot fall below a floor of about 22 u ||x||_2 / ||b||_2 (u = 2^-53, x the
 * level's solution), so a tolerance near the floor ends in stagnation rather than
 * convergence. */
#define EXCMG_EXIT_TOL 0       /* the true relative residual met the tolerance               */
#define EXCMG_EXIT_CAP 1       /* iteration, run or refinement-step cap reached               */
#define EXCMG_EXIT_FLOOR 2     /* floor-limited: the tolerance is below 10 x the estimated    */
                               /* floor and a further run or residual replacement no longer   */
                               /* halved the squared residual (status EXCMG_ENOCONV)          */
#define EXCMG_EXIT_BREAKDOWN 3 /* Bi-CG breakdown (status EXCMG_EBREAKDOWN)                  */

/* Per-level record filled by excmg_solve_ex (levels 0 and 1 report iterations = 0). */
typedef struct excmg_level_stats {
    int n;              /* cells per axis                                                    */
    int iterations;     /* Bi-CG iterations (all runs; FP32 inner iterations when mixed)     */
    int runs;           /* Bi-CG runs (FP64) or refinement steps (mixed: FP64 residual     */
                        /* replacements, or restarted FP32 solves)                           */
    int status;         /* EXCMG_OK / EXCMG_ENOCONV / EXCMG_EBREAKDOWN                        */
    double eps;         /* tolerance of the level                                             */
    double rel_residual;/* final true ||b - A x||_2 / ||b||_2                                 */
    double ms;          /* wall time of the level (device events)                            */
    double floor;       /* estimated FP64 relative-residual floor, 22 u ||x||_2 / ||b||_2 of  */
                        /* the returned iterate (0 on the direct levels)                     */
    int exit;           /* EXCMG_EXIT_TOL / _CAP / _FLOOR / _BREAKDOWN                       */
} excmg_level_stats;

typedef struct excmg_stats {
    int n_levels;
    excmg_level_stats level[EXCMG_MAX_LEVELS];
    double total_ms;    /* whole solve, from entry to outputs written (device events)        */
} excmg_stats;

/* Use `stream` (a hipStream_t) for all later work; NULL selects the null stream. */
int excmg_set_stream(void *stream);

/* Build (or rebuild) the context for a cascade: level sizes, device workspace and the
 * Cholesky factors of the two direct levels.  excmg_solve calls it implicitly. */
int excmg_setup(int n_finest, int n_levels, int bc_kind);

/* y = A_l x, or A_l^T x when transpose != 0, on level `level` (0 = coarsest) of the current
 * context: the left-hand side of eq. (method1) with the fictitious points of eqs.
 * (reflection2)/(reflection4) eliminated for zero boundary data (Sec. 2, eq. sec).  x and y
 * are interior vectors of (N_l - 1)^3 values.  A_l is exactly symmetric, so both products
 * use the same kernel.  The coefficients are the paper's integers (A u = h^4 f). */
int excmg_apply_stencil(int level, int transpose, const double *x, double *y);

/* The same operator on a grid of n cells per axis (n >= 2) without a context: y = A_h x (or
 * A_h^T x) for interior vectors of (n-1)^3 values and boundary kind bc_kind. */
int excmg_apply_operator(int n, int bc_kind, int transpose, const double *x, double *y);

/* b = f_h of eq. (sec) on level `level`: h^4 f minus the known boundary terms that the
 * 25-point scheme and the reflection formulas bring in (Sec. 2).  f, g1, g2 are FINEST-grid
 * node arrays of the current context (sampled by injection); b is an interior vector. */
int excmg_rhs(int level, const double *f, const double *g1, const double *g2, double *b);

/* x = A_l^{-1} b by the cached dense Cholesky factor; level must be 0 or 1 (DSOLVE,
 * Algorithm 1). */
int excmg_dsolve(int level, const double *b, double *x);

/* One run of Algorithm 2 with its options (Sec. 5, Bi-CG with the preconditioner), FP64, on
 * level `level` from the initial guess in x (overwritten by the final iterate):
 *   mdiag  the diagonal of a preconditioner M (interior vector, entries > 0; NULL: M = I;
 *          excmg_diagonal gives diag(A_h), the Jacobi choice);
 *   bstar, xstar  the shadow system: r*_0 = b* - A^T x*_0, and xstar (in: x*_0, out: the
 *          dual iterate x*_k = x*_0 + sum alpha_j p*_j, which approximates the solution of
 *          A^T x* = b*); or
 *   shadow the shadow residual r*_0 itself (no dual iterate); with neither, r*_0 = r_0.
 * Stops when the recurrence residual satisfies ||r||_2 <= eps ||b||_2 or after max_iters
 * iterations.  Outputs (may be NULL): iterations done, final recurrence ||r||_2^2.  Errors:
 * EXCMG_EINVAL (bstar without xstar or the reverse, shadow together with bstar),
 * EXCMG_ENOCONV, EXCMG_EBREAKDOWN (r*.M^-1 r or p*.A p zero or not finite). */
int excmg_bicg_ex(int level, const double *b, double *x, const double *shadow,
                  const double *bstar, double *xstar, const double *mdiag, double eps,
                  int max_iters, int *iters, double *rr);

/* diag(A_h) of level `level` of the current context (interior vector): 42 + m for the first
 * boundary kind, 42 - m for the second, m = number of faces the unknown is next to. */
int excmg_diagonal(int level, double *d);

/* One Bi-CG run (Algorithm 2, preconditioner M = I, shadow residual r*_0 = r_0) on level
 * `level` from the initial guess in x (overwritten by the final iterate): stops when the
 * recurrence residual satisfies ||r||_2 <= eps ||b||_2 or after max_iters iterations.
 * Outputs (may be NULL): iterations done and the final recurrence ||r||_2^2. */
int excmg_bicg(int level, const double *b, double *x, double eps, int max_iters, int *iters,
               double *rr);

/* Algorithm 1's while loop on one level: Bi-CG runs from x until the TRUE relative residual
 * ||b - A x||_2 / ||b||_2 <= eps (at most max_runs runs of max_iters iterations).  st may be
 * NULL. */
int excmg_level_solve(int level, const double *b, double *x, double eps, int max_iters,
                      int max_runs, excmg_level_stats *st);

/* ------------------------------------------------------------------------------------
 * The 2D equation, eq. (bvp2d), through the same pipeline.  The paper writes the equation
 * and names the 13-point scheme; the scheme here is the square of the 5-point Laplacian
 * (20 u - 8 * axis neighbours + neighbours at distance 2 + 2 * diagonal neighbours), the
 * fictitious points come from eqs. (reflection2) / (reflection4) along edge normals, and
 * EXP_finite / EXP_true are the bi-quadratic and planar forms of Sec. 4.2.  Node arrays are
 * (N+1)^2 (x fastest), interior vectors (N-1)^2; boundary data as in 3D (g2 on edges).
 * excmg2d_setup makes the current context two-dimensional: excmg_apply_stencil, excmg_rhs,
 * excmg_dsolve, excmg_bicg, excmg_bicg_ex, excmg_level_solve, excmg_diagonal and
 * excmg_get_level_solution then act on its levels.  n_finest <= 16384; the coarsest grid
 * may have up to 32 cells.
 * ------------------------------------------------------------------------------------ */
int excmg2d_setup(int n_finest, int n_levels, int bc_kind);
/* Algorithm 1 in 2D; options, outputs and return codes as excmg_solve_ex. */
int excmg2d_solve_ex(const excmg_opts *opts, const double *f, const double *g1, const double *g2,
                     double *u_out, double *ut_out, excmg_stats *stats);
/* w = EXP_finite(u1, u0) on the plane of n cells (n a multiple of 4). */
int excmg2d_exp_finite(int n, const double *u1, const double *u0, double *w);
/* ut = EXP_true(uh, u2h) on the plane of n cells (n even). */
int excmg2d_exp_true(int n, const double *uh, const double *u2h, double *ut);

/* Copy the finite-difference solution of level `level` from the last excmg_solve /
 * excmg_solve_ex on the current context (node array of N_l cells, boundary = g1): the
 * per-level solutions of Algorithm 1, e.g. to form ||w_h - u_h|| as in the paper's tables. */
int excmg_get_level_solution(int level, double *u);

/* w = EXP_finite(u1, u0) (Sec. 4.2.3, Steps 1-5): third-order approximation on the grid of n
 * cells (n divisible by 4) of the finite-difference solution, from the node arrays u1 (n/2
 * cells) and u0 (n/4 cells).  w is a node array of n cells.  Needs no context. */
int excmg_exp_finite(int n, const double *u1, const double *u0, double *w);

/* EXP_finite for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same operation and the same
 * results as excmg_exp_finite, with its intermediate grid in a fixed device array of the
 * library instead of an allocation.  That array holds (256/2 + 1)^3 doubles (17.2 MB), one
 * per GPU, allocated when the library is loaded and held until the process ends; so
 * n <= 256 (a multiple of 4).  u1, u0 and w must be device arrays (nothing is staged).
 * The work is queued on the library stream and the call returns without waiting for it
 * (results are complete when that stream reaches this point).  Every call on a GPU shares
 * its array: calls that overlap on one GPU (other streams or host threads) race.  Errors:
 * EXCMG_EINVAL (n out of range, NULL or host arrays), EXCMG_EHIP. */
int excmg_exp_finite_noalloc(int n, const double *u1, const double *u0, double *w);

/* ut = EXP_true(uh, u2h) (Sec. 4.2.1, eqs. t1 and chenlin): higher-order approximation of the
 * true solution on the grid of n cells (n even) from the node arrays uh (n cells) and u2h
 * (n/2 cells).  Needs no context. */
int excmg_exp_true(int n, const double *uh, const double *u2h, double *ut);

/* Algorithm 1 in FP64: solve and write the finest finite-difference solution u_out (node
 * array, boundary = g1).  f, g1, g2 are finest-grid node arrays; tol is eps of Algorithm 1. */
int excmg_solve(int n_finest, int n_levels, int bc_kind, const double *f, const double *g1,
                const double *g2, double tol, double *u_out);

/* Algorithm 1 with options: opts->precision selects plain FP64 or FP32 Bi-CG inside FP64
 * iterative refinement (residual, update, extrapolations and Bi-CG scalars stay FP64).
 * ut_out (may be NULL) receives EXP_true(u_h, u_2h); st (may be NULL) per-level records. */
int excmg_solve_ex(const excmg_opts *opts, const double *f, const double *g1, const double *g2,
                   double *u_out, double *ut_out, excmg_stats *st);

/* Measurement helper: launch one of the solver's sweeps `reps` times on the finest level of
 * the current context (between two device events on the library stream) and report the mean
 * duration of a launch and the algorithmic HBM bytes it moves (unknowns x vectors read and
 * written x element size; halos and padding not counted).  Scratch vectors only: no caller
 * array is touched, and the context's workspace contents are overwritten.
 *   which 0: y = A x                                         FP64 16 B, mixed 8 B
 *         1: r = b - A x, r.r partials (mixed: FP64 residual of the FP64 iterate, stored
 *            as FP32 r and r*)                                  FP64 24 B, mixed 24 B
 *         2: Bi-CG sweep A: p, p* update + A p, A^T p* + sigma  FP64 64 B, mixed 32 B
 *         3: Bi-CG sweep B: x, r, r* update + rho, r.r (mixed: FP64 x, FP32 rest)
 *                                                               FP64 72 B, mixed 44 B
 *         4: plain copy y = x (bandwidth reference)            FP64 16 B, mixed 8 B
 *         5: sweep A also applying the previous iteration's x += alpha p (the stored
 *            form with the deferred update)                            mixed 48 B
 *         6: sweep B without x (its partner)                              mixed 24 B
 *         7: sweep A of the recomputing form (the form solves run on 3D grids of 2^22
 *            unknowns and up): p, p* update + A p + sigma, stores p, p*
 *                                                               FP64 48 B, mixed 24 B
 *         8: its sweep B: A p, A^T p* formed again, x, r, r* update + rho, r.r
 *                                                               FP64 64 B, mixed 40 B
 *         9: the same sweep B leaving x alone (an odd iteration of the paired updates that
 *            solves run in this form)                            FP64 48 B, mixed 24 B
 *        10: the same sweep B applying the updates of two iterations to x (reads the
 *            previous direction too)                             FP64 72 B, mixed 44 B
 * (bytes per unknown).  precision selects EXCMG_FP64 or EXCMG_MIXED (sweeps 5 and 6: mixed
 * only; 5 to 10: 3D contexts only; 9 and 10: not with row_pad 2). */
int excmg_profile_sweep(int which, int precision, int reps, double *ms_per_launch,
                        double *bytes_per_launch);

/* Measurement helper: when on, every Bi-CG sweep launched by later solves is bracketed by
 * device events on the library stream and its duration is added to a per-level total
 * (sweep 0 = sweep A: direction update, A p, A^T p*, sigma; sweep 1 = sweep B: x, r, r*
 * updates, rho, r.r; sweep 2 = sweep A that also applies the previous iteration's x update,
 * in the stored form with the deferred update, its sweep B then leaving x alone; in the
 * recomputing form, whose sweeps B update x once per two iterations: sweep 3 = sweep B of
 * an odd iteration, which leaves x to the next one, sweep 4 = sweep B of an even iteration,
 * which applies both iterations' updates).  Only launches that did work are counted.
 * Turning it on resets the totals; excmg_get_timing reads them. */
int excmg_set_timing(int on);
int excmg_get_timing(int level, int sweep, double *ms_total, long long *launches);

/* Launch shape of the z-marched stencil kernels on grids of n cells: tiles of 64 x ty
 * columns marching through chunks of zc planes.  kind 0: the one-array kernels (operator,
 * residual; ty = 4, 8 or 16); kind 1 / 2: Bi-CG sweep A on FP64 / FP32 vectors (two arrays;
 * ty = 4 or 8 for FP64, 4, 8 or 16 for FP32).  ty = 0
 * restores the built-in table (the autotuner's MI355X picks per grid-size band).  Applies to later launches, including levels of the current
 * context.  The autotuner uses it; results do not depend on the shape (every output is
 * computed with the same arithmetic). */
int excmg_set_shape(int n, int kind, int ty, int zc);
int excmg_get_shape(int n, int kind, int *ty, int *zc);

/* One problem of a batch: finest-grid node arrays in the conventions above. */
typedef struct excmg_problem {
    int n_finest;
    int n_levels;
    int bc_kind;
    const double *f, *g1, *g2;
    double *u_out;          /* finest FD solution (node array)                      */
    double *ut_out;         /* EXP_true solution (node array), may be NULL            */
} excmg_problem;

/* Algorithm 1 for nprob independent problems (1..256) of possibly different grids, levels
 * and boundary kinds, advanced together: one Bi-CG iteration of all running systems is four
 * phase launches (opts.batch_mode 0) or one launch of a persistent work-queue kernel
 * (batch_mode 1), replayed in windows from captured hipGraphs, while each problem follows
 * its own cascade, tolerances and stopping decisions exactly as excmg_solve_ex would.
 * Mixed precision: levels of at least opts.fp32_min_unknowns unknowns (0: 2^18) run FP32
 * Bi-CG inside FP64 refinement; smaller levels run FP64 Bi-CG, as in an FP64 solve (systems
 * of the two kinds advance in separate launches on two streams).  opts.refine: with
 * EXCMG_RELIABLE (default) a run stops when its recurrence residual has fallen by
 * inner_tol (0: 0.1) or below half the level's target, the FP64 residual replaces r and r*
 * and the run goes on with its search directions; with EXCMG_RESTART each refinement step
 * is a fresh run to inner_tol (0: 1e-5), bit for bit as excmg_solve_ex with EXCMG_RESTART
 * and the same fp32_min_unknowns and inner_tol.  opts supplies tol,
 * precision and the iteration limits (its n_finest, n_levels and bc_kind are ignored).
 * stats, if not NULL, is an array of nprob records.  Runs on a stream of its own, ordered
 * after the library stream's earlier work.  Tile shapes of the batched sweep A: those
 * recorded by excmg_autotune_batch. */
int excmg_solve_batch(int nprob, const excmg_problem *probs, const excmg_opts *opts,
                      excmg_stats *stats);

/* Autotuner of the batched Bi-CG step (configuration of excmg_solve_batch): puts the finest
 * level of the batch's problems into running Bi-CG runs and, for tile heights of 4 and 8
 * rows and per distinct grid size, times steps of that size's systems alone (the phase
 * launches, replayed from a captured graph; `reps` graph replays of 8 steps per shape) with
 * z-chunks of 2, 4, ..., 128 planes and the whole depth.  The height with the smallest sum
 * of the sizes' best steps (one per batch: a launch has one workgroup shape) and the chunk
 * of every size are recorded for later excmg_solve_batch calls, per grid size and vector
 * precision (FP32 for the finest levels that a mixed batch runs in FP32); sizes never tuned
 * keep the single-problem table's chunk.  opts supplies precision and fp32_min_unknowns (its
 * tolerance is not used).  Outputs (may be NULL): the tile height and that sum of step
 * times in ms.  No caller array is written. */
int excmg_autotune_batch(int nprob, const excmg_problem *probs, const excmg_opts *opts, int reps,
                         int *ty, double *ms_per_step);
/* The batched sweep A's tile height and the z-chunk it takes on grids of n cells with FP32
 * (precision EXCMG_MIXED) or FP64 (EXCMG_FP64) vectors. */
int excmg_get_batch_shape(int n, int precision, int *ty, int *zc);

/* Autotuner: time the z-marched kernel of `kind` (0: one-array operator, 1: Bi-CG sweep A)
 * on a grid of n cells for every tile height and z-chunk length it supports, in FP64 or
 * FP32 (precision), `reps` launches each on scratch vectors, and record the fastest shape
 * for later launches (as excmg_set_shape; sweep A in FP32 is stored as kind 2).  On grids of
 * 2^22 unknowns and up, where Bi-CG forms q and q* again in its update sweep (which takes
 * sweep A's launch shape), kind 1 times that pair of sweeps together.  Outputs (may be
 * NULL): the chosen shape and its mean ms per launch (per pair of launches for the pair). */
int excmg_autotune(int n, int kind, int precision, int reps, int *ty, int *zc, double *ms);

/* Description of the last error (empty string if none). */
const char *excmg_last_error(void);

/* Free the context and all device workspace. */
void excmg_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* EXCMG_H */
