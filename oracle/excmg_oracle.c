/*
 * Plain FP64 CPU oracle of the EXCMG solver for the 3D biharmonic equation
 * (Pan, He & Ni, "An efficient multigrid solver for 3D biharmonic equation with a
 * discretization by 25-point difference scheme", arXiv:1901.05118).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, literal reference that the HIP
 * library is checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code with the GPU path.
 *
 * Every routine follows the paper's text directly:
 *   - the discrete operator is eq. (method1) evaluated on a padded node array whose
 *     fictitious points are filled by the reflection formulas eqs. (reflection2) and
 *     (reflection4) of Sec. 2 (no closed-form diagonal is used anywhere here);
 *   - known boundary values are moved to the right-hand side as Sec. 2 (eq. sec) says;
 *   - DSOLVE is a dense Cholesky factorisation (the paper does not name the direct solver);
 *   - Bi-CG is Algorithm 2 of Sec. 5 with M = I, the transpose product taken literally;
 *   - EXP_finite is Steps 1-5 of Sec. 4.2.3 per 5x5x5 interpolation cell;
 *   - EXP_true applies eqs. (t1) and (chenlin) of Sec. 4.2.1 per fine node class.
 *
 * Conventions shared (by specification, not by code) with the GPU library:
 *   - floating-point contraction is off (compile with -ffp-contract=off);
 *   - the 25-point sum is evaluated left to right in the order eq. (method1) prints it;
 *   - inner products are the compensated Dot2 algorithm of Ogita, Rump and Oishi
 *     (SIAM J. Sci. Comput. 26(6), 2005), so both sides obtain the dot product of the
 *     exact products rounded once, up to rare ties.
 *
 * Array layouts (all FP64, x index fastest):
 *   node array   : (N+1)^3 values, node (i,j,k) at (k*(N+1)+j)*(N+1)+i, i,j,k = 0..N
 *   interior vec : (N-1)^3 values, node (i,j,k) at ((k-1)*(N-1)+(j-1))*(N-1)+(i-1)
 *   padded array : (N+3)^3 values covering nodes -1..N+1 on each axis
 *
 * Boundary data: g1 = u on the boundary; g2 = outward normal derivative du/dn (first
 * kind, eq. BC) or the second normal derivative d2u/dn2 (second kind, eq. BC2).
 *
 * Return codes: 0 ok, -1 invalid argument, -2 out of memory, -3 not converged,
 * -4 Bi-CG breakdown (a zero or non-finite denominator in Algorithm 2).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOCONV (-3)
#define ORC_EBREAKDOWN (-4)

typedef long long i64;

/* ---------------------------------------------------------------- indexing */

static inline i64 nidx(int N, int i, int j, int k) {
    i64 M = (i64)N + 1;
    return ((i64)k * M + j) * M + i;
}
static inline i64 vidx(int N, int i, int j, int k) {
    i64 n = (i64)N - 1;
    return ((i64)(k - 1) * n + (j - 1)) * n + (i - 1);
}
static inline i64 pidx(int N, int i, int j, int k) {
    i64 Q = (i64)N + 3;
    return ((i64)(k + 1) * Q + (j + 1)) * Q + (i + 1);
}

/* ------------------------------------------------------------- Dot2 (ORO 2005) */

static inline void two_sum(double a, double b, double *s, double *e) {
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/* Compensated inner product: the sum of x_i*y_i computed as if in twice the working
 * precision and rounded once at the end. */
double oracle_dot(i64 n, const double *x, const double *y) {
    double s = 0.0, c = 0.0;
    for (i64 i = 0; i < n; i++) {
        double p = x[i] * y[i];
        double pe = fma(x[i], y[i], -p); /* exact low part of the product */
        double t, e;
        two_sum(s, p, &t, &e);
        s = t;
        c = c + (pe + e);
    }
    return s + c;
}

/* --------------------------------------------------------------- eq. method1 */

/* Left-hand side of eq. (method1) at the padded position c.  s1 and s2 are the padded
 * strides in y and z.  Sums run left to right in the printed order; the twelve terms of the
 * factor 2 are printed as three groups of four (the diagonals in plane k, the axis
 * neighbours in plane k-1, those in plane k+1): each group is summed first, then the three
 * group sums. */
static inline double eval25(const double *P, i64 c, i64 s1, i64 s2) {
    double S1 = P[c - 1] + P[c + 1] + P[c - s1] + P[c + s1] + P[c - s2] + P[c + s2];
    double S2 = P[c - 2] + P[c + 2] + P[c - 2 * s1] + P[c + 2 * s1] + P[c - 2 * s2] +
                P[c + 2 * s2];
    double Dk = P[c - 1 - s1] + P[c - 1 + s1] + P[c + 1 - s1] + P[c + 1 + s1];
    double Dm = P[c - 1 - s2] + P[c + 1 - s2] + P[c - s1 - s2] + P[c + s1 - s2];
    double Dp = P[c - 1 + s2] + P[c + 1 + s2] + P[c - s1 + s2] + P[c + s1 + s2];
    double S3 = Dk + Dm + Dp;
    return 42.0 * P[c] - 12.0 * S1 + S2 + 2.0 * S3;
}

/* Evaluate eq. (method1) at every interior node of a caller-filled padded array. */
int oracle_stencil_padded(int N, const double *P, double *out) {
    if (N < 2 || !P || !out) return ORC_EINVAL;
    i64 Q = (i64)N + 3, s1 = Q, s2 = Q * Q;
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= N - 1; k++)
        for (int j = 1; j <= N - 1; j++)
            for (int i = 1; i <= N - 1; i++)
                out[vidx(N, i, j, k)] = eval25(P, pidx(N, i, j, k), s1, s2);
    return ORC_OK;
}

/* ------------------------------------------------------ fictitious points (Sec. 2) */

/* Value at a fictitious point one step outside a face.
 *   mirror : u at the interior node one step inside the face (index 1 or N-1)
 *   u0     : u at the boundary node on the face (index 0 or N)
 *   g2     : the second boundary datum at that boundary node
 *   low    : 1 for the face at coordinate 0, 0 for the face at coordinate 1
 * First kind, eq. (reflection2): u_{-1} = u_1 - 2h (du/dx)_0, where du/dx = -du/dn on the
 * low face and +du/dn on the high face (mirrored: u_{N+1} = u_{N-1} + 2h (du/dx)_N).
 * Second kind, eq. (reflection4): u_{-1} = -u_1 + 2 u_0 + h^2 (d2u/dx2)_0, the same on
 * both faces since the second normal derivative does not depend on the orientation. */
static inline double ghost_value(int bc, double h, double mirror, double u0, double g2, int low) {
    if (bc == 1) {
        double dudx = low ? -g2 : g2;
        return low ? mirror - 2.0 * h * dudx : mirror + 2.0 * h * dudx;
    }
    return -mirror + 2.0 * u0 + h * h * g2;
}

/* Fill the fictitious layer of a padded array whose nodes 0..N are already set.  g2 is a
 * node array (N+1)^3 read on face-interior nodes only, or NULL for zero data.  Only the
 * fictitious points referenced by eq. (method1) at interior nodes are needed: those whose
 * other two coordinates are interior. */
static void fill_ghosts(int N, int bc, double *P, const double *g2) {
    double h = 1.0 / (double)N;
    for (int b = 1; b <= N - 1; b++)
        for (int a = 1; a <= N - 1; a++) {
            /* x faces: (i, j, k) = (-1 | N+1, a, b) */
            P[pidx(N, -1, a, b)] = ghost_value(bc, h, P[pidx(N, 1, a, b)], P[pidx(N, 0, a, b)],
                                               g2 ? g2[nidx(N, 0, a, b)] : 0.0, 1);
            P[pidx(N, N + 1, a, b)] =
                ghost_value(bc, h, P[pidx(N, N - 1, a, b)], P[pidx(N, N, a, b)],
                            g2 ? g2[nidx(N, N, a, b)] : 0.0, 0);
            /* y faces */
            P[pidx(N, a, -1, b)] = ghost_value(bc, h, P[pidx(N, a, 1, b)], P[pidx(N, a, 0, b)],
                                               g2 ? g2[nidx(N, a, 0, b)] : 0.0, 1);
            P[pidx(N, a, N + 1, b)] =
                ghost_value(bc, h, P[pidx(N, a, N - 1, b)], P[pidx(N, a, N, b)],
                            g2 ? g2[nidx(N, a, N, b)] : 0.0, 0);
            /* z faces */
            P[pidx(N, a, b, -1)] = ghost_value(bc, h, P[pidx(N, a, b, 1)], P[pidx(N, a, b, 0)],
                                               g2 ? g2[nidx(N, a, b, 0)] : 0.0, 1);
            P[pidx(N, a, b, N + 1)] =
                ghost_value(bc, h, P[pidx(N, a, b, N - 1)], P[pidx(N, a, b, N)],
                            g2 ? g2[nidx(N, a, b, N)] : 0.0, 0);
        }
}

static double *padded_alloc(int N) {
    i64 Q = (i64)N + 3;
    return (double *)calloc((size_t)(Q * Q * Q), sizeof(double));
}

/* Padded array of the homogeneous problem: interior = x, boundary = 0, fictitious points
 * from the reflection formulas with zero boundary data. */
static void fill_homogeneous(int N, int bc, const double *x, double *P) {
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= N - 1; k++)
        for (int j = 1; j <= N - 1; j++)
            for (int i = 1; i <= N - 1; i++) P[pidx(N, i, j, k)] = x[vidx(N, i, j, k)];
    fill_ghosts(N, bc, P, NULL);
}

/* ------------------------------------------------------------ operator A_h (eq. sec) */

/* y = A_h x: the unknown-dependent part of eq. (method1) after the fictitious points are
 * eliminated, i.e. method1 evaluated on the homogeneous padded array. */
int oracle_apply(int N, int bc, const double *x, double *y) {
    if (N < 2 || (bc != 1 && bc != 2) || !x || !y) return ORC_EINVAL;
    double *P = padded_alloc(N);
    if (!P) return ORC_ENOMEM;
    fill_homogeneous(N, bc, x, P);
    oracle_stencil_padded(N, P, y);
    free(P);
    return ORC_OK;
}

/* y = A_h^T x taken literally: every row of A_h scatters its coefficients to the columns
 * it touches.  A term that lands on a fictitious point belongs, through the reflection
 * formula, to the mirrored interior node with factor +1 (first kind) or -1 (second kind);
 * a term that lands on a boundary node is known data and is not part of A_h.
 * The 25 terms are scattered one after another, each in two passes: the terms that land on
 * an interior node, then those that land on a fictitious point.  Within one pass distinct
 * rows reach distinct columns, so a pass runs in parallel without races and the
 * accumulation order (term by term, pass by pass) does not depend on the thread count. */
int oracle_apply_transpose(int N, int bc, const double *x, double *y) {
    if (N < 2 || (bc != 1 && bc != 2) || !x || !y) return ORC_EINVAL;
    static const int off[25][3] = {
        {0, 0, 0},
        {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1},
        {-2, 0, 0}, {2, 0, 0}, {0, -2, 0}, {0, 2, 0}, {0, 0, -2}, {0, 0, 2},
        {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}, {1, 1, 0},
        {-1, 0, -1}, {1, 0, -1}, {0, -1, -1}, {0, 1, -1},
        {-1, 0, 1}, {1, 0, 1}, {0, -1, 1}, {0, 1, 1}};
    static const double coef[25] = {42.0,  -12.0, -12.0, -12.0, -12.0, -12.0, -12.0,
                                    1.0,   1.0,   1.0,   1.0,   1.0,   1.0,
                                    2.0,   2.0,   2.0,   2.0,   2.0,   2.0,
                                    2.0,   2.0,   2.0,   2.0,   2.0,   2.0};
    double sgn = (bc == 1) ? 1.0 : -1.0;
    i64 nu = (i64)(N - 1) * (N - 1) * (N - 1);
    for (i64 t = 0; t < nu; t++) y[t] = 0.0;
    for (int t = 0; t < 25; t++)
        for (int pass = 0; pass < 2; pass++) {
#pragma omp parallel for schedule(static)
        for (int k = 1; k <= N - 1; k++)
            for (int j = 1; j <= N - 1; j++)
                for (int i = 1; i <= N - 1; i++) {
                    int p[3] = {i + off[t][0], j + off[t][1], k + off[t][2]};
                    int ghost = 0, bnd = 0;
                    for (int a = 0; a < 3; a++) {
                        if (p[a] == 0 || p[a] == N) bnd = 1;
                        if (p[a] == -1) { p[a] = 1; ghost = 1; }
                        if (p[a] == N + 1) { p[a] = N - 1; ghost = 1; }
                    }
                    if (bnd || ghost != pass) continue;
                    double c = coef[t] * x[vidx(N, i, j, k)];
                    if (ghost) c = sgn * c;
                    y[vidx(N, p[0], p[1], p[2])] += c;
                }
    }
    return ORC_OK;
}

/* r = b - A_h x */
int oracle_residual(int N, int bc, const double *b, const double *x, double *r) {
    int rc = oracle_apply(N, bc, x, r);
    if (rc) return rc;
    i64 nu = (i64)(N - 1) * (N - 1) * (N - 1);
    for (i64 t = 0; t < nu; t++) r[t] = b[t] - r[t];
    return ORC_OK;
}

/* ------------------------------------------------------- right-hand side f_h (eq. sec) */

/* b = h^4 f - (method1 evaluated on the known values only): interior unknowns set to 0,
 * boundary nodes = g1, fictitious points from the reflection formulas with the mirrored
 * unknown set to 0 and the boundary data g1, g2.  f, g1, g2 are node arrays (N+1)^3 of the
 * level: f is read on interior nodes, g1 on all boundary nodes, g2 on face-interior nodes. */
int oracle_rhs(int N, int bc, const double *f, const double *g1, const double *g2, double *b) {
    if (N < 2 || (bc != 1 && bc != 2) || !f || !g1 || !g2 || !b) return ORC_EINVAL;
    double *P = padded_alloc(N);
    if (!P) return ORC_ENOMEM;
    for (int k = 0; k <= N; k++)
        for (int j = 0; j <= N; j++)
            for (int i = 0; i <= N; i++) {
                int on_bnd = (i == 0 || i == N || j == 0 || j == N || k == 0 || k == N);
                P[pidx(N, i, j, k)] = on_bnd ? g1[nidx(N, i, j, k)] : 0.0;
            }
    fill_ghosts(N, bc, P, g2);
    double h = 1.0 / (double)N;
    double h4 = h * h * h * h;
    i64 Q = (i64)N + 3;
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= N - 1; k++)
        for (int j = 1; j <= N - 1; j++)
            for (int i = 1; i <= N - 1; i++)
                b[vidx(N, i, j, k)] =
                    h4 * f[nidx(N, i, j, k)] - eval25(P, pidx(N, i, j, k), Q, Q * Q);
    free(P);
    return ORC_OK;
}

/* ------------------------------------------------------------- DSOLVE (Alg. 1) */

/* Direct solve of A_h x = b by dense Cholesky.  A_h is assembled column by column by
 * applying the operator to unit vectors.  Returns -4 if a pivot is not positive (A_h
 * would then not be symmetric positive definite). */
int oracle_dsolve(int N, int bc, const double *b, double *x) {
    if (N < 2 || (bc != 1 && bc != 2) || !b || !x) return ORC_EINVAL;
    i64 n = (i64)(N - 1) * (N - 1) * (N - 1);
    double *A = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *e = (double *)calloc((size_t)n, sizeof(double));
    double *col = (double *)malloc((size_t)n * sizeof(double));
    double *yv = (double *)malloc((size_t)n * sizeof(double));
    if (!A || !e || !col || !yv) {
        free(A); free(e); free(col); free(yv);
        return ORC_ENOMEM;
    }
    for (i64 c = 0; c < n; c++) {
        e[c] = 1.0;
        oracle_apply(N, bc, e, col);
        e[c] = 0.0;
        for (i64 r = 0; r < n; r++) A[r * n + c] = col[r];
    }
    /* A = L L^T, L stored in the lower triangle of A (row-major). */
    int rc = ORC_OK;
    for (i64 jj = 0; jj < n && rc == ORC_OK; jj++) {
        double s = A[jj * n + jj];
        for (i64 k = 0; k < jj; k++) s -= A[jj * n + k] * A[jj * n + k];
        if (!(s > 0.0)) { rc = ORC_EBREAKDOWN; break; }
        double d = sqrt(s);
        A[jj * n + jj] = d;
#pragma omp parallel for schedule(static)
        for (i64 i = jj + 1; i < n; i++) {
            double t = A[i * n + jj];
            for (i64 k = 0; k < jj; k++) t -= A[i * n + k] * A[jj * n + k];
            A[i * n + jj] = t / d;
        }
    }
    if (rc == ORC_OK) {
        for (i64 i = 0; i < n; i++) { /* L y = b */
            double t = b[i];
            for (i64 k = 0; k < i; k++) t -= A[i * n + k] * yv[k];
            yv[i] = t / A[i * n + i];
        }
        for (i64 i = n - 1; i >= 0; i--) { /* L^T x = y */
            double t = yv[i];
            for (i64 k = i + 1; k < n; k++) t -= A[k * n + i] * x[k];
            x[i] = t / A[i * n + i];
        }
    }
    free(A); free(e); free(col); free(yv);
    return rc;
}

/* Dense A_h (row-major n x n), assembled from unit vectors; for tests on small grids. */
int oracle_assemble(int N, int bc, double *A) {
    if (N < 2 || (bc != 1 && bc != 2) || !A) return ORC_EINVAL;
    i64 n = (i64)(N - 1) * (N - 1) * (N - 1);
    double *e = (double *)calloc((size_t)n, sizeof(double));
    double *col = (double *)malloc((size_t)n * sizeof(double));
    if (!e || !col) { free(e); free(col); return ORC_ENOMEM; }
    for (i64 c = 0; c < n; c++) {
        e[c] = 1.0;
        oracle_apply(N, bc, e, col);
        e[c] = 0.0;
        for (i64 r = 0; r < n; r++) A[r * n + c] = col[r];
    }
    free(e); free(col);
    return ORC_OK;
}

/* ------------------------------------------------------------- Bi-CG (Alg. 2) */

/* Algorithm 2 (Bi-CG with the preconditioner), real arithmetic.  M is diagonal: mdiag holds
 * its entries (NULL: M = I), so M^-1 v is v divided entrywise and v^T M^-1 = (M^-T v)^T =
 * M^-1 v as a column.  The shadow system is either
 *   - bstar and xstar given: r*_0 = b* - A^T x*_0 and the dual iterate x* is updated in place
 *     (x*_{k+1} = x*_k + alpha_k p*_k), so that on exit x* approximates the solution of
 *     A^T x* = b*; or
 *   - shadow given: r*_0 = shadow (no dual iterate); or
 *   - neither: r*_0 = r_0.
 * The products with A^T are formed by scattering the rows of A_h when literal_t, else as
 * A_h v (A_h is exactly symmetric).  The run stops when the recurrence residual satisfies
 * ||r_k||_2 <= eps ||b||_2, after maxit iterations (ENOCONV) or on a zero or non-finite
 * r*.M^-1 r or p*.A p (EBREAKDOWN). */
int oracle_bicg_ex(int N, int bc, const double *b, double *x, const double *shadow,
                   const double *bstar, double *xstar, const double *mdiag, double eps,
                   int maxit, int literal_t, int *iters, double *rr_out) {
    if (N < 2 || (bc != 1 && bc != 2) || !b || !x || maxit < 0) return ORC_EINVAL;
    if ((bstar == NULL) != (xstar == NULL)) return ORC_EINVAL;
    i64 n = (i64)(N - 1) * (N - 1) * (N - 1);
    double *r = malloc((size_t)n * sizeof(double)), *rs = malloc((size_t)n * sizeof(double));
    double *p = malloc((size_t)n * sizeof(double)), *ps = malloc((size_t)n * sizeof(double));
    double *q = malloc((size_t)n * sizeof(double)), *qs = malloc((size_t)n * sizeof(double));
    double *z = malloc((size_t)n * sizeof(double)), *zs = malloc((size_t)n * sizeof(double));
    if (!r || !rs || !p || !ps || !q || !qs || !z || !zs) {
        free(r); free(rs); free(p); free(ps); free(q); free(qs); free(z); free(zs);
        return ORC_ENOMEM;
    }
    double bb = oracle_dot(n, b, b);
    double thr = (eps * eps) * bb;
    oracle_residual(N, bc, b, x, r); /* r_0 = b - A x_0 */
    if (bstar) {                      /* r*_0 = b* - A^T x*_0 */
        if (literal_t) oracle_apply_transpose(N, bc, xstar, qs);
        else oracle_apply(N, bc, xstar, qs);
        for (i64 t = 0; t < n; t++) rs[t] = bstar[t] - qs[t];
    } else {
        for (i64 t = 0; t < n; t++) rs[t] = shadow ? shadow[t] : r[t];
    }
    /* z = M^-1 r, z* = M^-T r* */
#define PRECOND()                                                      \
    for (i64 t = 0; t < n; t++) {                                      \
        z[t] = mdiag ? r[t] / mdiag[t] : r[t];                         \
        zs[t] = mdiag ? rs[t] / mdiag[t] : rs[t];                      \
    }
    PRECOND();
    for (i64 t = 0; t < n; t++) { p[t] = z[t]; ps[t] = zs[t]; } /* p_0 = M^-1 r_0 */
    double rho = oracle_dot(n, rs, z);                             /* r*_0 M^-1 r_0 */
    double rr = oracle_dot(n, r, r);
    int k = 0, rc = ORC_OK;
    while (!(rr <= thr)) {
        if (k >= maxit) { rc = ORC_ENOCONV; break; }
        if (rho == 0.0 || !isfinite(rho)) { rc = ORC_EBREAKDOWN; break; }
        oracle_apply(N, bc, p, q);            /* A p_k */
        if (literal_t) oracle_apply_transpose(N, bc, ps, qs); /* (p*_k A)^T = A^T p*_k */
        else oracle_apply(N, bc, ps, qs);
        double sigma = oracle_dot(n, ps, q);
        if (sigma == 0.0 || !isfinite(sigma)) { rc = ORC_EBREAKDOWN; break; }
        double alpha = rho / sigma;
#pragma omp parallel for schedule(static)
        for (i64 t = 0; t < n; t++) {
            x[t] = x[t] + alpha * p[t];
            if (xstar) xstar[t] = xstar[t] + alpha * ps[t];
            r[t] = r[t] - alpha * q[t];
            rs[t] = rs[t] - alpha * qs[t];
        }
        PRECOND();
        double rho_new = oracle_dot(n, rs, z);
        rr = oracle_dot(n, r, r);
        double beta = rho_new / rho;
        rho = rho_new;
        k++;
#pragma omp parallel for schedule(static)
        for (i64 t = 0; t < n; t++) {
            p[t] = z[t] + beta * p[t];
            ps[t] = zs[t] + beta * ps[t];
        }
    }
#undef PRECOND
    if (iters) *iters = k;
    if (rr_out) *rr_out = rr;
    free(r); free(rs); free(p); free(ps); free(q); free(qs); free(z); free(zs);
    return rc;
}

/* One run of Algorithm 2 with M = I on A_h x = b, starting from x (updated in place).
 * shadow: the initial shadow residual r*_0, or NULL for r*_0 = r_0; the adjoint iterate is
 * not formed.  literal_t: 1 forms the shadow product p*_k A by the row scatter of
 * oracle_apply_transpose; 0 forms it as A_h p*_k, which is the same vector because A_h
 * equals its transpose entry for entry (the test suite checks this on assembled matrices);
 * the two differ only in rounding.  Stops when r.r <= (eps*eps)*(b.b), after maxit
 * iterations (-3) or on breakdown (-4); *iters gets the iteration count and *rr_out the
 * final recurrence r.r. */
int oracle_bicg(int N, int bc, const double *b, double *x, const double *shadow, double eps,
                int maxit, int literal_t, int *iters, double *rr_out) {
    return oracle_bicg_ex(N, bc, b, x, shadow, NULL, NULL, NULL, eps, maxit, literal_t, iters,
                          rr_out);
}

/* The diagonal of A_h (the Jacobi choice of M), read off the operator itself: A_h applied
 * to vectors that are 1 on one residue class of (i mod 5, j mod 5, k mod 5) and 0 elsewhere;
 * the 25-point stencil reaches 2 points per axis, so no two ones of a class share a row. */
int oracle_diagonal(int N, int bc, double *d) {
    if (N < 2 || (bc != 1 && bc != 2) || !d) return ORC_EINVAL;
    const int n1 = N - 1;
    i64 n = (i64)n1 * n1 * n1;
    double *e = malloc((size_t)n * sizeof(double)), *y = malloc((size_t)n * sizeof(double));
    if (!e || !y) { free(e); free(y); return ORC_ENOMEM; }
    for (int ck = 0; ck < 5; ck++)
        for (int cj = 0; cj < 5; cj++)
            for (int ci = 0; ci < 5; ci++) {
                for (int k = 0; k < n1; k++)
                    for (int j = 0; j < n1; j++)
                        for (int i = 0; i < n1; i++) {
                            const i64 t = ((i64)k * n1 + j) * n1 + i;
                            e[t] = (i % 5 == ci && j % 5 == cj && k % 5 == ck) ? 1.0 : 0.0;
                        }
                oracle_apply(N, bc, e, y);
                for (i64 t = 0; t < n; t++)
                    if (e[t] != 0.0) d[t] = y[t];
            }
    free(e); free(y);
    return ORC_OK;
}

/* Alg. 1, the while loop of a level: repeat Bi-CG from the current x until the true
 * relative residual satisfies ||b - A x||_2 <= eps ||b||_2, at most max_runs Bi-CG runs
 * of at most maxit iterations each.  Outputs: total iterations, Bi-CG runs, final true
 * r.r and b.b. */
int oracle_level_solve_ex(int N, int bc, const double *b, double *x, const double *mdiag,
                          double eps, int maxit, int max_runs, int literal_t, int *iters,
                          int *runs, double *rr_true, double *bb_out);

int oracle_level_solve(int N, int bc, const double *b, double *x, double eps, int maxit,
                       int max_runs, int literal_t, int *iters, int *runs, double *rr_true,
                       double *bb_out) {
    return oracle_level_solve_ex(N, bc, b, x, NULL, eps, maxit, max_runs, literal_t, iters,
                                 runs, rr_true, bb_out);
}

/* The same with Bi-CG preconditioned by M = diag(mdiag) (NULL: M = I). */
int oracle_level_solve_ex(int N, int bc, const double *b, double *x, const double *mdiag,
                          double eps, int maxit, int max_runs, int literal_t, int *iters,
                          int *runs, double *rr_true, double *bb_out) {
    if (N < 2 || (bc != 1 && bc != 2) || !b || !x) return ORC_EINVAL;
    i64 n = (i64)(N - 1) * (N - 1) * (N - 1);
    double *r = malloc((size_t)n * sizeof(double));
    if (!r) return ORC_ENOMEM;
    double bb = oracle_dot(n, b, b);
    double thr = (eps * eps) * bb;
    oracle_residual(N, bc, b, x, r);
    double rr = oracle_dot(n, r, r);
    int total = 0, nrun = 0, rc = ORC_OK;
    while (!(rr <= thr)) {
        if (nrun >= max_runs) { rc = ORC_ENOCONV; break; }
        int it = 0;
        double rrr = 0.0;
        int brc = oracle_bicg_ex(N, bc, b, x, NULL, NULL, NULL, mdiag, eps, maxit, literal_t,
                                 &it, &rrr);
        total += it;
        nrun++;
        double prev = rr;
        oracle_residual(N, bc, b, x, r);
        rr = oracle_dot(n, r, r);
        if (brc == ORC_EBREAKDOWN) { rc = brc; break; }
        if (brc == ORC_ENOMEM || brc == ORC_EINVAL) { rc = brc; break; }
        /* The true residual of FP64 arithmetic cannot fall below a floor of about
         * 22 u ||x||_2 / ||b||_2 (u = 2^-53): when the tolerance is within a factor 10 of that
         * floor, a run that no longer halves the squared residual ends the while loop
         * (floor-limited) instead of restarting Bi-CG until max_runs. */
        if (!(rr <= thr)) {
            double floor_est = bb > 0.0 ? 22.0 * 0x1p-53 * sqrt(oracle_dot(n, x, x) / bb) : 0.0;
            if (eps < 10.0 * floor_est && !(rr < 0.5 * prev)) { rc = ORC_ENOCONV; break; }
        }
    }
    if (iters) *iters = total;
    if (runs) *runs = nrun;
    if (rr_true) *rr_true = rr;
    if (bb_out) *bb_out = bb;
    free(r);
    return rc;
}

/* ----------------------------------------------------- EXP_finite (Sec. 4.2.2-4.2.3) */

/* Lagrange basis polynomial of degree 2, eq. (iinter), for nodes xi = 0, 1/2, 1. */
static double lagrange2(int i, double xi) {
    static const double node[3] = {0.0, 0.5, 1.0};
    double v = 1.0;
    for (int k = 0; k < 3; k++)
        if (k != i) v = v * ((xi - node[k]) / (node[i] - node[k]));
    return v;
}

/* w = EXP_finite(u1, u0): third-order approximation on grid Z2 (N cells per axis) of the
 * finite-difference solution, from the solutions u1 on Z1 (N/2 cells) and u0 on Z0 (N/4
 * cells).  All three are node arrays.  Each Z0 cell is an interpolation cell holding 27
 * nodes of Z1 and 125 nodes of Z2, numbered 1 + a + 5b + 25c (a, b, c = 0..4 in Z2 steps).
 *   Step 1, the 8 corners: eq. (secfff), w = (5 u1 - u0)/4.
 *   Step 2, the 12 edge midpoints: eq. (bfsec) along the edge.
 *   Step 3, the 6 face centres: mean of eq. (bfsec) along the two face diagonals.
 *   Step 4, the cell centre: mean of eq. (bfsec) along the four space diagonals.
 *   Step 5, the other 98 nodes: tri-quadratic interpolation, eqs. (inter)-(iinter).
 * Nodes shared by neighbouring cells receive the same value from each cell. */
int oracle_exp_finite(int N, const double *u1, const double *u0, double *w) {
    if (N < 4 || N % 4 != 0 || !u1 || !u0 || !w) return ORC_EINVAL;
    int N1 = N / 2, N0 = N / 4;
    double L[5][3]; /* L[a][i] = l_i(a/4) */
    for (int a = 0; a < 5; a++)
        for (int i = 0; i < 3; i++) L[a][i] = lagrange2(i, a / 4.0);
#pragma omp parallel for collapse(2) schedule(static)
    for (int cz = 0; cz < N0; cz++)
        for (int cy = 0; cy < N0; cy++)
            for (int cx = 0; cx < N0; cx++) {
                /* U1(al,be,ga): u1 at Z1 node (2cx+al, 2cy+be, 2cz+ga), al,be,ga = 0..2.
                 * D(al,be,ga): u1 - u0 at a corner (al,be,ga in {0,2}). */
#define U1(al, be, ga) u1[nidx(N1, 2 * cx + (al), 2 * cy + (be), 2 * cz + (ga))]
#define U0(al, be, ga) u0[nidx(N0, cx + (al) / 2, cy + (be) / 2, cz + (ga) / 2)]
/* eq. (bfsec) on the segment from corner e to corner f through the Z1 node m */
#define BFSEC(m0, m1, m2, e0, e1, e2, f0, f1, f2)                                          \
    (U1(m0, m1, m2) +                                                                      \
     (1.0 / 8.0) * (U1(e0, e1, e2) - U0(e0, e1, e2) + U1(f0, f1, f2) - U0(f0, f1, f2)))
                double V[3][3][3]; /* [ga][be][al] */
                /* Step 1: corners */
                for (int ga = 0; ga <= 2; ga += 2)
                    for (int be = 0; be <= 2; be += 2)
                        for (int al = 0; al <= 2; al += 2)
                            V[ga][be][al] = (5.0 * U1(al, be, ga) - U0(al, be, ga)) / 4.0;
                /* Step 2: edge midpoints */
                for (int s = 0; s <= 2; s += 2)
                    for (int t = 0; t <= 2; t += 2) {
                        V[t][s][1] = BFSEC(1, s, t, 0, s, t, 2, s, t); /* x edges */
                        V[t][1][s] = BFSEC(s, 1, t, s, 0, t, s, 2, t); /* y edges */
                        V[1][t][s] = BFSEC(s, t, 1, s, t, 0, s, t, 2); /* z edges */
                    }
                /* Step 3: face centres, mean over the two face diagonals */
                for (int s = 0; s <= 2; s += 2) {
                    V[s][1][1] = (BFSEC(1, 1, s, 0, 0, s, 2, 2, s) + BFSEC(1, 1, s, 2, 0, s, 0, 2, s)) / 2.0;
                    V[1][s][1] = (BFSEC(1, s, 1, 0, s, 0, 2, s, 2) + BFSEC(1, s, 1, 2, s, 0, 0, s, 2)) / 2.0;
                    V[1][1][s] = (BFSEC(s, 1, 1, s, 0, 0, s, 2, 2) + BFSEC(s, 1, 1, s, 2, 0, s, 0, 2)) / 2.0;
                }
                /* Step 4: cell centre, mean over the four space diagonals */
                V[1][1][1] = (BFSEC(1, 1, 1, 0, 0, 0, 2, 2, 2) + BFSEC(1, 1, 1, 2, 0, 0, 0, 2, 2) +
                              BFSEC(1, 1, 1, 0, 2, 0, 2, 0, 2) + BFSEC(1, 1, 1, 2, 2, 0, 0, 0, 2)) /
                             4.0;
#undef BFSEC
#undef U0
#undef U1
                /* Step 5 (and the 27 nodes themselves) */
                for (int c = 0; c < 5; c++)
                    for (int bq = 0; bq < 5; bq++)
                        for (int a = 0; a < 5; a++) {
                            double val;
                            if (a % 2 == 0 && bq % 2 == 0 && c % 2 == 0) {
                                val = V[c / 2][bq / 2][a / 2];
                            } else {
                                val = 0.0;
                                for (int ga = 0; ga < 3; ga++)
                                    for (int be = 0; be < 3; be++)
                                        for (int al = 0; al < 3; al++)
                                            val = val + L[a][al] * L[bq][be] * L[c][ga] * V[ga][be][al];
                            }
                            w[nidx(N, 4 * cx + a, 4 * cy + bq, 4 * cz + c)] = val;
                        }
            }
    return ORC_OK;
}

/* -------------------------------------------------------- EXP_true (Sec. 4.2.1) */

/* ut = EXP_true(uh, u2h): higher-order approximation of the true solution on the grid of
 * N cells from the finite-difference solutions uh (N cells) and u2h (N/2 cells), both node
 * arrays.  A fine node is a node, an edge midpoint, a face centre or the centre of a coarse
 * cell.  Coarse nodes: eq. (t1), (4 uh - u2h)/3.  Edge midpoints: eq. (chenlin) along the
 * edge.  Face and cell centres, as in Steps 3-4 of EXP_finite: the mean of eq. (chenlin)
 * along the two face diagonals or the four space diagonals. */
int oracle_exp_true(int N, const double *uh, const double *u2h, double *ut) {
    if (N < 2 || N % 2 != 0 || !uh || !u2h || !ut) return ORC_EINVAL;
    int Nc = N / 2;
#pragma omp parallel for schedule(static)
    for (int k = 0; k <= N; k++)
        for (int j = 0; j <= N; j++)
            for (int i = 0; i <= N; i++) {
                int oi = i & 1, oj = j & 1, ok = k & 1;
                double mid = uh[nidx(N, i, j, k)];
/* eq. (chenlin) at this node along the segment between fine nodes e and f (coarse nodes) */
#define CHENLIN(e0, e1, e2, f0, f1, f2)                                                     \
    (mid + (1.0 / 6.0) * (uh[nidx(N, e0, e1, e2)] - u2h[nidx(Nc, (e0) / 2, (e1) / 2, (e2) / 2)] + \
                          uh[nidx(N, f0, f1, f2)] - u2h[nidx(Nc, (f0) / 2, (f1) / 2, (f2) / 2)]))
                double v;
                int odd = oi + oj + ok;
                if (odd == 0) {
                    v = (4.0 * mid - u2h[nidx(Nc, i / 2, j / 2, k / 2)]) / 3.0;
                } else if (odd == 1) {
                    if (oi) v = CHENLIN(i - 1, j, k, i + 1, j, k);
                    else if (oj) v = CHENLIN(i, j - 1, k, i, j + 1, k);
                    else v = CHENLIN(i, j, k - 1, i, j, k + 1);
                } else if (odd == 2) {
                    if (!ok) v = (CHENLIN(i - 1, j - 1, k, i + 1, j + 1, k) +
                                  CHENLIN(i + 1, j - 1, k, i - 1, j + 1, k)) / 2.0;
                    else if (!oj) v = (CHENLIN(i - 1, j, k - 1, i + 1, j, k + 1) +
                                       CHENLIN(i + 1, j, k - 1, i - 1, j, k + 1)) / 2.0;
                    else v = (CHENLIN(i, j - 1, k - 1, i, j + 1, k + 1) +
                              CHENLIN(i, j + 1, k - 1, i, j - 1, k + 1)) / 2.0;
                } else {
                    v = (CHENLIN(i - 1, j - 1, k - 1, i + 1, j + 1, k + 1) +
                         CHENLIN(i + 1, j - 1, k - 1, i - 1, j + 1, k + 1) +
                         CHENLIN(i - 1, j + 1, k - 1, i + 1, j - 1, k + 1) +
                         CHENLIN(i + 1, j + 1, k - 1, i - 1, j - 1, k + 1)) / 4.0;
                }
#undef CHENLIN
                ut[nidx(N, i, j, k)] = v;
            }
    return ORC_OK;
}

/* OpenMP threads of the loops above (for timing runs of the oracle; results do not depend
 * on the thread count). */
int oracle_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
