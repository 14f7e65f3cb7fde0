/*
 * Plain FP64 CPU oracle of EXCMG for the 2D biharmonic equation, eq. (bvp2d), the
 * two-dimensional version of the problem the paper solves in 3D.
 *
 * TEST INFRASTRUCTURE ONLY (see excmg_oracle.c): loaded by the test suite only, shares no
 * code with the GPU path.
 *
 * The paper writes the 2D equation and names the 13-point discretization, but prints the
 * scheme, the boundary treatment and the extrapolations only in 3D.  This file takes the
 * 2D analogue of each, read off the 3D text:
 *   - the scheme is the square of the 5-point Laplacian, as eq. (method1) is the square of
 *     the 7-point one: h^4 (Delta^2 u)_ij ~ 20 u_ij - 8 (4 axis neighbours)
 *     + (4 neighbours at distance 2) + 2 (4 diagonal neighbours), summed left to right in
 *     this order within each group;
 *   - fictitious points one step outside an edge come from eqs. (reflection2) and
 *     (reflection4) along the edge normal, exactly as on a face in 3D;
 *   - EXP_finite works per 5x5 interpolation cell: corners by eq. (secfff), edge midpoints
 *     by eq. (bfsec) along the edge, the centre as the mean of eq. (bfsec) along the two
 *     diagonals, the other 16 nodes by bi-quadratic interpolation (Steps 1-4, the 2D form
 *     of Steps 1-5 of Sec. 4.2.3);
 *   - EXP_true applies eq. (t1) at coarse nodes, eq. (chenlin) at edge midpoints and the
 *     mean of eq. (chenlin) along the two diagonals at cell centres.
 *
 * Layouts (FP64, x fastest): node array (N+1)^2, node (i,j) at j*(N+1)+i; interior vector
 * (N-1)^2, node (i,j) at (j-1)*(N-1)+(i-1); padded array (N+3)^2 over nodes -1..N+1.
 * Return codes as in excmg_oracle.c.
 */
#include <math.h>
#include <stdlib.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOCONV (-3)
#define ORC_EBREAKDOWN (-4)

typedef long long i64;

double oracle_dot(i64 n, const double *x, const double *y); /* Dot2, excmg_oracle.c */

static inline i64 nidx2(int N, int i, int j) { return (i64)j * (N + 1) + i; }
static inline i64 vidx2(int N, int i, int j) { return (i64)(j - 1) * (N - 1) + (i - 1); }
static inline i64 pidx2(int N, int i, int j) { return (i64)(j + 1) * (N + 3) + (i + 1); }

/* the 13-point scheme at padded position c (row stride s) */
static inline double eval13(const double *P, i64 c, i64 s) {
    double S1 = P[c - 1] + P[c + 1] + P[c - s] + P[c + s];
    double S2 = P[c - 2] + P[c + 2] + P[c - 2 * s] + P[c + 2 * s];
    double S3 = P[c - 1 - s] + P[c - 1 + s] + P[c + 1 - s] + P[c + 1 + s];
    return 20.0 * P[c] - 8.0 * S1 + S2 + 2.0 * S3;
}

/* Fictitious point one step outside an edge (see ghost_value in excmg_oracle.c). */
static inline double ghost2(int bc, double h, double mirror, double u0, double g2, int low) {
    if (bc == 1) {
        double dudx = low ? -g2 : g2;
        return low ? mirror - 2.0 * h * dudx : mirror + 2.0 * h * dudx;
    }
    return -mirror + 2.0 * u0 + h * h * g2;
}

static void fill_ghosts2(int N, int bc, double *P, const double *g2) {
    double h = 1.0 / (double)N;
    for (int a = 1; a <= N - 1; a++) {
        P[pidx2(N, -1, a)] = ghost2(bc, h, P[pidx2(N, 1, a)], P[pidx2(N, 0, a)],
                                    g2 ? g2[nidx2(N, 0, a)] : 0.0, 1);
        P[pidx2(N, N + 1, a)] = ghost2(bc, h, P[pidx2(N, N - 1, a)], P[pidx2(N, N, a)],
                                       g2 ? g2[nidx2(N, N, a)] : 0.0, 0);
        P[pidx2(N, a, -1)] = ghost2(bc, h, P[pidx2(N, a, 1)], P[pidx2(N, a, 0)],
                                    g2 ? g2[nidx2(N, a, 0)] : 0.0, 1);
        P[pidx2(N, a, N + 1)] = ghost2(bc, h, P[pidx2(N, a, N - 1)], P[pidx2(N, a, N)],
                                       g2 ? g2[nidx2(N, a, N)] : 0.0, 0);
    }
}

static double *padded2(int N) {
    i64 Q = (i64)N + 3;
    return (double *)calloc((size_t)(Q * Q), sizeof(double));
}

/* y = A_h x (homogeneous boundary data), interior vectors */
int oracle2d_apply(int N, int bc, const double *x, double *y) {
    if (N < 2 || (bc != 1 && bc != 2) || !x || !y) return ORC_EINVAL;
    double *P = padded2(N);
    if (!P) return ORC_ENOMEM;
    for (int j = 1; j <= N - 1; j++)
        for (int i = 1; i <= N - 1; i++) P[pidx2(N, i, j)] = x[vidx2(N, i, j)];
    fill_ghosts2(N, bc, P, NULL);
    for (int j = 1; j <= N - 1; j++)
        for (int i = 1; i <= N - 1; i++) y[vidx2(N, i, j)] = eval13(P, pidx2(N, i, j), N + 3);
    free(P);
    return ORC_OK;
}

int oracle2d_residual(int N, int bc, const double *b, const double *x, double *r) {
    int rc = oracle2d_apply(N, bc, x, r);
    if (rc) return rc;
    i64 nu = (i64)(N - 1) * (N - 1);
    for (i64 t = 0; t < nu; t++) r[t] = b[t] - r[t];
    return ORC_OK;
}

/* b = h^4 f - (the scheme on the known values): interior 0, boundary g1, fictitious points
 * from the reflections with the mirrored unknown 0 */
int oracle2d_rhs(int N, int bc, const double *f, const double *g1, const double *g2,
                 double *b) {
    if (N < 2 || (bc != 1 && bc != 2) || !f || !g1 || !g2 || !b) return ORC_EINVAL;
    double *P = padded2(N);
    if (!P) return ORC_ENOMEM;
    for (int j = 0; j <= N; j++)
        for (int i = 0; i <= N; i++) {
            int on_bnd = (i == 0 || i == N || j == 0 || j == N);
            P[pidx2(N, i, j)] = on_bnd ? g1[nidx2(N, i, j)] : 0.0;
        }
    fill_ghosts2(N, bc, P, g2);
    double h = 1.0 / (double)N;
    double h4 = h * h * h * h;
    for (int j = 1; j <= N - 1; j++)
        for (int i = 1; i <= N - 1; i++)
            b[vidx2(N, i, j)] = h4 * f[nidx2(N, i, j)] - eval13(P, pidx2(N, i, j), N + 3);
    free(P);
    return ORC_OK;
}

/* dense A_h from unit vectors (row-major) */
int oracle2d_assemble(int N, int bc, double *A) {
    if (N < 2 || (bc != 1 && bc != 2) || !A) return ORC_EINVAL;
    i64 n = (i64)(N - 1) * (N - 1);
    double *e = (double *)calloc((size_t)n, sizeof(double));
    double *col = (double *)malloc((size_t)n * sizeof(double));
    if (!e || !col) { free(e); free(col); return ORC_ENOMEM; }
    for (i64 c = 0; c < n; c++) {
        e[c] = 1.0;
        oracle2d_apply(N, bc, e, col);
        e[c] = 0.0;
        for (i64 r = 0; r < n; r++) A[r * n + c] = col[r];
    }
    free(e); free(col);
    return ORC_OK;
}

/* DSOLVE: dense Cholesky of the assembled A_h */
int oracle2d_dsolve(int N, int bc, const double *b, double *x) {
    if (N < 2 || (bc != 1 && bc != 2) || !b || !x) return ORC_EINVAL;
    i64 n = (i64)(N - 1) * (N - 1);
    double *A = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *yv = (double *)malloc((size_t)n * sizeof(double));
    if (!A || !yv) { free(A); free(yv); return ORC_ENOMEM; }
    oracle2d_assemble(N, bc, A);
    int rc = ORC_OK;
    for (i64 jj = 0; jj < n && rc == ORC_OK; jj++) {
        double s = A[jj * n + jj];
        for (i64 k = 0; k < jj; k++) s -= A[jj * n + k] * A[jj * n + k];
        if (!(s > 0.0)) { rc = ORC_EBREAKDOWN; break; }
        double d = sqrt(s);
        A[jj * n + jj] = d;
        for (i64 i = jj + 1; i < n; i++) {
            double t = A[i * n + jj];
            for (i64 k = 0; k < jj; k++) t -= A[i * n + k] * A[jj * n + k];
            A[i * n + jj] = t / d;
        }
    }
    if (rc == ORC_OK) {
        for (i64 i = 0; i < n; i++) {
            double t = b[i];
            for (i64 k = 0; k < i; k++) t -= A[i * n + k] * yv[k];
            yv[i] = t / A[i * n + i];
        }
        for (i64 i = n - 1; i >= 0; i--) {
            double t = yv[i];
            for (i64 k = i + 1; k < n; k++) t -= A[k * n + i] * x[k];
            x[i] = t / A[i * n + i];
        }
    }
    free(A); free(yv);
    return rc;
}

/* Algorithm 2 with M = I and r*_0 = r_0 (A^T applied as A: A_h is symmetric entry for
 * entry, checked on the assembled matrix by the tests); stops as oracle_bicg does. */
int oracle2d_bicg(int N, int bc, const double *b, double *x, double eps, int maxit,
                  int *iters, double *rr_out) {
    if (N < 2 || (bc != 1 && bc != 2) || !b || !x || maxit < 0) return ORC_EINVAL;
    i64 n = (i64)(N - 1) * (N - 1);
    double *r = malloc((size_t)n * sizeof(double)), *rs = malloc((size_t)n * sizeof(double));
    double *p = malloc((size_t)n * sizeof(double)), *ps = malloc((size_t)n * sizeof(double));
    double *q = malloc((size_t)n * sizeof(double)), *qs = malloc((size_t)n * sizeof(double));
    if (!r || !rs || !p || !ps || !q || !qs) {
        free(r); free(rs); free(p); free(ps); free(q); free(qs);
        return ORC_ENOMEM;
    }
    double bb = oracle_dot(n, b, b);
    double thr = (eps * eps) * bb;
    oracle2d_residual(N, bc, b, x, r);
    for (i64 t = 0; t < n; t++) { rs[t] = r[t]; p[t] = r[t]; ps[t] = rs[t]; }
    double rho = oracle_dot(n, rs, r);
    double rr = oracle_dot(n, r, r);
    int k = 0, rc = ORC_OK;
    while (!(rr <= thr)) {
        if (k >= maxit) { rc = ORC_ENOCONV; break; }
        if (rho == 0.0 || !isfinite(rho)) { rc = ORC_EBREAKDOWN; break; }
        oracle2d_apply(N, bc, p, q);
        oracle2d_apply(N, bc, ps, qs);
        double sigma = oracle_dot(n, ps, q);
        if (sigma == 0.0 || !isfinite(sigma)) { rc = ORC_EBREAKDOWN; break; }
        double alpha = rho / sigma;
        for (i64 t = 0; t < n; t++) {
            x[t] = x[t] + alpha * p[t];
            r[t] = r[t] - alpha * q[t];
            rs[t] = rs[t] - alpha * qs[t];
        }
        double rho_new = oracle_dot(n, rs, r);
        rr = oracle_dot(n, r, r);
        double beta = rho_new / rho;
        rho = rho_new;
        k++;
        for (i64 t = 0; t < n; t++) {
            p[t] = r[t] + beta * p[t];
            ps[t] = rs[t] + beta * ps[t];
        }
    }
    if (iters) *iters = k;
    if (rr_out) *rr_out = rr;
    free(r); free(rs); free(p); free(ps); free(q); free(qs);
    return rc;
}

/* Algorithm 1's while loop on one level: Bi-CG runs from the current x until the true
 * relative residual is at most eps (at most max_runs runs). */
int oracle2d_level_solve(int N, int bc, const double *b, double *x, double eps, int maxit,
                         int max_runs, int *iters, int *runs, double *rr_true, double *bb_out) {
    if (N < 2 || (bc != 1 && bc != 2) || !b || !x) return ORC_EINVAL;
    i64 n = (i64)(N - 1) * (N - 1);
    double *r = malloc((size_t)n * sizeof(double));
    if (!r) return ORC_ENOMEM;
    double bb = oracle_dot(n, b, b);
    double thr = (eps * eps) * bb;
    oracle2d_residual(N, bc, b, x, r);
    double rr = oracle_dot(n, r, r);
    int total = 0, nrun = 0, rc = ORC_OK;
    while (!(rr <= thr)) {
        if (nrun >= max_runs) { rc = ORC_ENOCONV; break; }
        int it = 0;
        double rrr = 0.0;
        int brc = oracle2d_bicg(N, bc, b, x, eps, maxit, &it, &rrr);
        total += it;
        nrun++;
        double prev = rr;
        oracle2d_residual(N, bc, b, x, r);
        rr = oracle_dot(n, r, r);
        if (brc == ORC_EBREAKDOWN || brc == ORC_ENOMEM || brc == ORC_EINVAL) { rc = brc; break; }
        /* floor-limited: the same stop as the 3D while loop (tolerance within a factor 10 of
         * the FP64 floor 22 u ||x||_2 / ||b||_2 and a run that no longer halves r.r) */
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

static double lagrange2_2d(int i, double xi) {
    static const double node[3] = {0.0, 0.5, 1.0};
    double v = 1.0;
    for (int k = 0; k < 3; k++)
        if (k != i) v = v * ((xi - node[k]) / (node[i] - node[k]));
    return v;
}

/* w = EXP_finite(u1, u0) on the grid of N cells from u1 (N/2 cells) and u0 (N/4 cells),
 * node arrays; per 5x5 interpolation cell (Steps 1-4 above). */
int oracle2d_exp_finite(int N, const double *u1, const double *u0, double *w) {
    if (N < 4 || N % 4 != 0 || !u1 || !u0 || !w) return ORC_EINVAL;
    int N1 = N / 2, N0 = N / 4;
    double L[5][3];
    for (int a = 0; a < 5; a++)
        for (int i = 0; i < 3; i++) L[a][i] = lagrange2_2d(i, a / 4.0);
    for (int cy = 0; cy < N0; cy++)
        for (int cx = 0; cx < N0; cx++) {
#define U1(al, be) u1[nidx2(N1, 2 * cx + (al), 2 * cy + (be))]
#define U0(al, be) u0[nidx2(N0, cx + (al) / 2, cy + (be) / 2)]
#define BFSEC(m0, m1, e0, e1, f0, f1) \
    (U1(m0, m1) + (1.0 / 8.0) * (U1(e0, e1) - U0(e0, e1) + U1(f0, f1) - U0(f0, f1)))
            double V[3][3]; /* [be][al] */
            /* Step 1: corners, eq. (secfff) */
            for (int be = 0; be <= 2; be += 2)
                for (int al = 0; al <= 2; al += 2)
                    V[be][al] = (5.0 * U1(al, be) - U0(al, be)) / 4.0;
            /* Step 2: edge midpoints, eq. (bfsec) along the edge */
            for (int s = 0; s <= 2; s += 2) {
                V[s][1] = BFSEC(1, s, 0, s, 2, s); /* x edges */
                V[1][s] = BFSEC(s, 1, s, 0, s, 2); /* y edges */
            }
            /* Step 3: the centre, mean over the two diagonals */
            V[1][1] = (BFSEC(1, 1, 0, 0, 2, 2) + BFSEC(1, 1, 2, 0, 0, 2)) / 2.0;
#undef BFSEC
#undef U0
#undef U1
            /* Step 4: bi-quadratic interpolation of the other nodes */
            for (int bq = 0; bq < 5; bq++)
                for (int a = 0; a < 5; a++) {
                    double val;
                    if (a % 2 == 0 && bq % 2 == 0) {
                        val = V[bq / 2][a / 2];
                    } else {
                        val = 0.0;
                        for (int be = 0; be < 3; be++)
                            for (int al = 0; al < 3; al++)
                                val = val + L[a][al] * L[bq][be] * V[be][al];
                    }
                    w[nidx2(N, 4 * cx + a, 4 * cy + bq)] = val;
                }
        }
    return ORC_OK;
}

/* u~ = EXP_true(u_h, u_2h) over all (N+1)^2 nodes */
int oracle2d_exp_true(int N, const double *uh, const double *u2h, double *ut) {
    if (N < 2 || N % 2 != 0 || !uh || !u2h || !ut) return ORC_EINVAL;
    int Nc = N / 2;
    for (int j = 0; j <= N; j++)
        for (int i = 0; i <= N; i++) {
            int oi = i & 1, oj = j & 1;
            double mid = uh[nidx2(N, i, j)];
#define CHENLIN(e0, e1, f0, f1)                                                      \
    (mid + (1.0 / 6.0) * (uh[nidx2(N, e0, e1)] - u2h[nidx2(Nc, (e0) / 2, (e1) / 2)] + \
                          uh[nidx2(N, f0, f1)] - u2h[nidx2(Nc, (f0) / 2, (f1) / 2)]))
            double v;
            if (!oi && !oj) v = (4.0 * mid - u2h[nidx2(Nc, i / 2, j / 2)]) / 3.0;
            else if (oi && !oj) v = CHENLIN(i - 1, j, i + 1, j);
            else if (!oi && oj) v = CHENLIN(i, j - 1, i, j + 1);
            else v = (CHENLIN(i - 1, j - 1, i + 1, j + 1) + CHENLIN(i + 1, j - 1, i - 1, j + 1)) / 2.0;
#undef CHENLIN
            ut[nidx2(N, i, j)] = v;
        }
    return ORC_OK;
}
