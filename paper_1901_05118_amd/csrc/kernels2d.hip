// Level kernels of the 2D biharmonic equation (eq. bvp2d) through the EXCMG pipeline (gfx950):
// right-hand side of the 13-point scheme, node/interior transfers, the bi-quadratic
// EXP_finite and EXP_true.  Node arrays are
// (N+1)^2 (x fastest), interior vectors (N-1)^2.  Every formula is evaluated in the order
// it is specified in (contraction off), as in the 3D kernels.
#include "common.hpp"
#include "internal.hpp"

namespace excmg {

namespace {

struct Finest2 {
    const double *a;
    int Nf, stride;
    __device__ __forceinline__ double at(int i, int j) const {
        const i64 M = (i64)Nf + 1;
        return a[(i64)j * stride * M + (i64)i * stride];
    }
};

// Known value at node (i, j) of the level (-1..N+1 per axis): interior unknowns 0,
// boundary nodes g1, a fictitious point the data part of eq. (reflection2) or
// (reflection4) along the edge normal with the mirrored unknown set to 0.
__device__ __forceinline__ double known2(int i, int j, int N, int bc, double h, const Finest2 &g1,
                                         const Finest2 &g2) {
    const bool ii = (i >= 1 && i <= N - 1), ji = (j >= 1 && j <= N - 1);
    if (ii && ji) return 0.0;
    const bool ib = (i >= 0 && i <= N), jb = (j >= 0 && j <= N);
    if (ib && jb) return g1.at(i, j);
    int fi = i, fj = j;
    bool low;
    if (!ib) { low = (i < 0); fi = low ? 0 : N; }
    else { low = (j < 0); fj = low ? 0 : N; }
    const double gv = g2.at(fi, fj);
    const double mirror = 0.0;
    if (bc == 1) {
        const double dudx = low ? -gv : gv;
        return low ? mirror - 2.0 * h * dudx : mirror + 2.0 * h * dudx;
    }
    const double u0 = g1.at(fi, fj);
    return -mirror + 2.0 * u0 + h * h * gv;
}

__global__ void __launch_bounds__(256)
    k_rhs2d(int N, int bc, Finest2 f, Finest2 g1, Finest2 g2, double *b) {
    const int n = N - 1;
    const i64 total = (i64)n * n;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int i = (int)(t % n) + 1, j = (int)(t / n) + 1;
    const double h = 1.0 / (double)N;
    const double h4 = h * h * h * h;
    const double fv = f.at(i, j);
    if (i >= 3 && i <= N - 3 && j >= 3 && j <= N - 3) {
        b[t] = h4 * fv - 0.0;
        return;
    }
#define KV(di, dj) known2(i + (di), j + (dj), N, bc, h, g1, g2)
    const double c = KV(0, 0);
    const double S1 = KV(-1, 0) + KV(1, 0) + KV(0, -1) + KV(0, 1);
    const double S2 = KV(-2, 0) + KV(2, 0) + KV(0, -2) + KV(0, 2);
    const double S3 = KV(-1, -1) + KV(-1, 1) + KV(1, -1) + KV(1, 1);
#undef KV
    const double E = 20.0 * c - 8.0 * S1 + S2 + 2.0 * S3;
    b[t] = h4 * fv - E;
}

template <typename T>
__global__ void __launch_bounds__(256) k_to_nodes2d(int N, Finest2 g1, const T *x, double *u) {
    const i64 M = (i64)N + 1;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * M) return;
    const int i = (int)(t % M), j = (int)(t / M);
    if (i >= 1 && i <= N - 1 && j >= 1 && j <= N - 1)
        u[t] = (double)x[(i64)(j - 1) * (N - 1) + (i - 1)];
    else
        u[t] = g1.at(i, j);
}

__global__ void __launch_bounds__(256) k_from_nodes2d(int N, const double *u, double *x) {
    const i64 n = N - 1;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    const i64 i = t % n + 1, j = t / n + 1;
    x[t] = u[j * ((i64)N + 1) + i];
}

// EXP_finite phase 1, every node of Z1 (N/2 cells) by its place in the Z0 cells: Step 1
// corners, eq. (secfff); Step 2 edge midpoints, eq. (bfsec) along the edge; Step 3 cell
// centres, the mean of eq. (bfsec) along the two diagonals.
struct Z1Plane {
    const double *u1, *u0;
    int N1, N0;
    __device__ __forceinline__ double U1(int a, int b) const { return u1[(i64)b * (N1 + 1) + a]; }
    __device__ __forceinline__ double U0(int a, int b) const {
        return u0[(i64)(b / 2) * (N0 + 1) + a / 2];
    }
    __device__ __forceinline__ double bfsec(int ma, int mb, int ea, int eb, int fa, int fb) const {
        return U1(ma, mb) + (1.0 / 8.0) * (U1(ea, eb) - U0(ea, eb) + U1(fa, fb) - U0(fa, fb));
    }
};

__global__ void __launch_bounds__(256) k_exp_finite2d_z1(Z1Plane z, double *v) {
    const i64 M = (i64)z.N1 + 1;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * M) return;
    const int a = (int)(t % M), b = (int)(t / M);
    const int pa = a & 1, pb = b & 1;
    double val;
    if (!pa && !pb) val = (5.0 * z.U1(a, b) - z.U0(a, b)) / 4.0;
    else if (pa && !pb) val = z.bfsec(a, b, a - 1, b, a + 1, b);
    else if (!pa && pb) val = z.bfsec(a, b, a, b - 1, a, b + 1);
    else
        val = (z.bfsec(a, b, a - 1, b - 1, a + 1, b + 1) + z.bfsec(a, b, a + 1, b - 1, a - 1, b + 1)) /
              2.0;
    v[t] = val;
}

// Phase 2 (Step 4): every node of Z2 from the 9 Z1 values of its cell by bi-quadratic
// Lagrange interpolation (weights l_0, l_1, l_2 at xi = a/4 per axis), summed in the node
// order of the cell (y slowest) with zero-weight terms skipped.
__constant__ double kLag2[5][3] = {{1.0, 0.0, 0.0},
                                   {0.375, 0.75, -0.125},
                                   {0.0, 1.0, 0.0},
                                   {-0.125, 0.75, 0.375},
                                   {0.0, 0.0, 1.0}};

__global__ void __launch_bounds__(256) k_exp_finite2d_z2(int N, const double *v, double *w) {
    const i64 M = (i64)N + 1;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * M) return;
    const int i = (int)(t % M), j = (int)(t / M);
    const int N0 = N / 4;
    const i64 M1 = (i64)N / 2 + 1;
    if (((i | j) & 1) == 0) {
        w[t] = v[(i64)(j / 2) * M1 + i / 2];
        return;
    }
    const int cx = min(i / 4, N0 - 1), cy = min(j / 4, N0 - 1);
    const int a = i - 4 * cx, b = j - 4 * cy;
    const int alo = (a & 1) ? 0 : a / 2, ahi = (a & 1) ? 2 : a / 2;
    const int blo = (b & 1) ? 0 : b / 2, bhi = (b & 1) ? 2 : b / 2;
    double val = 0.0;
    for (int be = blo; be <= bhi; be++)
        for (int al = alo; al <= ahi; al++) {
            const double wgt = kLag2[a][al] * kLag2[b][be];
            val = val + wgt * v[(i64)(2 * cy + be) * M1 + (2 * cx + al)];
        }
    w[t] = val;
}

// EXP_true: eq. (t1) at coarse nodes, eq. (chenlin) at edge midpoints, the mean of eq.
// (chenlin) along the two diagonals at cell centres.
__global__ void __launch_bounds__(256)
    k_exp_true2d(int N, const double *uh, const double *u2h, double *ut) {
    const i64 M = (i64)N + 1, Mc = (i64)N / 2 + 1;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * M) return;
    const int i = (int)(t % M), j = (int)(t / M);
    const int oi = i & 1, oj = j & 1;
    const double mid = uh[t];
    auto H = [&](int a, int b) { return uh[(i64)b * M + a]; };
    auto C = [&](int a, int b) { return u2h[(i64)(b / 2) * Mc + a / 2]; };
    auto chenlin = [&](int ei, int ej, int fi, int fj) {
        return mid + (1.0 / 6.0) * (H(ei, ej) - C(ei, ej) + H(fi, fj) - C(fi, fj));
    };
    double v;
    if (!oi && !oj) v = (4.0 * mid - C(i, j)) / 3.0;
    else if (oi && !oj) v = chenlin(i - 1, j, i + 1, j);
    else if (!oi && oj) v = chenlin(i, j - 1, i, j + 1);
    else v = (chenlin(i - 1, j - 1, i + 1, j + 1) + chenlin(i + 1, j - 1, i - 1, j + 1)) / 2.0;
    ut[t] = v;
}

inline dim3 grid_for(i64 total) { return dim3((unsigned)((total + 255) / 256)); }

}  // namespace

hipError_t rhs_assemble_2d(int N, int bc, int stride, int Nf, const double *f, const double *g1,
                           const double *g2, double *b, hipStream_t st) {
    Finest2 F{f, Nf, stride}, G1{g1, Nf, stride}, G2{g2, Nf, stride};
    hipLaunchKernelGGL(k_rhs2d, grid_for((i64)(N - 1) * (N - 1)), dim3(256), 0, st, N, bc, F, G1,
                       G2, b);
    return hipGetLastError();
}

template <typename T>
hipError_t to_nodes_2d(int N, int stride, int Nf, const T *x, const double *g1, double *u,
                       hipStream_t st) {
    Finest2 G1{g1, Nf, stride};
    hipLaunchKernelGGL(k_to_nodes2d<T>, grid_for((i64)(N + 1) * (N + 1)), dim3(256), 0, st, N, G1,
                       x, u);
    return hipGetLastError();
}
template hipError_t to_nodes_2d<double>(int, int, int, const double *, const double *, double *,
                                        hipStream_t);

hipError_t from_nodes_2d(int N, const double *u, double *x, hipStream_t st) {
    hipLaunchKernelGGL(k_from_nodes2d, grid_for((i64)(N - 1) * (N - 1)), dim3(256), 0, st, N, u, x);
    return hipGetLastError();
}

hipError_t exp_finite_2d(int N, const double *u1, const double *u0, double *v_scratch, double *w,
                         hipStream_t st) {
    Z1Plane z{u1, u0, N / 2, N / 4};
    hipLaunchKernelGGL(k_exp_finite2d_z1, grid_for((i64)(N / 2 + 1) * (N / 2 + 1)), dim3(256), 0,
                       st, z, v_scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_exp_finite2d_z2, grid_for((i64)(N + 1) * (N + 1)), dim3(256), 0, st, N,
                       v_scratch, w);
    return hipGetLastError();
}

hipError_t exp_true_2d(int N, const double *uh, const double *u2h, double *ut, hipStream_t st) {
    hipLaunchKernelGGL(k_exp_true2d, grid_for((i64)(N + 1) * (N + 1)), dim3(256), 0, st, N, uh,
                       u2h, ut);
    return hipGetLastError();
}


}  // namespace excmg
