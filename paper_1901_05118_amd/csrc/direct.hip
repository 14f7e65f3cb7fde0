// DSOLVE of Algorithm 1 (the two coarsest levels) on gfx950: Cholesky A_h = L L^T of the
// banded operator, then L y = b and L^T x = y.
//
// In lexicographic order (x fastest) the farthest coupling of the scheme is two lines (2D)
// or two planes (3D) away, and the folded fictitious points stay inside that reach, so A_h
// and L have lower bandwidth w = 2 (N-1)^(dim-1).  Only band entries are stored and
// visited: every entry of L outside the band is an exact zero of the dense elimination, and
// dropping its products (signed zeros) leaves every stored value unchanged.  Each
// accumulation keeps the textbook order of the dense algorithm: entry (i, j) of the
// factor subtracts L(i,k) L(j,k) for k ascending, y_i subtracts L(i,k) y_k for k
// ascending, and x_i subtracts L(k,i) x_k for k ascending from i+1.
//
// Band storage (column-major band of the lower triangle): column c of the matrix occupies
// C[c (w+1) + d], d = 0..w, holding entry (c+d, c); slots past the last row stay zero.
#include "common.hpp"
#include "internal.hpp"

namespace excmg {

namespace {

// Scatter row r of A_h into the band: a term on a fictitious point folds onto the mirrored
// unknown with factor +1 (first kind) or -1 (second kind), a term on a boundary node is
// data.  Row r writes the entries (r, c) with c <= r, which nobody else writes.  Entries
// are small integers, exact in any order.  A coupling outside the band sets bad[0].
template <int DIM>
__global__ void __launch_bounds__(256) k_band_assemble(int N, int bc, int w, double *C, int *bad) {
    const int n = N - 1;
    const int nu = DIM == 3 ? n * n * n : n * n;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nu) return;
    constexpr int NT = DIM == 3 ? 25 : 13;
    const int off3[25][3] = {{0, 0, 0},   {-1, 0, 0},  {1, 0, 0},   {0, -1, 0},  {0, 1, 0},
                             {0, 0, -1},  {0, 0, 1},   {-2, 0, 0},  {2, 0, 0},   {0, -2, 0},
                             {0, 2, 0},   {0, 0, -2},  {0, 0, 2},   {-1, -1, 0}, {-1, 1, 0},
                             {1, -1, 0},  {1, 1, 0},   {-1, 0, -1}, {1, 0, -1},  {0, -1, -1},
                             {0, 1, -1},  {-1, 0, 1},  {1, 0, 1},   {0, -1, 1},  {0, 1, 1}};
    const int off2[13][2] = {{0, 0},  {-1, 0}, {1, 0},   {0, -1},  {0, 1},  {-2, 0}, {2, 0},
                             {0, -2}, {0, 2},  {-1, -1}, {-1, 1}, {1, -1}, {1, 1}};
    int q[3] = {r % n + 1, (r / n) % n + 1, DIM == 3 ? r / (n * n) + 1 : 1};
    const double sgn = (bc == 1) ? 1.0 : -1.0;
    const i64 ld = (i64)w + 1;
    for (int t = 0; t < NT; t++) {
        double coef;
        int p[3];
        if (DIM == 3) {
            coef = (t == 0) ? 42.0 : (t <= 6) ? -12.0 : (t <= 12) ? 1.0 : 2.0;
            for (int a = 0; a < 3; a++) p[a] = q[a] + off3[t][a];
        } else {
            coef = (t == 0) ? 20.0 : (t <= 4) ? -8.0 : (t <= 8) ? 1.0 : 2.0;
            p[0] = q[0] + off2[t][0];
            p[1] = q[1] + off2[t][1];
            p[2] = 1;
        }
        bool bnd = false, ghost = false;
        for (int a = 0; a < DIM; a++) {
            if (p[a] == 0 || p[a] == N) bnd = true;
            if (p[a] == -1) { p[a] = 1; ghost = true; }
            if (p[a] == N + 1) { p[a] = N - 1; ghost = true; }
        }
        if (bnd) continue;
        const int c = ((p[2] - 1) * n + (p[1] - 1)) * n + (p[0] - 1);
        if (c > r) continue;
        if (r - c > w) {
            bad[0] = 1;
            continue;
        }
        C[(i64)c * ld + (r - c)] += ghost ? sgn * coef : coef;
    }
}

// Right-looking Cholesky of the band in one workgroup.  Step k takes the pivot (already
// reduced by steps 0..k-1), scales column k, and subtracts L(i,k) L(j,k) from every band
// entry (i, j) of the trailing window; each entry thus receives its subtractions in the
// order k = 0, 1, ... of the dense left-looking form.  info = k+1 for a pivot that is not
// positive.
__global__ void __launch_bounds__(1024) k_band_cholesky(int n, int w, double *C, int *info) {
    __shared__ double piv;
    __shared__ int fail;
    const int tid = threadIdx.x;
    const i64 ld = (i64)w + 1;
    if (tid == 0) fail = 0;
    for (int k = 0; k < n; k++) {
        double *col = C + (i64)k * ld;
        const int m = min(w, n - 1 - k);
        if (tid == 0) {
            const double s = col[0];
            if (!(s > 0.0)) fail = k + 1;
            const double d = sqrt(s);
            col[0] = d;
            piv = d;
        }
        __syncthreads();
        if (fail) break;
        const double d = piv;
        for (int e = 1 + tid; e <= m; e += blockDim.x) col[e] = col[e] / d;
        __syncthreads();
        for (int e = tid; e < m * m; e += blockDim.x) {
            const int a = e / m, b = e - a * m;  // column k+1+a, row k+1+b
            if (b < a) continue;
            C[(i64)(k + 1 + a) * ld + (b - a)] -= col[1 + b] * col[1 + a];
        }
        __syncthreads();
    }
    if (tid == 0) *info = fail;
}

constexpr int kBandMaxN = 4096;

// L y = b, then L^T x = y, in one wavefront with the vector in LDS (b and x may alias).
// Forward: column k is applied to the rows below it in parallel.  Backward: row i needs
// x_{i+1} before its first subtraction, so the chain itself is serial; the lanes form the
// products L(k,i) x_k in parallel and one lane subtracts them in ascending k.  Either way
// a step is short next to the latency of a column's load, so the columns come in chunks of
// DP: while the steps of one chunk run, the next chunk's loads are in flight (waited for
// once, at the end of the chunk).  Entry e = lane + 64 q of a column (e = 0 the diagonal,
// which lane 0 broadcasts) is loaded unconditionally from an index clamped into the
// column's w+1 stored entries; the steps mask what lies past the column's last row.
template <int PER, int DP>
__global__ void __launch_bounds__(64) k_band_solve(int n, int w, const double *C, const double *b,
                                                   double *x) {
    __shared__ double t[kBandMaxN];
    __shared__ double prod[64 * PER];
    const int lane = threadIdx.x;
    const i64 ld = (i64)w + 1;
    for (int i = lane; i < n; i += 64) t[i] = b[i];
    __syncthreads();

    auto load_col = [&](int k, double (&v)[PER]) {
        const double *col = C + (i64)k * ld;
#pragma unroll
        for (int q = 0; q < PER; q++) v[q] = col[min(lane + 64 * q, w)];
    };
    double cur[DP][PER], nxt[DP][PER];
#pragma unroll
    for (int s = 0; s < DP; s++)
#pragma unroll
        for (int q = 0; q < PER; q++) cur[s][q] = nxt[s][q] = 0.0;
    auto swap_in = [&]() {
#pragma unroll
        for (int s = 0; s < DP; s++)
#pragma unroll
            for (int q = 0; q < PER; q++) cur[s][q] = nxt[s][q];
    };

#pragma unroll
    for (int s = 0; s < DP; s++) load_col(min(s, n - 1), cur[s]);
    for (int k0 = 0; k0 < n; k0 += DP) {
        // unconditional (clamped) requests, so the loads in flight are counted exactly
#pragma unroll
        for (int s = 0; s < DP; s++) load_col(min(k0 + DP + s, n - 1), nxt[s]);
#pragma unroll
        for (int s = 0; s < DP; s++) {
            const int k = k0 + s;
            if (k < n) {
                const int m = min(w, n - 1 - k);
                const double yk = t[k] / __shfl(cur[s][0], 0);
#pragma unroll
                for (int q = 0; q < PER; q++) {
                    const int e = lane + 64 * q;
                    if (e >= 1 && e <= m) t[k + e] -= cur[s][q] * yk;
                }
                if (lane == 0) t[k] = yk;
                __syncthreads();
            }
        }
        swap_in();
    }

#pragma unroll
    for (int s = 0; s < DP; s++) load_col(max(n - 1 - s, 0), cur[s]);
    for (int k0 = 0; k0 < n; k0 += DP) {
#pragma unroll
        for (int s = 0; s < DP; s++) load_col(max(n - 1 - (k0 + DP + s), 0), nxt[s]);
#pragma unroll
        for (int s = 0; s < DP; s++) {
            const int i = n - 1 - (k0 + s);
            if (i >= 0) {
                const int m = min(w, n - 1 - i);
#pragma unroll
                for (int q = 0; q < PER; q++) {
                    const int e = lane + 64 * q;
                    if (e >= 1 && e <= m) prod[e - 1] = cur[s][q] * t[i + e];
                }
                const double d = __shfl(cur[s][0], 0);
                __syncthreads();
                if (lane == 0) {
                    double acc = t[i];
                    for (int e = 0; e < m; e++) acc -= prod[e];
                    t[i] = acc / d;
                }
                __syncthreads();
            }
        }
        swap_in();
    }
    for (int i = lane; i < n; i += 64) x[i] = t[i];
}

}  // namespace

int band_width(int N, int dim) { return dim == 2 ? 2 * (N - 1) : 2 * (N - 1) * (N - 1); }

hipError_t band_assemble(int N, int bc, int dim, int w, double *C, int *bad, hipStream_t st) {
    const int n = N - 1;
    const int nu = dim == 3 ? n * n * n : n * n;
    hipError_t e = hipMemsetAsync(C, 0, (size_t)nu * (w + 1) * sizeof(double), st);
    if (e != hipSuccess) return e;
    if (dim == 3)
        hipLaunchKernelGGL(k_band_assemble<3>, dim3((nu + 255) / 256), dim3(256), 0, st, N, bc, w,
                           C, bad);
    else
        hipLaunchKernelGGL(k_band_assemble<2>, dim3((nu + 255) / 256), dim3(256), 0, st, N, bc, w,
                           C, bad);
    return hipGetLastError();
}

hipError_t band_cholesky(int n, int w, double *C, int *info, hipStream_t st) {
    hipLaunchKernelGGL(k_band_cholesky, dim3(1), dim3(1024), 0, st, n, w, C, info);
    return hipGetLastError();
}

hipError_t band_solve(int n, int w, const double *C, const double *b, double *x, hipStream_t st) {
    if (n < 1 || n > kBandMaxN || w < 0 || w + 1 > 64 * 8) return hipErrorInvalidValue;
    const int per = (w + 64) / 64;   // the w+1 entries of a column (diagonal included)
    if (per <= 1)
        hipLaunchKernelGGL((k_band_solve<1, 8>), dim3(1), dim3(64), 0, st, n, w, C, b, x);
    else if (per <= 2)
        hipLaunchKernelGGL((k_band_solve<2, 8>), dim3(1), dim3(64), 0, st, n, w, C, b, x);
    else if (per <= 4)
        hipLaunchKernelGGL((k_band_solve<4, 4>), dim3(1), dim3(64), 0, st, n, w, C, b, x);
    else
        hipLaunchKernelGGL((k_band_solve<8, 4>), dim3(1), dim3(64), 0, st, n, w, C, b, x);
    return hipGetLastError();
}

}  // namespace excmg
