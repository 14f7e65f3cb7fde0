// Streaming, reduction, transfer and direct-solve kernels of the EXCMG library (gfx950).
//
// Every kernel here reproduces the arithmetic order its operation is specified with
// (contraction off, sums left to right as the formulas are written), so results are
// deterministic and independent of the launch shape.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"
#include "step.hpp"

namespace excmg {

constexpr int kVecThreads = 256;

int vec_blocks(long long n) {
    long long b = (n + kVecThreads * 4 - 1) / (kVecThreads * 4);
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    return (int)b;
}

// Bi-CG updates: fewer, larger workgroups (their partials are merged again by every
// workgroup of the next sweep A), four elements per thread; on grids of up to 2^18 unknowns,
// which are bound by latency, one element per thread (32^3: 18.2 -> 16.0 ms per level).
constexpr int kUpdateThreads = 512;

int update_blocks(long long n) {
    long long b = (n + kUpdateThreads * 4 - 1) / (kUpdateThreads * 4);
    if (n <= (1LL << 18)) b = (n + kUpdateThreads - 1) / kUpdateThreads;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

// Address of element v of a grid-stride walk v = v0, v0 + stride, ... over the n unknowns
// of a vector stored with padded rows (Rows): the walk, and so the elements each thread
// takes and the order of its partial sums, is the contiguous vector's; only the address
// moves.  Row and column are carried by additions, so no division per element.
template <bool PAD>
struct Walk {
    long long row = 0, srow = 0;
    int col = 0, scol = 0, len = 1, ld = 1;
    __device__ Walk(Rows r, long long v0, long long stride) {
        if constexpr (PAD) {
            len = r.len;
            ld = r.ld;
            row = v0 / len;
            col = (int)(v0 % len);
            srow = stride / len;
            scol = (int)(stride % len);
        }
    }
    __device__ long long at(long long v) const {
        if constexpr (PAD) return row * ld + col;
        else return v;
    }
    __device__ void advance() {
        if constexpr (PAD) {
            col += scol;
            row += srow;
            if (col >= len) {
                col -= len;
                row++;
            }
        }
    }
};

// ------------------------------------------------------------------ Bi-CG updates

// Algorithm 2: x_{k+1} = x_k + alpha p_k, r_{k+1} = r_k - alpha A p_k,
// r*_{k+1} = r*_k - alpha (p*_k A); partials of r*.r (rho of the next step) and r.r.
// The iterate x may be FP64 while the Bi-CG vectors are FP32 (iterative refinement updates
// the FP64 solution directly).
// With a StepLink the kernel first merges sweep A's partials itself (sigma, alpha).
template <typename TX, typename T, bool PAD>
__global__ void __launch_bounds__(kUpdateThreads)
    k_bicg_update(long long n, const BicgState *s, TX *x, const T *p, T *r, const T *q, T *rs,
                  const T *qs, Pair *partials, StepLink link, Rows rows) {
    __shared__ Pair sh[2 * (kUpdateThreads / kWave)];
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long v0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    Walk<PAD> w(rows, v0, stride);
    // this thread's first element is requested before the status and the scalars, whose
    // loads and merge would otherwise be waited for first (launch latency on small grids)
    TX x0 = 0;
    T p0 = 0, r0 = 0, q0 = 0, s0 = 0, t0 = 0;
    const bool upd_x = (x != nullptr);   // else the next sweep A applies x += alpha p
    if (v0 < n) {
        const long long i0 = w.at(v0);
        if (upd_x) {
            x0 = x[i0];
            p0 = p[i0];
        }
        r0 = r[i0];
        q0 = q[i0];
        s0 = rs[i0];
        t0 = qs[i0];
    }
    if (!block_running(&s->status)) {
        // after a sweep A that stopped the run owing the iterate's update: the final status
        BicgState *w = link.state;   // deferred updates run with folded finalisations
        if (!upd_x && w && blockIdx.x == 0 && threadIdx.x == 0 && w->status == kStopping)
            w->status = w->poll_status;
        return;
    }
    double alpha;
    if (link.state) {
        if (!link_alpha(link, alpha, sh)) return;
    } else {
        alpha = s->alpha;
    }
    Pair acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (long long v = v0; v < n; v += stride, w.advance()) {
        const long long i = w.at(v);
        if (v != v0) {
            if (upd_x) {
                x0 = x[i];
                p0 = p[i];
            }
            r0 = r[i];
            q0 = q[i];
            s0 = rs[i];
            t0 = qs[i];
        }
        double ri = (double)r0 - alpha * (double)q0;
        double si = (double)s0 - alpha * (double)t0;
        T rt = (T)ri, st = (T)si;
        if (upd_x) x[i] = (TX)((double)x0 + alpha * (double)p0);
        r[i] = rt;
        rs[i] = st;
        dot2_acc(acc[0], (double)st, (double)rt);
        dot2_acc(acc[1], (double)rt, (double)rt);
    }
    block_merge<2>(acc, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = acc[0];
        partials[gridDim.x + blockIdx.x] = acc[1];
    }
}

template <typename TX, typename T>
hipError_t bicg_update(long long n, const BicgState *s, TX *x, const T *p, T *r, const T *q,
                       T *rs, const T *qs, Pair *partials, hipStream_t st, StepLink link,
                       Rows rows) {
    if (rows.ld != rows.len)
        hipLaunchKernelGGL((k_bicg_update<TX, T, true>), dim3(update_blocks(n)), dim3(kUpdateThreads),
                           0, st, n, s, x, p, r, q, rs, qs, partials, link, rows);
    else
        hipLaunchKernelGGL((k_bicg_update<TX, T, false>), dim3(update_blocks(n)), dim3(kUpdateThreads),
                           0, st, n, s, x, p, r, q, rs, qs, partials, link, rows);
    return hipGetLastError();
}
template hipError_t bicg_update<double, double>(long long, const BicgState *, double *,
                                                const double *, double *, const double *,
                                                double *, const double *, Pair *, hipStream_t,
                                                StepLink, Rows);
template hipError_t bicg_update<double, float>(long long, const BicgState *, double *,
                                               const float *, float *, const float *, float *,
                                               const float *, Pair *, hipStream_t, StepLink,
                                               Rows);


// CG sweep B: the primal half of the Bi-CG update (the shadow half repeats it bit for bit
// when r*_0 = r_0), and the partials of r.r, which is also rho of the next iteration.
template <typename TX, typename T, bool PAD>
__global__ void __launch_bounds__(kUpdateThreads)
    k_cg_update(long long n, const BicgState *s, TX *x, const T *p, T *r, const T *q,
                Pair *partials, StepLink link, Rows rows) {
    __shared__ Pair sh[kUpdateThreads / kWave];
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long v0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    Walk<PAD> w(rows, v0, stride);
    // first element requested before the status and the scalars (see k_bicg_update)
    TX x0 = 0;
    T p0 = 0, r0 = 0, q0 = 0;
    if (v0 < n) {
        const long long i0 = w.at(v0);
        x0 = x[i0];
        p0 = p[i0];
        r0 = r[i0];
        q0 = q[i0];
    }
    if (!block_running(&s->status)) return;
    double alpha;
    if (link.state) {
        if (!link_alpha(link, alpha, sh)) return;
    } else {
        alpha = s->alpha;
    }
    Pair acc[1] = {{0.0, 0.0}};
    for (long long v = v0; v < n; v += stride, w.advance()) {
        const long long i = w.at(v);
        if (v != v0) {
            x0 = x[i];
            p0 = p[i];
            r0 = r[i];
            q0 = q[i];
        }
        double xi = (double)x0 + alpha * (double)p0;
        double ri = (double)r0 - alpha * (double)q0;
        T rt = (T)ri;
        x[i] = (TX)xi;
        r[i] = rt;
        dot2_acc(acc[0], (double)rt, (double)rt);
    }
    block_merge<1>(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

template <typename TX, typename T>
hipError_t cg_update(long long n, const BicgState *s, TX *x, const T *p, T *r, const T *q,
                     Pair *partials, hipStream_t st, StepLink link, Rows rows) {
    if (rows.ld != rows.len)
        hipLaunchKernelGGL((k_cg_update<TX, T, true>), dim3(update_blocks(n)), dim3(kUpdateThreads), 0,
                           st, n, s, x, p, r, q, partials, link, rows);
    else
        hipLaunchKernelGGL((k_cg_update<TX, T, false>), dim3(update_blocks(n)), dim3(kUpdateThreads), 0,
                           st, n, s, x, p, r, q, partials, link, rows);
    return hipGetLastError();
}
template hipError_t cg_update<double, double>(long long, const BicgState *, double *,
                                              const double *, double *, const double *, Pair *,
                                              hipStream_t, StepLink, Rows);
template hipError_t cg_update<double, float>(long long, const BicgState *, double *,
                                             const float *, float *, const float *, Pair *,
                                             hipStream_t, StepLink, Rows);

// Partials of r*.r and r.r with the block layout of the Bi-CG update kernels, for a run
// whose residuals were just replaced (its next sweep A merges them as the rho of the step).
template <typename T>
__global__ void __launch_bounds__(kUpdateThreads)
    k_rho_partials(long long n, const T *r, const T *rs, const T *d, Pair *partials, Rows rows) {
    __shared__ Pair sh[2 * (kUpdateThreads / kWave)];
    Pair acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long v0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    Walk<true> w(rows, v0, stride);
    for (long long v = v0; v < n; v += stride, w.advance()) {
        const long long i = w.at(v);
        const double z = d ? (double)r[i] / (double)d[i] : (double)r[i];
        dot2_acc(acc[0], (double)rs[i], z);
        dot2_acc(acc[1], (double)r[i], (double)r[i]);
    }
    block_merge<2>(acc, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = acc[0];
        partials[gridDim.x + blockIdx.x] = acc[1];
    }
}

template <typename T>
hipError_t rho_partials(long long n, const T *r, const T *rs, Pair *partials, hipStream_t st,
                        const T *d, Rows rows, int nblocks) {
    // nblocks: the partial count the next sweep A merges (default: the update sweep's)
    hipLaunchKernelGGL(k_rho_partials<T>, dim3(nblocks > 0 ? nblocks : update_blocks(n)),
                       dim3(kUpdateThreads), 0, st, n, r, rs, d, partials, rows);
    return hipGetLastError();
}
template hipError_t rho_partials<float>(long long, const float *, const float *, Pair *,
                                        hipStream_t, const float *, Rows, int);
template hipError_t rho_partials<double>(long long, const double *, const double *, Pair *,
                                         hipStream_t, const double *, Rows, int);

// Sweep B of Algorithm 2 with its options, in the order of the algorithm: x, x*, r, r*
// updates, then M^-1 r and the partials of r*.(M^-1 r) and r.r.
template <bool PRE, bool DUAL>
__global__ void __launch_bounds__(kUpdateThreads)
    k_bicg_update_ex(long long n, const BicgState *s, double *x, const double *p, double *r,
                     const double *q, double *rs, const double *qs, const double *d, double *xs,
                     const double *ps, Pair *partials, StepLink link) {
    __shared__ Pair sh[2 * (kUpdateThreads / kWave)];
    if (!block_running(&s->status)) return;
    double alpha;
    if (link.state) {
        if (!link_alpha(link, alpha, sh)) return;
    } else {
        alpha = s->alpha;
    }
    Pair acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xi = x[i] + alpha * p[i];
        x[i] = xi;
        if (DUAL) xs[i] = xs[i] + alpha * ps[i];
        const double ri = r[i] - alpha * q[i];
        const double si = rs[i] - alpha * qs[i];
        r[i] = ri;
        rs[i] = si;
        const double z = PRE ? ri / d[i] : ri;
        dot2_acc(acc[0], si, z);
        dot2_acc(acc[1], ri, ri);
    }
    block_merge<2>(acc, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = acc[0];
        partials[gridDim.x + blockIdx.x] = acc[1];
    }
}

hipError_t bicg_update_ex(long long n, const BicgState *s, double *x, const double *p,
                          double *r, const double *q, double *rs, const double *qs,
                          const double *d, double *xs, const double *ps, Pair *partials,
                          hipStream_t st, StepLink link) {
    const dim3 grid(update_blocks(n)), block(kUpdateThreads);
    if (d && xs)
        hipLaunchKernelGGL((k_bicg_update_ex<true, true>), grid, block, 0, st, n, s, x, p, r, q,
                           rs, qs, d, xs, ps, partials, link);
    else if (d)
        hipLaunchKernelGGL((k_bicg_update_ex<true, false>), grid, block, 0, st, n, s, x, p, r, q,
                           rs, qs, d, xs, ps, partials, link);
    else if (xs)
        hipLaunchKernelGGL((k_bicg_update_ex<false, true>), grid, block, 0, st, n, s, x, p, r, q,
                           rs, qs, d, xs, ps, partials, link);
    else
        hipLaunchKernelGGL((k_bicg_update_ex<false, false>), grid, block, 0, st, n, s, x, p, r, q,
                           rs, qs, d, xs, ps, partials, link);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kVecThreads)
    k_operator_diagonal(int n, double sgn, double *d, int dim) {
    const i64 total = (i64)n * n * (dim == 2 ? 1 : n);
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int i = (int)(t % n), j = (int)((t / n) % n), k = (dim == 2) ? 1 : (int)(t / ((i64)n * n));
    int m = (i == 0) + (i == n - 1) + (j == 0) + (j == n - 1);
    if (dim == 3) m += (k == 0) + (k == n - 1);
    d[t] = (dim == 2 ? 20.0 : 42.0) + sgn * (double)m;
}

hipError_t operator_diagonal(int n, double sgn, double *d, hipStream_t st, int dim) {
    const i64 total = (i64)n * n * (dim == 2 ? 1 : n);
    hipLaunchKernelGGL(k_operator_diagonal, dim3((unsigned)((total + kVecThreads - 1) / kVecThreads)),
                       dim3(kVecThreads), 0, st, n, sgn, d, dim);
    return hipGetLastError();
}

// Let a stopped run go on: running again (unless at its iteration cap), with a new
// stopping threshold for the recurrence residual.
__global__ void k_state_resume(BicgState *s, double thr) {
    if (threadIdx.x == 0) {
        s->thr = thr;
        s->status = (s->iter >= s->maxit) ? kNoConv : kRunning;
        s->poll_status = s->status;
    }
}

hipError_t state_resume(BicgState *s, double thr, hipStream_t st) {
    hipLaunchKernelGGL(k_state_resume, dim3(1), dim3(kWave), 0, st, s, thr);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kReduceThreads) k_step_check(StepLink link) {
    __shared__ Pair sh[2 * (kReduceThreads / kWave)];
    if (!block_running(&link.state->status)) return;
    double beta;
    (void)link_step(link, beta, sh);
}

hipError_t step_check(StepLink link, hipStream_t st) {
    hipLaunchKernelGGL(k_step_check, dim3(1), dim3(kReduceThreads), 0, st, link);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kVecThreads)
    k_dot(long long n, const T *x, const T *y, Pair *partials, Rows rows) {
    __shared__ Pair sh[kVecThreads / kWave];
    Pair acc[1] = {{0.0, 0.0}};
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long v0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    Walk<true> w(rows, v0, stride);
    for (long long v = v0; v < n; v += stride, w.advance()) {
        const long long i = w.at(v);
        dot2_acc(acc[0], (double)x[i], (double)y[i]);
    }
    block_merge<1>(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

template <typename T>
hipError_t dot_partials(long long n, const T *x, const T *y, Pair *partials, int nblocks,
                        hipStream_t st, Rows rows) {
    hipLaunchKernelGGL(k_dot<T>, dim3(nblocks), dim3(kVecThreads), 0, st, n, x, y, partials, rows);
    return hipGetLastError();
}
template hipError_t dot_partials<double>(long long, const double *, const double *, Pair *, int,
                                         hipStream_t, Rows);
template hipError_t dot_partials<float>(long long, const float *, const float *, Pair *, int,
                                        hipStream_t, Rows);

// One workgroup row at a time (grid-stride over the n^2 rows of an n^3 vector).
__global__ void __launch_bounds__(kVecThreads)
    k_pad_rows(int n, int ld, const double *src, double *dst) {
    const long long rows = (long long)n * n;
    for (long long row = blockIdx.x; row < rows; row += gridDim.x)
        for (int c = threadIdx.x; c < ld; c += blockDim.x)
            dst[row * ld + c] = c < n ? src[row * n + c] : 0.0;
}

__global__ void __launch_bounds__(kVecThreads)
    k_unpad_rows(int n, int ld, const double *src, double *dst) {
    const long long rows = (long long)n * n;
    for (long long row = blockIdx.x; row < rows; row += gridDim.x)
        for (int c = threadIdx.x; c < n; c += blockDim.x) dst[row * n + c] = src[row * ld + c];
}

hipError_t pad_rows(int n, int ld, const double *src, double *dst, hipStream_t st) {
    if (n < 1 || ld < n) return hipErrorInvalidValue;
    const long long rows = (long long)n * n;
    hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)std::min(rows, 8192LL)), dim3(kVecThreads), 0, st,
                       n, ld, src, dst);
    return hipGetLastError();
}

hipError_t unpad_rows(int n, int ld, const double *src, double *dst, hipStream_t st) {
    if (n < 1 || ld < n) return hipErrorInvalidValue;
    const long long rows = (long long)n * n;
    hipLaunchKernelGGL(k_unpad_rows, dim3((unsigned)std::min(rows, 8192LL)), dim3(kVecThreads), 0, st,
                       n, ld, src, dst);
    return hipGetLastError();
}

template <typename TD, typename TS>
__global__ void k_copy_convert(long long n, const TS *src, TD *dst) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = (TD)src[i];
}

template <typename TD, typename TS>
hipError_t copy_convert(long long n, const TS *src, TD *dst, hipStream_t st) {
    hipLaunchKernelGGL((k_copy_convert<TD, TS>), dim3(vec_blocks(n)), dim3(kVecThreads), 0, st, n,
                       src, dst);
    return hipGetLastError();
}
template hipError_t copy_convert<double, double>(long long, const double *, double *,
                                                 hipStream_t);
template hipError_t copy_convert<float, double>(long long, const double *, float *, hipStream_t);
template hipError_t copy_convert<double, float>(long long, const float *, double *, hipStream_t);
template hipError_t copy_convert<float, float>(long long, const float *, float *, hipStream_t);

// ------------------------------------------------------------------ finalisation

// Merge `count` pairs (stride apart per value) in a fixed order; result in thread 0.
template <int NV>
__device__ void merge_partials(const Pair *part, int count, Pair (&out)[NV], Pair *sh) {
    for (int q = 0; q < NV; q++) out[q] = Pair{0.0, 0.0};
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < NV; q++) out[q] = pair_merge(out[q], part[q * count + i]);
    }
    block_merge<NV>(out, sh);
}

__device__ void set_status(BicgState *s) {
    // the order of the checks follows the loop of Algorithm 2 as run by the oracle
    if (s->rr <= s->thr) s->status = kConverged;
    else if (s->iter >= s->maxit) s->status = kNoConv;
    else if (s->rho == 0.0 || !isfinite(s->rho)) s->status = kBreakdown;
    else s->status = kRunning;
    s->poll_status = s->status;
}

__global__ void __launch_bounds__(kReduceThreads)
    k_bicg_start(BicgState *s, const Pair *part, int count, double eps, int maxit) {
    __shared__ Pair sh[kReduceThreads / kWave];
    Pair v[1];
    merge_partials<1>(part, count, v, sh);
    if (threadIdx.x == 0) {
        double rr = pair_value(v[0]);
        s->rr = rr;
        s->rho = rr;  // r*_0 = r_0
        s->rho_slot[0] = rr;
        s->thr = (eps * eps) * s->bb;
        s->iter = 0;
        s->maxit = maxit;
        s->alpha = 0.0;
        s->beta = 0.0;
        s->sigma = 0.0;
        set_status(s);
    }
}

__global__ void __launch_bounds__(kReduceThreads)
    k_bicg_start2(BicgState *s, const Pair *part, int count, double eps, int maxit) {
    __shared__ Pair sh[2 * (kReduceThreads / kWave)];
    Pair v[2];
    merge_partials<2>(part, count, v, sh);
    if (threadIdx.x == 0) {
        s->rho = pair_value(v[0]);
        s->rho_slot[0] = s->rho;
        s->rr = pair_value(v[1]);
        s->thr = (eps * eps) * s->bb;
        s->iter = 0;
        s->maxit = maxit;
        s->alpha = 0.0;
        s->beta = 0.0;
        s->sigma = 0.0;
        set_status(s);
    }
}

hipError_t bicg_start2(BicgState *s, const Pair *part, int count, double eps, int maxit,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_bicg_start2, dim3(1), dim3(kReduceThreads), 0, st, s, part, count, eps,
                       maxit);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kReduceThreads)
    k_reduce_to(double *out, const Pair *part, int count, int slot) {
    __shared__ Pair sh[kReduceThreads / kWave];
    Pair v[1];
    merge_partials<1>(part, count, v, sh);
    if (threadIdx.x == 0) out[slot] = pair_value(v[0]);
}

hipError_t bicg_start(BicgState *s, const Pair *rr_part, int count, double eps, int maxit,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_bicg_start, dim3(1), dim3(kReduceThreads), 0, st, s, rr_part, count, eps,
                       maxit);
    return hipGetLastError();
}
hipError_t reduce_to(double *out, const Pair *part, int count, int slot, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(kReduceThreads), 0, st, out, part, count, slot);
    return hipGetLastError();
}

// ------------------------------------------------------------------ right-hand side

struct Finest {
    const double *a;
    int Nf, stride;
    __device__ __forceinline__ double at(int i, int j, int k) const {
        const i64 M = (i64)Nf + 1;
        return a[((i64)k * stride * M + (i64)j * stride) * M + (i64)i * stride];
    }
};

// Known value of the 25-point equation at node (i, j, k) of the level (-1..N+1 per axis):
// interior nodes are unknowns (0 here), boundary nodes are g1, and a fictitious point
// carries the data part of eq. (reflection2) or (reflection4) with the mirrored unknown
// set to 0.
__device__ __forceinline__ double known_value(int i, int j, int k, int N, int bc, double h,
                                              const Finest &g1, const Finest &g2) {
    const bool ii = (i >= 1 && i <= N - 1), ji = (j >= 1 && j <= N - 1), ki = (k >= 1 && k <= N - 1);
    if (ii && ji && ki) return 0.0;
    const bool ib = (i >= 0 && i <= N), jb = (j >= 0 && j <= N), kb = (k >= 0 && k <= N);
    if (ib && jb && kb) return g1.at(i, j, k);
    // fictitious point: exactly one coordinate is -1 or N+1, the others are interior
    int fi = i, fj = j, fk = k;
    bool low;
    if (!ib) { low = (i < 0); fi = low ? 0 : N; }
    else if (!jb) { low = (j < 0); fj = low ? 0 : N; }
    else { low = (k < 0); fk = low ? 0 : N; }
    const double gv = g2.at(fi, fj, fk);
    const double mirror = 0.0;
    if (bc == 1) {
        const double dudx = low ? -gv : gv;
        return low ? mirror - 2.0 * h * dudx : mirror + 2.0 * h * dudx;
    }
    const double u0 = g1.at(fi, fj, fk);
    return -mirror + 2.0 * u0 + h * h * gv;
}

__global__ void __launch_bounds__(256)
    k_rhs(int N, int bc, Finest f, Finest g1, Finest g2, double *b) {
    const int n = N - 1;
    const i64 total = (i64)n * n * n;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int i = (int)(t % n) + 1;
    const int j = (int)((t / n) % n) + 1;
    const int k = (int)(t / ((i64)n * n)) + 1;
    const double h = 1.0 / (double)N;
    const double h4 = h * h * h * h;
    const double fv = f.at(i, j, k);
    const bool deep = (i >= 3 && i <= N - 3 && j >= 3 && j <= N - 3 && k >= 3 && k <= N - 3);
    if (deep) {  // every neighbour is an unknown: the known part is exactly +0
        b[t] = h4 * fv - 0.0;
        return;
    }
#define KV(di, dj, dk) known_value(i + (di), j + (dj), k + (dk), N, bc, h, g1, g2)
    const double c = KV(0, 0, 0);
    const double S1 = KV(-1, 0, 0) + KV(1, 0, 0) + KV(0, -1, 0) + KV(0, 1, 0) + KV(0, 0, -1) +
                      KV(0, 0, 1);
    const double S2 = KV(-2, 0, 0) + KV(2, 0, 0) + KV(0, -2, 0) + KV(0, 2, 0) + KV(0, 0, -2) +
                      KV(0, 0, 2);
    // the three printed groups of four (plane k, k-1, k+1), each summed first
    const double Dk = KV(-1, -1, 0) + KV(-1, 1, 0) + KV(1, -1, 0) + KV(1, 1, 0);
    const double Dm = KV(-1, 0, -1) + KV(1, 0, -1) + KV(0, -1, -1) + KV(0, 1, -1);
    const double Dp = KV(-1, 0, 1) + KV(1, 0, 1) + KV(0, -1, 1) + KV(0, 1, 1);
    const double S3 = Dk + Dm + Dp;
#undef KV
    const double E = 42.0 * c - 12.0 * S1 + S2 + 2.0 * S3;
    b[t] = h4 * fv - E;
}

hipError_t rhs_assemble(int N, int bc, int stride, int Nf, const double *f, const double *g1,
                        const double *g2, double *b, hipStream_t st) {
    const i64 total = (i64)(N - 1) * (N - 1) * (N - 1);
    Finest F{f, Nf, stride}, G1{g1, Nf, stride}, G2{g2, Nf, stride};
    hipLaunchKernelGGL(k_rhs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, N, bc, F,
                       G1, G2, b);
    return hipGetLastError();
}

// ------------------------------------------------------------------ node arrays

template <typename T>
__global__ void __launch_bounds__(256)
    k_to_nodes(int N, Finest g1, const T *x, double *u) {
    const i64 M = (i64)N + 1;
    const i64 total = M * M * M;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int i = (int)(t % M), j = (int)((t / M) % M), k = (int)(t / (M * M));
    const bool interior = (i >= 1 && i <= N - 1 && j >= 1 && j <= N - 1 && k >= 1 && k <= N - 1);
    if (interior) {
        const i64 n = N - 1;
        u[t] = (double)x[((i64)(k - 1) * n + (j - 1)) * n + (i - 1)];
    } else {
        u[t] = g1.at(i, j, k);
    }
}

template <typename T>
hipError_t to_nodes(int N, int stride, int Nf, const T *x, const double *g1, double *u,
                    hipStream_t st) {
    const i64 M = (i64)N + 1;
    Finest G1{g1, Nf, stride};
    hipLaunchKernelGGL(k_to_nodes<T>, dim3((unsigned)((M * M * M + 255) / 256)), dim3(256), 0, st,
                       N, G1, x, u);
    return hipGetLastError();
}
template hipError_t to_nodes<double>(int, int, int, const double *, const double *, double *,
                                     hipStream_t);

__global__ void __launch_bounds__(256) k_from_nodes(int N, const double *u, double *x) {
    const i64 n = N - 1;
    const i64 total = n * n * n;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const i64 i = t % n + 1, j = (t / n) % n + 1, k = t / (n * n) + 1;
    const i64 M = (i64)N + 1;
    x[t] = u[(k * M + j) * M + i];
}

hipError_t from_nodes(int N, const double *u, double *x, hipStream_t st) {
    const i64 n = N - 1;
    hipLaunchKernelGGL(k_from_nodes, dim3((unsigned)((n * n * n + 255) / 256)), dim3(256), 0, st,
                       N, u, x);
    return hipGetLastError();
}

// ------------------------------------------------------------------ EXP_finite

// Phase 1: the value of every node of Z1 (grid of N1 = N/2 cells), by its place in the
// interpolation cells of Z0 (N0 = N/4 cells): Step 1 for nodes of Z0, eq. (secfff); Step 2
// for edge midpoints, eq. (bfsec); Step 3 for face centres, the mean of eq. (bfsec) on the
// two face diagonals; Step 4 for cell centres, the mean on the four space diagonals.
struct Z1Grid {
    const double *u1, *u0;
    int N1, N0;
    __device__ __forceinline__ double U1(int a, int b, int c) const {
        const i64 M = (i64)N1 + 1;
        return u1[((i64)c * M + b) * M + a];
    }
    __device__ __forceinline__ double U0(int a, int b, int c) const {  // even Z1 coordinates
        const i64 M = (i64)N0 + 1;
        return u0[((i64)(c / 2) * M + b / 2) * M + a / 2];
    }
    // eq. (bfsec) at Z1 node m on the segment from corner e to corner f
    __device__ __forceinline__ double bfsec(int ma, int mb, int mc, int ea, int eb, int ec,
                                            int fa, int fb, int fc) const {
        return U1(ma, mb, mc) +
               (1.0 / 8.0) * (U1(ea, eb, ec) - U0(ea, eb, ec) + U1(fa, fb, fc) - U0(fa, fb, fc));
    }
};

__global__ void __launch_bounds__(256) k_exp_finite_z1(Z1Grid z, double *v) {
    const i64 M = (i64)z.N1 + 1;
    const i64 total = M * M * M;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int a = (int)(t % M), b = (int)((t / M) % M), c = (int)(t / (M * M));
    const int pa = a & 1, pb = b & 1, pc = c & 1;
    const int odd = pa + pb + pc;
    double val;
    if (odd == 0) {
        val = (5.0 * z.U1(a, b, c) - z.U0(a, b, c)) / 4.0;
    } else if (odd == 1) {
        if (pa) val = z.bfsec(a, b, c, a - 1, b, c, a + 1, b, c);
        else if (pb) val = z.bfsec(a, b, c, a, b - 1, c, a, b + 1, c);
        else val = z.bfsec(a, b, c, a, b, c - 1, a, b, c + 1);
    } else if (odd == 2) {
        if (!pc) {        // face normal to z: diagonals in x-y
            val = (z.bfsec(a, b, c, a - 1, b - 1, c, a + 1, b + 1, c) +
                   z.bfsec(a, b, c, a + 1, b - 1, c, a - 1, b + 1, c)) / 2.0;
        } else if (!pb) { // face normal to y: diagonals in x-z
            val = (z.bfsec(a, b, c, a - 1, b, c - 1, a + 1, b, c + 1) +
                   z.bfsec(a, b, c, a + 1, b, c - 1, a - 1, b, c + 1)) / 2.0;
        } else {          // face normal to x: diagonals in y-z
            val = (z.bfsec(a, b, c, a, b - 1, c - 1, a, b + 1, c + 1) +
                   z.bfsec(a, b, c, a, b + 1, c - 1, a, b - 1, c + 1)) / 2.0;
        }
    } else {
        val = (z.bfsec(a, b, c, a - 1, b - 1, c - 1, a + 1, b + 1, c + 1) +
               z.bfsec(a, b, c, a + 1, b - 1, c - 1, a - 1, b + 1, c + 1) +
               z.bfsec(a, b, c, a - 1, b + 1, c - 1, a + 1, b - 1, c + 1) +
               z.bfsec(a, b, c, a + 1, b + 1, c - 1, a - 1, b - 1, c + 1)) / 4.0;
    }
    v[t] = val;
}

// Phase 2 (Step 5): every node of Z2 (N cells) from the 27 Z1 values of its interpolation
// cell by tri-quadratic Lagrange interpolation, eqs. (inter)-(iinter).  Along an axis the
// local position a = 0..4 (in steps of h) has the weights l_0, l_1, l_2 at xi = a/4; even
// positions select one node with weight 1.  Terms are summed in the node order of the cell
// (z slowest, x fastest) and zero-weight terms are skipped, which leaves every sum unchanged.
__constant__ double kLag[5][3] = {{1.0, 0.0, 0.0},
                                  {0.375, 0.75, -0.125},
                                  {0.0, 1.0, 0.0},
                                  {-0.125, 0.75, 0.375},
                                  {0.0, 0.0, 1.0}};

__global__ void __launch_bounds__(256) k_exp_finite_z2(int N, const double *v, double *w) {
    const i64 M = (i64)N + 1;
    const i64 total = M * M * M;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int i = (int)(t % M), j = (int)((t / M) % M), k = (int)(t / (M * M));
    const int N1 = N / 2, N0 = N / 4;
    const i64 M1 = (i64)N1 + 1;
    if (((i | j | k) & 1) == 0) {
        w[t] = v[((i64)(k / 2) * M1 + j / 2) * M1 + i / 2];
        return;
    }
    const int cx = min(i / 4, N0 - 1), cy = min(j / 4, N0 - 1), cz = min(k / 4, N0 - 1);
    const int a = i - 4 * cx, b = j - 4 * cy, c = k - 4 * cz;
    const int alo = (a & 1) ? 0 : a / 2, ahi = (a & 1) ? 2 : a / 2;
    const int blo = (b & 1) ? 0 : b / 2, bhi = (b & 1) ? 2 : b / 2;
    const int clo = (c & 1) ? 0 : c / 2, chi = (c & 1) ? 2 : c / 2;
    double val = 0.0;
    for (int ga = clo; ga <= chi; ga++)
        for (int be = blo; be <= bhi; be++)
            for (int al = alo; al <= ahi; al++) {
                const double wgt = kLag[a][al] * kLag[b][be] * kLag[c][ga];
                val = val + wgt * v[((i64)(2 * cz + ga) * M1 + (2 * cy + be)) * M1 + (2 * cx + al)];
            }
    w[t] = val;
}

hipError_t exp_finite(int N, const double *u1, const double *u0, double *v_scratch, double *w,
                      hipStream_t st) {
    Z1Grid z{u1, u0, N / 2, N / 4};
    const i64 M1 = (i64)N / 2 + 1;
    hipLaunchKernelGGL(k_exp_finite_z1, dim3((unsigned)((M1 * M1 * M1 + 255) / 256)), dim3(256), 0,
                       st, z, v_scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const i64 M = (i64)N + 1;
    hipLaunchKernelGGL(k_exp_finite_z2, dim3((unsigned)((M * M * M + 255) / 256)), dim3(256), 0,
                       st, N, v_scratch, w);
    return hipGetLastError();
}

// ------------------------------------------------------------------ EXP_true

// Coarse nodes: eq. (t1); edge midpoints of coarse cells: eq. (chenlin) along the edge; face
// and cell centres: mean of eq. (chenlin) over the two face diagonals or four space
// diagonals (the three-dimensional form of Steps 3-4).
struct TrueGrid {
    const double *uh, *u2h;
    int N;
    __device__ __forceinline__ double H(int i, int j, int k) const {
        const i64 M = (i64)N + 1;
        return uh[((i64)k * M + j) * M + i];
    }
    __device__ __forceinline__ double C(int i, int j, int k) const {  // even fine coordinates
        const i64 M = (i64)N / 2 + 1;
        return u2h[((i64)(k / 2) * M + j / 2) * M + i / 2];
    }
    __device__ __forceinline__ double chenlin(double mid, int ei, int ej, int ek, int fi, int fj,
                                              int fk) const {
        return mid + (1.0 / 6.0) * (H(ei, ej, ek) - C(ei, ej, ek) + H(fi, fj, fk) - C(fi, fj, fk));
    }
};

__global__ void __launch_bounds__(256) k_exp_true(TrueGrid g, double *ut) {
    const int N = g.N;
    const i64 M = (i64)N + 1;
    const i64 total = M * M * M;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int i = (int)(t % M), j = (int)((t / M) % M), k = (int)(t / (M * M));
    const int oi = i & 1, oj = j & 1, ok = k & 1;
    const double mid = g.H(i, j, k);
    double v;
    const int odd = oi + oj + ok;
    if (odd == 0) {
        v = (4.0 * mid - g.C(i, j, k)) / 3.0;
    } else if (odd == 1) {
        if (oi) v = g.chenlin(mid, i - 1, j, k, i + 1, j, k);
        else if (oj) v = g.chenlin(mid, i, j - 1, k, i, j + 1, k);
        else v = g.chenlin(mid, i, j, k - 1, i, j, k + 1);
    } else if (odd == 2) {
        if (!ok) v = (g.chenlin(mid, i - 1, j - 1, k, i + 1, j + 1, k) +
                      g.chenlin(mid, i + 1, j - 1, k, i - 1, j + 1, k)) / 2.0;
        else if (!oj) v = (g.chenlin(mid, i - 1, j, k - 1, i + 1, j, k + 1) +
                           g.chenlin(mid, i + 1, j, k - 1, i - 1, j, k + 1)) / 2.0;
        else v = (g.chenlin(mid, i, j - 1, k - 1, i, j + 1, k + 1) +
                  g.chenlin(mid, i, j + 1, k - 1, i, j - 1, k + 1)) / 2.0;
    } else {
        v = (g.chenlin(mid, i - 1, j - 1, k - 1, i + 1, j + 1, k + 1) +
             g.chenlin(mid, i + 1, j - 1, k - 1, i - 1, j + 1, k + 1) +
             g.chenlin(mid, i - 1, j + 1, k - 1, i + 1, j - 1, k + 1) +
             g.chenlin(mid, i + 1, j + 1, k - 1, i - 1, j - 1, k + 1)) / 4.0;
    }
    ut[t] = v;
}

hipError_t exp_true(int N, const double *uh, const double *u2h, double *ut, hipStream_t st) {
    TrueGrid g{uh, u2h, N};
    const i64 M = (i64)N + 1;
    hipLaunchKernelGGL(k_exp_true, dim3((unsigned)((M * M * M + 255) / 256)), dim3(256), 0, st, g,
                       ut);
    return hipGetLastError();
}

}  // namespace excmg
