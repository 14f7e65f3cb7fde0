// Batched Bi-CG: every running system of a batch (systems of different grid sizes and boundary
// kinds, each with its own scalars) advances by one iteration of Algorithm 2 per step, in one
// of two forms:
//  * phase kernels (default): sweep A over the tiles of all systems, alpha per system, sweep B
//    over the chunks of all systems, beta per system -- four grid-stride launches with no
//    communication between workgroups inside a launch, captured G steps at a time in a
//    hipGraph;
//  * one persistent launch per step (below).  Inside a launch the workgroups hand results to
//    each other, which on MI355X needs an agent-scope release/acquire per work item (an L2
//    write-back and invalidate on each XCD); measured, this costs more than the three kernel
//    boundaries it removes, so it is the second choice.
//
// Persistent form.  Work queue.  A launch processes a list of items claimed in order through one atomic
// counter: first every sweep-A item (one z-marched stencil tile of one system: direction
// update, A p, A^T p*, partial of sigma), then every sweep-B item (one chunk of one system's
// vectors: x, r, r* updates, partials of rho and r.r).  The last sweep-A item of a system
// (per-system arrival counter) merges that system's partials and computes alpha; the last
// sweep-B item computes beta, r.r and the stopping status.  A sweep-B item waits (bounded
// spin) until its system's alpha is published.  Every item it waits for was claimed earlier
// by a running workgroup that itself never waits, so the launch cannot deadlock whatever
// the number of resident workgroups.  The last workgroup to leave resets the counters and
// advances the launch epoch, so consecutive launches (captured in a hipGraph) need no host
// work in between.  Epochs start at 1 (the control block is zeroed once per batch), so a
// zeroed alpha_epoch[] never reads as published.
#include "zmarch.hpp"

namespace excmg {

constexpr int kSpinLimit = 1 << 26;   // bounded wait; exceeding it sets ctl->error

__device__ __forceinline__ Pair load_pair_coherent(const Pair *p) {
    Pair v;
    v.s = __hip_atomic_load(&p->s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v.c = __hip_atomic_load(&p->c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return v;
}

// Merge count pairs (NV interleaved arrays of `count`) written by other workgroups.
template <int NV>
__device__ void merge_remote(const Pair *part, int count, Pair (&out)[NV], Pair *sh) {
    for (int q = 0; q < NV; q++) out[q] = Pair{0.0, 0.0};
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nt = blockDim.x * blockDim.y;
    for (int i = tid; i < count; i += nt) {
#pragma unroll
        for (int q = 0; q < NV; q++) out[q] = pair_merge(out[q], load_pair_coherent(&part[q * count + i]));
    }
    block_merge<NV>(out, sh);
}

template <typename T, int TY>
__device__ void sweep_a_item(const BatchRun &R, int run, int tile, BatchCtl *ctl, int epoch,
                             Pair *red) {
    __shared__ int sh_last;
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    BicgState *S = R.state;
    const int status = __hip_atomic_load(&S->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int iter = __hip_atomic_load(&S->iter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int cur = iter & 1;
    OutPairApply<T> out;
    out.p_new[0] = (T *)R.p[cur ^ 1];
    out.p_new[1] = (T *)R.ps[cur ^ 1];
    out.q[0] = (T *)R.q;
    out.q[1] = (T *)R.qs;
    out.partials = R.part_a;
    out.status = &S->status;
    out.acc = Pair{0.0, 0.0};
    if (status == kRunning) {
        InDirection<T> in;
        in.r[0] = (const T *)R.r;
        in.r[1] = (const T *)R.rs;
        in.p[0] = (const T *)R.p[cur];
        in.p[1] = (const T *)R.ps[cur];
        in.beta_dev = &S->beta;
        in.first = (iter == 0);
        in.prepare();
        zmarch_tile<2, TY, T>(R.g, tile, in, out);
    }
    __threadfence();  // every thread releases its p, p*, q, q* stores before the arrival count
    Pair v[1] = {out.acc};
    block_merge<1>(v, red);
    if (tid == 0) {
        R.part_a[tile] = v[0];
        __threadfence();
        const int c = atomicAdd(&ctl->a_done[run], 1);
        sh_last = (c == R.a_count - 1);
    }
    __syncthreads();
    if (sh_last) {  // all sweep-A tiles of this system are done: alpha = rho / sigma
        __threadfence();
        Pair m[1];
        merge_remote<1>(R.part_a, R.a_count, m, red);
        if (tid == 0) {
            if (S->status == kRunning) {
                const double sigma = pair_value(m[0]);
                S->sigma = sigma;
                if (sigma == 0.0 || !isfinite(sigma)) S->status = kBreakdown;
                else S->alpha = S->rho / sigma;
            }
            __threadfence();
            __hip_atomic_store(&ctl->alpha_epoch[run], epoch, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
}

template <typename T>
__device__ void sweep_b_item(const BatchRun &R, int run, int chunk, BatchCtl *ctl, int epoch,
                             Pair *red) {
    __shared__ int sh_last;
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nt = blockDim.x * blockDim.y;
    if (tid == 0) {
        int spins = 0;
        while (__hip_atomic_load(&ctl->alpha_epoch[run], __ATOMIC_ACQUIRE,
                                 __HIP_MEMORY_SCOPE_AGENT) != epoch) {
            __builtin_amdgcn_s_sleep(4);
            if (++spins > kSpinLimit) {
                atomicExch(&ctl->error, 1);
                break;
            }
        }
    }
    __syncthreads();
    __threadfence();
    BicgState *S = R.state;
    const int status = __hip_atomic_load(&S->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double alpha = __hip_atomic_load(&S->alpha, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int cur = __hip_atomic_load(&S->iter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1;
    Pair acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    if (status == kRunning) {
        const long long i0 = (long long)chunk * R.chunk;
        const long long i1 = min(R.nu, i0 + R.chunk);
        const T *p = (const T *)R.p[cur ^ 1];
        const T *q = (const T *)R.q;
        const T *qs = (const T *)R.qs;
        T *r = (T *)R.r;
        T *rs = (T *)R.rs;
        double *x = R.x;
        for (long long i = i0 + tid; i < i1; i += nt) {
            double xi = x[i] + alpha * (double)p[i];
            double ri = (double)r[i] - alpha * (double)q[i];
            double si = (double)rs[i] - alpha * (double)qs[i];
            T rt = (T)ri, st = (T)si;
            x[i] = xi;
            r[i] = rt;
            rs[i] = st;
            dot2_acc(acc[0], (double)st, (double)rt);
            dot2_acc(acc[1], (double)rt, (double)rt);
        }
    }
    __threadfence();  // release this chunk's x, r, r* stores before the arrival count
    block_merge<2>(acc, red);
    if (tid == 0) {
        R.part_b[chunk] = acc[0];
        R.part_b[R.b_count + chunk] = acc[1];
        __threadfence();
        const int c = atomicAdd(&ctl->b_done[run], 1);
        sh_last = (c == R.b_count - 1);
    }
    __syncthreads();
    if (sh_last) {  // all chunks done: rho', r.r, beta and the stopping test
        __threadfence();
        Pair m[2];
        merge_remote<2>(R.part_b, R.b_count, m, red);
        if (tid == 0 && S->status == kRunning) {
            const double rho_new = pair_value(m[0]);
            S->rr = pair_value(m[1]);
            S->beta = rho_new / S->rho;
            S->rho_slot[1] = S->rho;   // rho of the previous iteration (residual replacement)
            S->rho = rho_new;
            S->iter = S->iter + 1;
            if (S->rr <= S->thr) S->status = kConverged;
            else if (S->iter >= S->maxit) S->status = kNoConv;
            else if (S->rho == 0.0 || !isfinite(S->rho)) S->status = kBreakdown;
        }
    }
    __syncthreads();
}

template <typename T, int TY>
__global__ void __launch_bounds__(kWave *TY)
    k_batch_step(const BatchRun *runs, const int2 *items, BatchCtl *ctl) {
    __shared__ int sh_item, sh_epoch;
    __shared__ Pair red[2 * TY];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    if (tid == 0) sh_epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int epoch = sh_epoch;
    const int n_a = ctl->n_a, n_items = ctl->n_items;
    for (;;) {
        if (tid == 0) sh_item = atomicAdd(&ctl->queue, 1);
        __syncthreads();
        const int it = sh_item;
        __syncthreads();
        if (it >= n_items) break;
        const int2 item = items[it];
        const BatchRun &R = runs[item.x];
        if (it < n_a) sweep_a_item<T, TY>(R, item.x, item.y, ctl, epoch, red);
        else sweep_b_item<T>(R, item.x, item.y, ctl, epoch, red);
    }
    if (tid == 0) {
        __threadfence();
        const int c = atomicAdd(&ctl->exit_count, 1);
        if (c == (int)(gridDim.x * gridDim.y * gridDim.z) - 1) {  // last workgroup out
            ctl->queue = 0;
            for (int r = 0; r < ctl->n_runs; r++) {
                ctl->a_done[r] = 0;
                ctl->b_done[r] = 0;
            }
            ctl->exit_count = 0;
            __threadfence();
            __hip_atomic_store(&ctl->epoch, epoch + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------------------ phase kernels

constexpr int kPhaseGridA = 2048, kPhaseGridB = 2048, kPhaseGridR = kMaxRuns;

template <typename T, int TY>
__global__ void __launch_bounds__(kWave *TY)
    k_phase_sweep_a(const BatchRun *runs, const int2 *items, const BatchCtl *ctl) {
    __shared__ Pair red[TY];
    const int n_a = ctl->n_a;
    for (int it = blockIdx.x; it < n_a; it += gridDim.x) {
        const int2 item = items[it];
        const BatchRun &R = runs[item.x];
        BicgState *S = R.state;
        if (S->status != kRunning) continue;  // uniform per workgroup
        const int iter = S->iter;
        const int cur = iter & 1;
        OutPairApply<T> out;
        out.p_new[0] = (T *)R.p[cur ^ 1];
        out.p_new[1] = (T *)R.ps[cur ^ 1];
        out.q[0] = (T *)R.q;
        out.q[1] = (T *)R.qs;
        out.partials = R.part_a;
        out.status = &S->status;
        out.acc = Pair{0.0, 0.0};
        InDirection<T> in;
        in.r[0] = (const T *)R.r;
        in.r[1] = (const T *)R.rs;
        in.p[0] = (const T *)R.p[cur];
        in.p[1] = (const T *)R.ps[cur];
        in.beta_dev = &S->beta;
        in.first = (iter == 0);
        in.prepare();
        zmarch_tile<2, TY, T>(R.g, item.y, in, out);
        Pair v[1] = {out.acc};
        block_merge<1>(v, red);
        if (threadIdx.x == 0 && threadIdx.y == 0) R.part_a[item.y] = v[0];
    }
}

__global__ void __launch_bounds__(kReduceThreads)
    k_phase_alpha(const BatchRun *runs, const BatchCtl *ctl) {
    __shared__ Pair sh[kReduceThreads / kWave];
    const int na = ctl->n_active;
    for (int k = blockIdx.x; k < na; k += gridDim.x) {
        const BatchRun &R = runs[ctl->active[k]];
        BicgState *S = R.state;
        if (S->status != kRunning) continue;
        Pair v[1] = {{0.0, 0.0}};
        for (int i = threadIdx.x; i < R.a_count; i += blockDim.x) v[0] = pair_merge(v[0], R.part_a[i]);
        block_merge<1>(v, sh);
        if (threadIdx.x == 0) {
            const double sigma = pair_value(v[0]);
            S->sigma = sigma;
            if (sigma == 0.0 || !isfinite(sigma)) S->status = kBreakdown;
            else S->alpha = S->rho / sigma;
        }
    }
}

template <typename T, int TY>
__global__ void __launch_bounds__(kWave *TY)
    k_phase_sweep_b(const BatchRun *runs, const int2 *items, const BatchCtl *ctl) {
    __shared__ Pair red[2 * TY];
    const int n_a = ctl->n_a, n_b = ctl->n_items - ctl->n_a;
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nt = blockDim.x * blockDim.y;
    for (int it = blockIdx.x; it < n_b; it += gridDim.x) {
        const int2 item = items[n_a + it];
        const BatchRun &R = runs[item.x];
        BicgState *S = R.state;
        if (S->status != kRunning) continue;
        const double alpha = S->alpha;
        const int cur = S->iter & 1;
        const long long i0 = (long long)item.y * R.chunk;
        const long long i1 = min(R.nu, i0 + R.chunk);
        const T *p = (const T *)R.p[cur ^ 1];
        const T *q = (const T *)R.q;
        const T *qs = (const T *)R.qs;
        T *r = (T *)R.r;
        T *rs = (T *)R.rs;
        double *x = R.x;
        Pair acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
        for (long long i = i0 + tid; i < i1; i += nt) {
            double xi = x[i] + alpha * (double)p[i];
            double ri = (double)r[i] - alpha * (double)q[i];
            double si = (double)rs[i] - alpha * (double)qs[i];
            T rt = (T)ri, st = (T)si;
            x[i] = xi;
            r[i] = rt;
            rs[i] = st;
            dot2_acc(acc[0], (double)st, (double)rt);
            dot2_acc(acc[1], (double)rt, (double)rt);
        }
        block_merge<2>(acc, red);
        if (tid == 0) {
            R.part_b[item.y] = acc[0];
            R.part_b[R.b_count + item.y] = acc[1];
        }
    }
}

__global__ void __launch_bounds__(kReduceThreads)
    k_phase_beta(const BatchRun *runs, const BatchCtl *ctl) {
    __shared__ Pair sh[2 * (kReduceThreads / kWave)];
    const int na = ctl->n_active;
    for (int k = blockIdx.x; k < na; k += gridDim.x) {
        const BatchRun &R = runs[ctl->active[k]];
        BicgState *S = R.state;
        if (S->status != kRunning) continue;
        Pair v[2] = {{0.0, 0.0}, {0.0, 0.0}};
        for (int i = threadIdx.x; i < R.b_count; i += blockDim.x) {
            v[0] = pair_merge(v[0], R.part_b[i]);
            v[1] = pair_merge(v[1], R.part_b[R.b_count + i]);
        }
        block_merge<2>(v, sh);
        if (threadIdx.x == 0) {
            const double rho_new = pair_value(v[0]);
            S->rr = pair_value(v[1]);
            S->beta = rho_new / S->rho;
            S->rho_slot[1] = S->rho;   // rho of the previous iteration (residual replacement)
            S->rho = rho_new;
            S->iter = S->iter + 1;
            if (S->rr <= S->thr) S->status = kConverged;
            else if (S->iter >= S->maxit) S->status = kNoConv;
            else if (S->rho == 0.0 || !isfinite(S->rho)) S->status = kBreakdown;
        }
    }
}

// Residual replacement of a stopped FP32 run: r and r* already hold the FP64 residual of the
// iterate (rounded to FP32); rho = r*.r from their partials, beta = rho / rho of the
// previous iteration (so the next direction is formed from the new residual with the old
// search direction), a new stopping threshold, and the run goes on from its iteration count
// (which keeps the direction buffers' parity).
__global__ void __launch_bounds__(kReduceThreads)
    k_batch_resume(BicgState *s, const Pair *part, int count, double thr) {
    __shared__ Pair sh[kReduceThreads / kWave];
    Pair v[1] = {{0.0, 0.0}};
    for (int i = threadIdx.x; i < count; i += blockDim.x) v[0] = pair_merge(v[0], part[i]);
    block_merge<1>(v, sh);
    if (threadIdx.x == 0) {
        const double rho = pair_value(v[0]);
        s->beta = rho / s->rho_slot[1];
        s->rho = rho;
        s->rr = rho;
        s->thr = thr;
        if (s->iter >= s->maxit) s->status = kNoConv;
        else if (rho == 0.0 || !isfinite(rho) || !isfinite(s->beta)) s->status = kBreakdown;
        else s->status = kRunning;
        s->poll_status = s->status;
    }
}

hipError_t batch_resume(BicgState *s, const Pair *part, int count, double thr, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_resume, dim3(1), dim3(kReduceThreads), 0, st, s, part, count, thr);
    return hipGetLastError();
}

template <typename T, int TY>
static hipError_t phases(const BatchRun *runs, const int2 *items, const BatchCtl *ctl,
                         hipStream_t st) {
    hipLaunchKernelGGL((k_phase_sweep_a<T, TY>), dim3(kPhaseGridA), dim3(kWave, TY), 0, st, runs,
                       items, ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_phase_alpha, dim3(kPhaseGridR), dim3(kReduceThreads), 0, st, runs, ctl);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_phase_sweep_b<T, TY>), dim3(kPhaseGridB), dim3(kWave, TY), 0, st, runs,
                       items, ctl);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_phase_beta, dim3(kPhaseGridR), dim3(kReduceThreads), 0, st, runs, ctl);
    return hipGetLastError();
}

template <typename T>
hipError_t batch_step_phases(int ty, const BatchRun *runs, const int2 *items, const BatchCtl *ctl,
                             hipStream_t st) {
    switch (ty) {
        case 4: return phases<T, 4>(runs, items, ctl, st);
        case 8: return phases<T, 8>(runs, items, ctl, st);
        default: return hipErrorInvalidValue;
    }
}
template hipError_t batch_step_phases<double>(int, const BatchRun *, const int2 *,
                                              const BatchCtl *, hipStream_t);
template hipError_t batch_step_phases<float>(int, const BatchRun *, const int2 *,
                                             const BatchCtl *, hipStream_t);

// ------------------------------------------------------------------ persistent kernel

template <typename T>
hipError_t batch_step(int ty, int grid, const BatchRun *runs, const int2 *items, BatchCtl *ctl,
                      hipStream_t st) {
    switch (ty) {
        case 4:
            hipLaunchKernelGGL((k_batch_step<T, 4>), dim3(grid), dim3(kWave, 4), 0, st, runs,
                               items, ctl);
            break;
        case 8:
            hipLaunchKernelGGL((k_batch_step<T, 8>), dim3(grid), dim3(kWave, 8), 0, st, runs,
                               items, ctl);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t batch_step<double>(int, int, const BatchRun *, const int2 *, BatchCtl *,
                                       hipStream_t);
template hipError_t batch_step<float>(int, int, const BatchRun *, const int2 *, BatchCtl *,
                                      hipStream_t);

template <typename T>
hipError_t batch_step_grid(int ty, int *grid) {
    int per_cu = 0;
    hipError_t e = ty == 4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_step<T, 4>,
                                                                         kWave * 4, 0)
                 : ty == 8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_step<T, 8>,
                                                                         kWave * 8, 0)
                           : hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    *grid = (per_cu > 0 ? per_cu : 1) * cus;
    return hipSuccess;
}
template hipError_t batch_step_grid<double>(int, int *);
template hipError_t batch_step_grid<float>(int, int *);

}  // namespace excmg
