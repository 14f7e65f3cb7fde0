// Finalisations of a Bi-CG step folded into the sweeps (device code).
//
// Algorithm 2 needs two global reductions per iteration: sigma = p*.A p before the updates
// and rho' = r*.r (with r.r for the stopping test) before the next direction.  Instead of a
// one-workgroup kernel after each sweep, every workgroup of the following sweep merges the
// previous sweep's partials itself, in one fixed order (that of a 256-thread merge), so all
// workgroups obtain the same scalars bit for bit and take the same decision; workgroup 0
// publishes them in the state.  rho is kept in two slots by iteration parity, so the sweep
// that computes rho_j never overwrites rho_{j-1} while other workgroups still read it.
#pragma once

#include "common.hpp"
#include "internal.hpp"

namespace excmg {

__device__ __forceinline__ int block_tid() {
    return threadIdx.x + threadIdx.y * blockDim.x + threadIdx.z * blockDim.x * blockDim.y;
}

// A value that every lane of the wave holds, moved to scalar registers (frees two vector
// registers in the march that follows).
__device__ __forceinline__ double wave_uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Merge NV interleaved sets of `count` pairs in the order of a kReduceThreads-thread block
// (strided per thread, butterfly per wave, waves in order).  Any block shape of at least
// kReduceThreads threads; the result is returned to every thread.  `sh` needs 4 * NV pairs.
template <int NV>
__device__ void merge_fixed(const Pair *part, int count, Pair (&out)[NV], Pair *sh) {
    constexpr int W = kReduceThreads / kWave;
    const int tid = block_tid();
    Pair v[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) v[q] = Pair{0.0, 0.0};
    if (tid < kReduceThreads) {
#pragma nounroll
        for (int i = tid; i < count; i += kReduceThreads) {
#pragma unroll
            for (int q = 0; q < NV; q++) v[q] = pair_merge(v[q], part[q * count + i]);
        }
    }
#pragma unroll
    for (int q = 0; q < NV; q++) v[q] = wave_merge(v[q]);
    if (tid < kReduceThreads && (tid % kWave) == 0) {
#pragma unroll
        for (int q = 0; q < NV; q++) sh[q * W + tid / kWave] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; q++) {
        Pair a = sh[q * W];
        for (int w = 1; w < W; w++) a = pair_merge(a, sh[q * W + w]);
        out[q] = a;
    }
    __syncthreads();
}

// End of iteration j-1, at the start of sweep A of iteration j (parity par = j & 1): rho_j
// and r.r from the partials of the previous sweep B, the stopping checks in the order of
// the loop (residual, iteration cap, breakdown), beta_{j-1} = rho_j / rho_{j-1}.  Returns
// true while the run goes on.
__device__ __forceinline__ bool link_step(const StepLink &L, double &beta, Pair *sh) {
    BicgState *s = L.state;
    // state fields of the previous launches, requested before the merge waits on memory
    const double thr = s->thr, rho_old = s->rho_slot[L.par ^ 1];
    const int iter = s->iter, maxit = s->maxit, prev_st = s->poll_status;
    Pair v[2];
    if (L.nv == 2) {
        merge_fixed<2>(L.part, L.count, v, sh);
    } else {
        Pair w[1];
        merge_fixed<1>(L.part, L.count, w, sh);
        v[0] = w[0];
        v[1] = w[0];
    }
    const double rho_new = pair_value(v[0]);
    const double rr = pair_value(v[1]);
    int st;
    // a breakdown of the preceding sweep B that owed the iterate's update comes first
    if (prev_st == kBreakdown) st = kBreakdown;
    else if (rr <= thr) st = kConverged;
    else if (iter >= maxit) st = kNoConv;
    else if (rho_new == 0.0 || !isfinite(rho_new)) st = kBreakdown;
    else st = kRunning;
    beta = wave_uniform(rho_new / rho_old);
    if (blockIdx.x == 0 && block_tid() == 0) {
        s->rr = rr;
        s->beta = beta;
        s->rho = rho_new;
        s->rho_slot[L.par] = rho_new;
        s->poll_status = st;
        // a poll-only check leaves the run going: the next sweep A takes the same decision
        // and applies the iterate's pending update before it stops
        if (!L.poll_only) s->status = (L.defer && st != kRunning) ? kStopping : st;
    }
    return st == kRunning;
}

// Start of sweep B of iteration j: sigma from the partials of sweep A, alpha_j =
// rho_j / sigma.  Counts the iteration.  Returns false on breakdown.
__device__ __forceinline__ bool link_alpha(const StepLink &L, double &alpha, Pair *sh) {
    BicgState *s = L.state;
    const double rho = s->rho_slot[L.par];   // requested before the merge waits on memory
    Pair v[1];
    merge_fixed<1>(L.part, L.count, v, sh);
    const double sigma = pair_value(v[0]);
    const bool bad = (sigma == 0.0 || !isfinite(sigma));
    alpha = wave_uniform(bad ? 0.0 : rho / sigma);
    if (blockIdx.x == 0 && block_tid() == 0) {
        s->sigma = sigma;
        if (bad) {
            // with an update owed, the status stays running until the next check, so the
            // workgroups that start later take the same decision and apply their part
            if (!L.defer) s->status = kBreakdown;
            s->poll_status = kBreakdown;
        } else {
            s->alpha = alpha;
            s->alpha_slot[L.par] = alpha;
            s->iter = s->iter + 1;
        }
    }
    return !bad;
}

// Is the run still going?  Read once per workgroup: inside a fused sweep, workgroup 0 may
// publish a new status while other workgroups start, and all threads of a workgroup must
// take the same branch.
__device__ __forceinline__ bool block_running(const int *status) {
    __shared__ int s_run;
    if (block_tid() == 0) s_run = (*status == kRunning) ? 1 : 0;
    __syncthreads();
    return s_run != 0;
}

}  // namespace excmg
