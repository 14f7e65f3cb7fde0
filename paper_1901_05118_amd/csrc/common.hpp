// Shared device helpers of the EXCMG library (gfx950, wave64).
//
// Arithmetic conventions, fixed for the whole library (compiled with -ffp-contract=off):
//  * the 25-point sum of eq. (method1) is evaluated left to right in the printed order;
//  * inner products use the compensated Dot2 algorithm (Ogita, Rump & Oishi, SIAM J. Sci.
//    Comput. 26(6), 2005): every thread keeps a (sum, compensation) pair, pairs are merged
//    with an error-free TwoSum, and the result is rounded once;
//  * reductions combine partials in a fixed order, so every result is run-to-run
//    deterministic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace excmg {

typedef long long i64;

constexpr int kWave = 64;
constexpr int kNumXcd = 8;        // MI355X: 8 accelerator complex dies, 32 CUs each
constexpr int kReduceThreads = 256;

// ------------------------------------------------------------------ Dot2 pairs

struct Pair {
    double s, c;
};

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    double x = a + b;
    double z = x - a;
    e = (a - (x - z)) + (b - z);
    s = x;
}

// acc += a*b with the product's rounding error and the sum's rounding error carried in c
__device__ __forceinline__ void dot2_acc(Pair &acc, double a, double b) {
    double p = a * b;
    double pe = __builtin_fma(a, b, -p);
    double t, e;
    two_sum(acc.s, p, t, e);
    acc.s = t;
    acc.c = acc.c + (pe + e);
}

__device__ __forceinline__ Pair pair_merge(Pair x, Pair y) {
    Pair r;
    double e;
    two_sum(x.s, y.s, r.s, e);
    r.c = (x.c + y.c) + e;
    return r;
}

__device__ __forceinline__ double pair_value(Pair p) { return p.s + p.c; }

// Wave-level merge with a fixed butterfly.  pair_merge is commutative bit for bit (TwoSum
// returns the same rounded sum and the same exact error for either operand order), so
// every lane ends with the same pair.
__device__ __forceinline__ Pair wave_merge(Pair v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Pair o;
        o.s = __shfl_xor(v.s, off, kWave);
        o.c = __shfl_xor(v.c, off, kWave);
        v = pair_merge(v, o);
    }
    return v;
}

// Block-level merge of NV independent pairs; results valid in thread 0.  `sh` needs
// NV * (blockDim / 64) pairs of LDS.  Ends with a barrier, so `sh` can be reused.
template <int NV>
__device__ __forceinline__ void block_merge(Pair (&v)[NV], Pair *sh) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x + threadIdx.z * blockDim.x * blockDim.y;
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    const int nwaves = (nthreads + kWave - 1) / kWave;
    const int wave = tid / kWave, lane = tid % kWave;
#pragma unroll
    for (int q = 0; q < NV; q++) v[q] = wave_merge(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; q++) sh[q * nwaves + wave] = v[q];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NV; q++) {
            Pair a = sh[q * nwaves];
            for (int w = 1; w < nwaves; w++) a = pair_merge(a, sh[q * nwaves + w]);
            v[q] = a;
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------ XCD-aware tile order

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b % 8).
// Give each XCD a contiguous range of tiles so that tiles sharing halos share an L2.
__device__ __forceinline__ int xcd_tile(int block, int ntiles) {
    int per = (ntiles + kNumXcd - 1) / kNumXcd;
    return (block % kNumXcd) * per + block / kNumXcd;
}

inline int xcd_grid(int ntiles) {
    int per = (ntiles + kNumXcd - 1) / kNumXcd;
    return per * kNumXcd;
}

}  // namespace excmg
