// The 13-point scheme of the 2D biharmonic equation (eq. bvp2d) on the GPU: the operator is
// the square of the 5-point Laplacian, as eq. (method1) is the square of the 7-point one,
//   h^4 (Delta^2 u)_ij ~ 20 u - 8 (x-, x+, y-, y+) + (x-2, x+2, y-2, y+2)
//                        + 2 (x-y-, x-y+, x+y-, x+y+),
// each group summed left to right in this order.  Fictitious points one step outside an edge
// come from the reflection of eq. (reflection2) / (reflection4) along the edge normal, exactly
// as on a face in 3D.  A workgroup stages one 64 x TY tile of every input array with a
// 2-wide halo in LDS (through the same input policies as the z-march: direction updates,
// preconditioning) and evaluates the scheme once per point; the epilogues are those of the
// z-march (centre() and emit() per point, then the block reduction).
#pragma once

#include "zmarch.hpp"

namespace excmg {

// One tile; `begin()` prepares `in` after the tile's loads have been issued (see
// zmarch_tile).  Returns false (nothing written) when begin() ends the run.
template <int NA, int TY, typename T, class In, class Out, class Begin>
__device__ __forceinline__ bool plane_tile(const Geom &g, int tile, const In &in, Out &out,
                                           Begin begin) {
    constexpr int TX = kWave;
    constexpr int LS = TX + 4;
    constexpr int LR = TY + 4;
    constexpr int LE = LS * LR;
    constexpr int NT = TX * TY;
    constexpr int NL = (LE + NT - 1) / NT;
    constexpr int R = In::R;
    __shared__ T buf[NA][LE];
    const int n = g.n;
    const int tx = tile % g.tiles_x;
    const int ty = tile / g.tiles_x;
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = ly * TX + lx;
    const int ix = tx * TX + lx, iy = ty * TY + ly;
    // every staged element is requested first (positions outside the grid read a valid
    // clamped element and are multiplied by 0)
    T raw[NL][NA][R];
    double mul[NL];
#pragma unroll
    for (int q = 0; q < NL; q++) {
        const int e = min(tid + q * NT, LE - 1);
        const int row = e / LS, col = e % LS;
        int sx, sy;
        const double mx = reflect(tx * TX + col - 2, n, g.sgn, sx);
        const double my = reflect(ty * TY + row - 2, n, g.sgn, sy);
        mul[q] = mx * my;
        const i64 idx = (i64)sy * n + sx;
#pragma unroll
        for (int a = 0; a < NA; a++) in.load(a, idx, raw[q][a]);
    }
    if (!begin()) return false;
#pragma unroll
    for (int q = 0; q < NL; q++) {
        const int e = tid + q * NT;
        if (e < LE) {
#pragma unroll
            for (int a = 0; a < NA; a++) {
                const double v = in.combine(raw[q][a]);
                buf[a][e] = (T)((mul[q] != 0.0) ? mul[q] * v : 0.0);
            }
        }
    }
    __syncthreads();
    if (ix < n && iy < n) {
        const int centre = (ly + 2) * LS + (lx + 2);
        double y[NA], c0[NA];
#pragma unroll
        for (int a = 0; a < NA; a++) {
            const T *B = &buf[a][centre];
            const double c = B[0];
            const double S1 = (double)B[-1] + (double)B[1] + (double)B[-LS] + (double)B[LS];
            const double S2 = (double)B[-2] + (double)B[2] + (double)B[-2 * LS] + (double)B[2 * LS];
            const double S3 = (double)B[-1 - LS] + (double)B[-1 + LS] + (double)B[1 - LS] +
                              (double)B[1 + LS];
            y[a] = 20.0 * c - 8.0 * S1 + S2 + 2.0 * S3;
            c0[a] = c;
        }
        const i64 idx = (i64)iy * n + ix;
        out.centre(idx, c0);
        if constexpr (HasPre<Out>::value) out.emit(idx, y, c0, out.pre(idx));
        else out.emit(idx, y, c0);
    }
    return true;
}

template <int NA, int TY, typename T, class In, class Out>
__global__ void __launch_bounds__(kWave *TY) plane2d(Geom g, In in_arg, Out out) {
    __shared__ Pair red[4 * TY];
    __shared__ int s_skip;
    In in = in_arg;
    auto start = [&]() {    // status, then scalars, once the tile's loads are in flight
        if (threadIdx.x == 0 && threadIdx.y == 0) s_skip = out.skip() ? 1 : 0;
        __syncthreads();
        if (s_skip) return false;
        return in.begin(red);
    };
    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const bool go = tile < g.ntiles ? plane_tile<NA, TY, T>(g, tile, in, out, start) : start();
    if (!go) return;
    __syncthreads();
    out.finish(blockIdx.x, red);
}

}  // namespace excmg
