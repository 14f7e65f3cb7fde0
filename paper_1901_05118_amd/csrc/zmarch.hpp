// Matrix-free 25-point operator A_h of Sec. 2 on interior vectors, for gfx950: the device code
// shared by the single-system kernels (stencil.hip) and the batched persistent kernel
// (batch.hip).
//
// Design (one kernel template, several epilogues):
//  * A workgroup owns a 64 x TY column tile of the (n = N-1)^2 plane and marches through a
//    chunk of ZC planes in z.  Each plane is staged once in LDS with a 2-wide halo in x and
//    y (double-buffered, so one barrier per plane); the next plane's global loads are issued
//    before the current plane is consumed, which hides HBM latency behind the LDS work.
//  * Every lane keeps the z-direction terms of its column in registers: the centre values
//    of the last two planes, the sum of the previous plane's four axis neighbours and the
//    partial sums of the two outputs that are still open, each term added as soon as its
//    plane is consumed (a two-deep pipeline, so an unroll by two renames it for free).  An
//    output on plane k is complete when plane k+2 arrives.
//  * Every global load of the march belongs to one pipeline: a stage holds the raw values
//    of one staged plane and the per-output data (e.g. the iterate of an update sweep) of
//    the output that is complete when that plane is staged, and is consumed D planes after
//    it was requested.  The planes are marched in whole groups of D with no exit inside a
//    group, so the compiler keeps D planes of loads in flight (a load consumed in the plane
//    it is requested in, or a loop path that skips a group's loads, makes it wait for every
//    load in flight).
//  * The left-hand side of eq. (method1) is summed in the order the paper prints it, with
//    contraction off; the twelve terms of the factor 2 are summed per printed group of four
//    (in-plane diagonals, then plane k-1, then plane k+1) and the three group sums left to
//    right:
//      y = 42 c - 12 S1 + S2 + 2 S3,
//      S1 = x- + x+ + y- + y+ + z- + z+,   S2 = the same at distance 2,
//      S3 = [(x-y-) + (x-y+) + (x+y-) + (x+y+)] + [x- + x+ + y- + y+ on plane k-1]
//           + [x- + x+ + y- + y+ on plane k+1].
//  * Fictitious points (eqs. reflection2 / reflection4 with zero boundary data) are produced
//    while staging: a halo position one step outside the boundary node holds +x (first kind)
//    or -x (second kind) of the mirrored interior node, a boundary node holds 0.  The
//    resulting operator is exactly the paper's A_h, including its boundary rows, with no
//    per-row branches in the arithmetic.
//  * Tiles are ordered XCD-aware: each of the 8 XCDs processes a contiguous range of tiles.
//  * Rows of the vectors are Geom::ld elements apart (n: contiguous).  With padded rows
//    (an option of the mixed-precision solver) every row starts on a cache line, so no
//    128-byte line is split between the row segments of two tiles.
#pragma once

#include <type_traits>
#include <utility>

#include "common.hpp"
#include "internal.hpp"
#include "step.hpp"

namespace excmg {

// Where a staged coordinate comes from: multiplier 1 (interior), sgn (fictitious point,
// mirrored source) or 0 (boundary node or beyond the grid).
__device__ __forceinline__ double reflect(int c, int n, double sgn, int &src) {
    if (c >= 0 && c < n) {
        src = c;
        return 1.0;
    }
    if (c == -2) {
        src = 0;
        return sgn;
    }
    if (c == n + 1) {
        src = n - 1;
        return sgn;
    }
    src = 0;
    return 0.0;
}

// Per-column register state of one marched array.  Each term of an output is added as
// soon as its plane has been consumed, in the order of eq. (method1); the state is a
// two-deep pipeline: output k = m-2 (completed by plane m) and output j = m-1.
struct Column {
    double c1, c2;               // centre values of planes m-1, m-2
    double ap;                   // x- + x+ + y- + y+ of plane m-1
    double s1k, s1j;             // S1 of output k (complete); of output j (without z+)
    double s2k, s2j;             // S2 of outputs k and j without their z+2 term
    double ek, ej;               // S3 of output k (complete); of output j (without plane j+1)
};

__device__ __forceinline__ void column_init(Column &s) {
    s.c1 = s.c2 = s.ap = 0.0;
    s.s1k = s.s1j = s.s2k = s.s2j = s.ek = s.ej = 0.0;
}

// Consume plane m from LDS (row stride LS, centre at B) and return the completed output of
// plane m-2.  `c0` receives the centre value of plane m.
template <int LS, typename TL>
__device__ __forceinline__ double column_step(Column &s, const TL *B, double &c0) {
    const double c = B[0];
    const double n0 = B[-1], n1 = B[1], n2 = B[-LS], n3 = B[LS];
    const double f0 = B[-2], f1 = B[2], f2 = B[-2 * LS], f3 = B[2 * LS];
    const double d0 = B[-1 - LS], d1 = B[-1 + LS], d2 = B[1 - LS], d3 = B[1 + LS];
    // output m-2 is complete once its S2 has this plane's centre (z+2)
    const double y = 42.0 * s.c2 - 12.0 * s.s1k + (s.s2k + c) + 2.0 * s.ek;
    const double a0 = n0 + n1 + n2 + n3;
    // output m-1 receives z+ (S1) and its plane k+1 group (S3)
    const double s1 = s.s1j + c;
    const double e1 = s.ej + a0;
    // output m opens with the terms of planes m, m-1 and m-2 that are already known
    const double b0 = f0 + f1 + f2 + f3;
    const double e0 = (d0 + d1 + d2 + d3) + s.ap;
    s.s1k = s1;
    s.s1j = a0 + s.c1;
    s.s2k = s.s2j;
    s.s2j = b0 + s.c2;
    s.ek = e1;
    s.ej = e0;
    s.c2 = s.c1;
    s.c1 = c;
    s.ap = a0;
    c0 = c;
    return y;
}

// The same pipeline for a march towards decreasing z (planes m+2, m+1, m, ... arrive in that
// order).  Every output is summed with the association of the upward pipeline, term by term
// (the z-2 centre still joins S2 first and the z+2 one last), so both directions give the
// same value bit for bit; the down pipeline holds one plane more of history for that.
struct ColumnDown {
    double c1, c2, c3, c4;       // centre values of planes m+1 .. m+4
    double a1, a2;               // x- + x+ + y- + y+ of planes m+1, m+2
    double d1;                   // the diagonal group of plane m+1
    double b1, b2;               // the distance-2 group of planes m+1, m+2
    double s1, e;                // S1 and S3 of output m+2 (complete)
};

__device__ __forceinline__ void column_init(ColumnDown &s) {
    s.c1 = s.c2 = s.c3 = s.c4 = 0.0;
    s.a1 = s.a2 = s.d1 = s.b1 = s.b2 = s.s1 = s.e = 0.0;
}

// Consume plane m and return the completed output of plane m+2.
template <int LS, typename TL>
__device__ __forceinline__ double column_step(ColumnDown &s, const TL *B, double &c0) {
    const double c = B[0];
    const double n0 = B[-1], n1 = B[1], n2 = B[-LS], n3 = B[LS];
    const double f0 = B[-2], f1 = B[2], f2 = B[-2 * LS], f3 = B[2 * LS];
    const double d0 = B[-1 - LS], d1 = B[-1 + LS], d2 = B[1 - LS], d3 = B[1 + LS];
    const double a0 = n0 + n1 + n2 + n3;
    const double b0 = f0 + f1 + f2 + f3;
    const double dg = d0 + d1 + d2 + d3;
    // output m+2: S2 = (its distance-2 group + this plane's centre) + the centre of m+4
    const double y = 42.0 * s.c2 - 12.0 * s.s1 + ((s.b2 + c) + s.c4) + 2.0 * s.e;
    // output m+1: S1 and S3 complete with this plane (its z-1 terms)
    const double s1 = (s.a1 + c) + s.c2;
    const double e1 = (s.d1 + a0) + s.a2;
    s.c4 = s.c3;
    s.c3 = s.c2;
    s.c2 = s.c1;
    s.c1 = c;
    s.a2 = s.a1;
    s.a1 = a0;
    s.d1 = dg;
    s.b2 = s.b1;
    s.b1 = b0;
    s.s1 = s1;
    s.e = e1;
    c0 = c;
    return y;
}

// Inputs of the marched arrays.  Staging is split in two so that global loads stay in
// flight while earlier planes are consumed: load() fetches the R raw values of a staged
// element (into registers, no arithmetic), combine() turns them into the staged value.
// prepare() runs once per thread before the march.
template <typename T>
struct InPlain {            // x itself
    static constexpr int R = 1;
    const T *x[2];
    __device__ __forceinline__ void prepare() {}
    __device__ __forceinline__ bool begin(Pair *) { return true; }
    __device__ __forceinline__ void load(int a, i64 idx, T (&raw)[R]) const { raw[0] = x[a][idx]; }
    __device__ __forceinline__ double combine(const T (&raw)[R]) const { return (double)raw[0]; }
};

template <typename T>
struct InDirection {        // p_new = r + beta p_old (p_new = r on the first iteration)
    static constexpr int R = 2;
    const T *r[2];
    const T *p[2];
    const double *beta_dev; // beta of Algorithm 2, written by the previous finalisation
    int first;
    double beta;
    StepLink link;          // folded finalisation of the previous sweep B (if link.state)
    __device__ __forceinline__ void prepare() { beta = first ? 0.0 : *beta_dev; }
    // Called by every thread of the workgroup; returns false when the run has stopped.
    __device__ __forceinline__ bool begin(Pair *sh) {
        if (first || link.state == nullptr) {
            prepare();
            return true;
        }
        return link_step(link, beta, sh);
    }
    __device__ __forceinline__ void load(int a, i64 idx, T (&raw)[R]) const {
        raw[0] = r[a][idx];
        raw[1] = p[a][idx];
    }
    __device__ __forceinline__ double combine(const T (&raw)[R]) const {
        const double rv = (double)raw[0];
        // rounded to the storage type, so the operator acts on exactly the stored vector
        const double pn = (double)(T)(rv + beta * (double)raw[1]);
        return first ? rv : pn;
    }
};

// Preconditioned direction (Algorithm 2 with a diagonal M, entries d): p_new = M^-1 r +
// beta p_old, p*_new = M^-T r* + beta p*_old (p_new = M^-1 r on the first iteration).
template <typename T>
struct InDirectionM {
    static constexpr int R = 3;
    const T *r[2];
    const T *p[2];
    const T *d;
    const double *beta_dev;
    int first;
    double beta;
    StepLink link;
    __device__ __forceinline__ void prepare() { beta = first ? 0.0 : *beta_dev; }
    __device__ __forceinline__ bool begin(Pair *sh) {
        if (first || link.state == nullptr) {
            prepare();
            return true;
        }
        return link_step(link, beta, sh);
    }
    __device__ __forceinline__ void load(int a, i64 idx, T (&raw)[R]) const {
        raw[0] = r[a][idx];
        raw[1] = p[a][idx];
        raw[2] = d[idx];
    }
    __device__ __forceinline__ double combine(const T (&raw)[R]) const {
        const double z = (double)raw[0] / (double)raw[2];
        const double pn = (double)(T)(z + beta * (double)raw[1]);
        return first ? z : pn;
    }
};

// Stored vectors (the directions of the current iteration), with alpha of Algorithm 2 from
// the partials of sweep A merged at the start (the update sweep of the recomputing form).
template <typename T>
struct InPlainAlpha {
    static constexpr int R = 1;
    const T *x[2];
    const double *alpha_dev;  // alpha as finalised by a separate kernel (no link)
    StepLink link;
    double alpha;
    __device__ __forceinline__ void prepare() {}
    __device__ __forceinline__ bool begin(Pair *sh) {
        if (link.state == nullptr) {
            alpha = wave_uniform(*alpha_dev);
            return true;
        }
        return link_alpha(link, alpha, sh);
    }
    __device__ __forceinline__ void load(int a, i64 idx, T (&raw)[R]) const { raw[0] = x[a][idx]; }
    __device__ __forceinline__ double combine(const T (&raw)[R]) const { return (double)raw[0]; }
};

// Kernel: NA marched arrays (1 or 2), input policy In, epilogue Out.
//   Out::emit(lane_state, idx, y[NA], c[NA]) is called for every valid output with the
//   operator values y and the centre values c of the output plane;
//   Out::centre(idx, c[NA]) is called for every valid centre of a plane inside the chunk;
//   Out::finish(block, tile) runs after the march (block-level reductions).
// Epilogues that owe work on their outputs even when the run stops at the start of the
// launch provide Out::prepare() (once per thread), Out::gate() (0 run, 1 skip, 2 the run
// stops in this launch) and Out::finish_output(idx) (the owed work on one output).
template <class O, class = void>
struct HasGate : std::false_type {};
template <class O>
struct HasGate<O, std::void_t<decltype(std::declval<const O &>().gate())>> : std::true_type {};
// Epilogues that read per-output data (Out::Pre, Out::pre(idx)): the values of an output
// are requested with the loads of a staged plane, D planes before the output is complete,
// and handed to emit() then.
template <class O, class = void>
struct HasPre : std::false_type {};
template <class O>
struct HasPre<O, std::void_t<typename O::Pre>> : std::true_type {};
template <class O, bool = HasPre<O>::value>
struct PreOf {
    struct type {};
};
template <class O>
struct PreOf<O, true> {
    using type = typename O::Pre;
};
// Epilogues that take scalars of the input policy once its begin() has made them
// (Out::bind(in)).
template <class O, class I, class = void>
struct HasBind : std::false_type {};
template <class O, class I>
struct HasBind<O, I, std::void_t<decltype(std::declval<O &>().bind(std::declval<const I &>()))>>
    : std::true_type {};

// No step before the march: `in` is already prepared.
struct NoBegin {
    __device__ bool operator()() const { return true; }
};

// March one tile (x-tile, y-tile, z-chunk) of the grid.  Called by a whole 64 x TY
// workgroup; contains barriers.  `begin()` prepares `in` (its scalars, e.g. beta from the
// partials of the previous sweep); it is called after the first planes have been requested,
// so that their loads and the scalars' merge overlap.  Returns false (nothing written) when
// begin() ends the run.
// DOWN: march the chunk's planes from its top down (same outputs, same values).
template <int NA, int TY, typename T, class In, class Out, class Begin = NoBegin, int D = 2,
          bool DOWN = false>
__device__ __forceinline__ bool zmarch_tile(const Geom &g, int tile, const In &in, Out &out,
                                            Begin begin = Begin{}) {
    constexpr int TX = kWave;
    constexpr int LS = TX + 4;          // LDS row stride
    constexpr int LR = TY + 4;          // LDS rows
    constexpr int LE = LS * LR;         // elements per plane
    constexpr int NT = TX * TY;
    constexpr int NL = (LE + NT - 1) / NT;
    // staged values are exactly representable in the storage type T (a stored vector entry
    // times 0 or +-1), so the planes are kept in LDS as T
    __shared__ T buf[2][NA][LE];
    const int n = g.n;
    const int tx = tile % g.tiles_x;
    const int ty = (tile / g.tiles_x) % g.tiles_y;
    const int tz = tile / (g.tiles_x * g.tiles_y);
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = ly * TX + lx;
    const int ix = tx * TX + lx, iy = ty * TY + ly;
    const bool valid = (ix < n) && (iy < n);
    const int k0 = tz * g.zc;
    const int k1 = min(k0 + g.zc, n);
    const i64 plane = g.ps;

    // staging slots of this thread: LDS element e = tid + q*NT.  Every slot has a valid
    // source address (positions outside the grid are clamped and multiplied by 0), so the
    // loads need no branches and can stay in flight.
    int soff[NL];     // source offset inside a plane (row-major, x fastest)
    float smul[NL];   // in-plane multiplier (0 = boundary node, outside, or unused slot),
                      // exactly 0 or +-1, so single precision holds it in fewer registers
#pragma unroll
    for (int q = 0; q < NL; q++) {
        int e = tid + q * NT;
        smul[q] = 0.0f;
        soff[q] = 0;
        if (e < LE) {
            int row = e / LS, col = e % LS;
            int sx, sy;
            double mx = reflect(tx * TX + col - 2, n, g.sgn, sx);
            double my = reflect(ty * TY + row - 2, n, g.sgn, sy);
            smul[q] = (float)(mx * my);
            soff[q] = sy * g.ld + sx;
        }
    }

    constexpr int R = In::R;
    constexpr bool kPre = HasPre<Out>::value;
    using PreT = typename PreOf<Out>::type;
    const int mbeg = k0 - 2, mend = k1 + 1;     // planes mbeg..mend are staged
    constexpr int DZ = DOWN ? -1 : 1;           // direction of the march
    const int mfirst = DOWN ? mend : mbeg;
    // in-plane offset of this lane's column (< 2^31), clamped so that lanes outside the grid
    // request valid addresses
    const int col_off = min(iy, n - 1) * g.ld + min(ix, n - 1);

    // One stage of the load pipeline: the raw values of staged plane p and the per-output
    // data of output p - 3 (complete when plane p is staged, i.e. in the body of plane p - 1).
    struct Stage {
        T raw[NL][NA][R];
        float mz;
        PreT pre;
    };
    auto fetch = [&](int p, Stage &st) {
        int sz;
        st.mz = (float)reflect(DOWN ? max(p, mbeg) : min(p, mend), n, g.sgn, sz);
#pragma unroll
        for (int q = 0; q < NL; q++) {
            const i64 idx = (i64)sz * plane + soff[q];
#pragma unroll
            for (int a = 0; a < NA; a++) in.load(a, idx, st.raw[q][a]);
        }
        if constexpr (kPre)
            st.pre = out.pre((i64)min(max(p - 3 * DZ, k0), k1 - 1) * plane + col_off);
    };
    // the staged value is the input times 0 or +-1, which is exact in the storage type
    auto stash = [&](int b, const Stage &st) {
#pragma unroll
        for (int q = 0; q < NL; q++) {
            const int e = tid + q * NT;
            const float mul = smul[q] * st.mz;
            if (e < LE) {
#pragma unroll
                for (int a = 0; a < NA; a++) {
                    const T v = (T)in.combine(st.raw[q][a]);
                    buf[b][a][e] = mul == 0.0f ? (T)0 : (mul > 0.0f ? v : -v);
                }
            }
        }
    };

    using Col = std::conditional_t<DOWN, ColumnDown, Column>;
    Col col[NA];
#pragma unroll
    for (int a = 0; a < NA; a++) column_init(col[a]);

    Stage stage[D], stage0;
    fetch(mfirst, stage0);
#pragma unroll
    for (int k = 0; k < D; k++) fetch(mfirst + DZ * (1 + k), stage[k]);
    if (!begin()) return false;
    stash(0, stage0);
    __syncthreads();
    int cur = 0;
    const int centre = (ly + 2) * LS + (lx + 2);
    // consume plane m from LDS, stage the next plane (m+1, or m-1 down) from `st`, refill
    // `st` with the plane D after it
    auto body = [&](int m, Stage &st) {
        double y[NA], c0[NA], cprev[NA];
#pragma unroll
        for (int a = 0; a < NA; a++) {
            cprev[a] = col[a].c2;    // centre of the output plane m-2 (m+2) before the shift
            y[a] = column_step<LS, T>(col[a], &buf[cur][a][centre], c0[a]);
        }
        if (valid) {
            if (m >= k0 && m < k1) out.centre((i64)m * plane + col_off, c0);
            const int k = m - 2 * DZ;
            if (k >= k0 && k < k1) {
                if constexpr (kPre) out.emit((i64)k * plane + col_off, y, cprev, st.pre);
                else out.emit((i64)k * plane + col_off, y, cprev);
            }
        }
        stash(cur ^ 1, st);
        fetch(m + DZ * (1 + D), st);
        __syncthreads();
        cur ^= 1;
    };
    // Whole groups of D planes with no exit inside a group, then the remaining planes.
    const int groups = (mend - mbeg + 1) / D;
    int m = mfirst;
    for (int grp = 0; grp < groups; grp++, m += DZ * D) {
#pragma unroll
        for (int u = 0; u < D; u++) body(m + DZ * u, stage[u]);
    }
#pragma unroll
    for (int u = 0; u < D - 1; u++)
        if (DOWN ? (m - u >= mbeg) : (m + u <= mend)) body(m + DZ * u, stage[u]);
    return true;
}

// The outputs of one tile without the march: Out::finish_output(idx) for each (used when a
// run stops at the start of a sweep whose epilogue still owes work on its outputs).
template <int TY, class Out>
__device__ __forceinline__ void zmarch_tile_outputs(const Geom &g, int tile, Out &out) {
    const int n = g.n;
    const int tx = tile % g.tiles_x;
    const int ty = (tile / g.tiles_x) % g.tiles_y;
    const int tz = tile / (g.tiles_x * g.tiles_y);
    const int ix = tx * kWave + threadIdx.x, iy = ty * TY + threadIdx.y;
    if (ix >= n || iy >= n) return;
    const int k0 = tz * g.zc, k1 = min(k0 + g.zc, n);
    const i64 plane = g.ps;
    const i64 col = (i64)iy * g.ld + ix;
    for (int k = k0; k < k1; k++) out.finish_output((i64)k * plane + col);
}

// One workgroup per tile (XCD-aware order), then the epilogue's block-level reduction.  D:
// planes in flight.
template <int NA, int TY, typename T, class In, class Out, int D, bool DOWN>
__device__ __forceinline__ void zmarch_launch(const Geom &g, const In &in_arg, Out &out) {
    __shared__ Pair red[4 * TY];
    __shared__ int s_skip;
    In in = in_arg;
    if constexpr (HasGate<Out>::value) out.prepare();
    bool stops = false;      // the run stops at the start of this launch
    // after the tile's first loads are in flight: the status (one decision per workgroup, as
    // a folded finalisation may publish a new status meanwhile), then the scalars
    auto start = [&]() {
        if (threadIdx.x == 0 && threadIdx.y == 0) {
            if constexpr (HasGate<Out>::value) s_skip = out.gate();
            else s_skip = out.skip() ? 1 : 0;
        }
        __syncthreads();
        if (s_skip == 2) {     // the run stops in this launch (decided by another workgroup)
            stops = true;
            return false;
        }
        if (s_skip) return false;
        const bool run = in.begin(red);
        stops = !run;
        if constexpr (HasBind<Out, In>::value) {
            if (run) out.bind(in);
        }
        return run;
    };
    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const bool go = tile < g.ntiles
                        ? zmarch_tile<NA, TY, T, In, Out, decltype(start), D, DOWN>(g, tile, in,
                                                                                 out, start)
                        : start();
    if (!go) {
        if constexpr (HasGate<Out>::value) {
            if (stops && tile < g.ntiles) zmarch_tile_outputs<TY>(g, tile, out);
        }
        return;
    }
    out.finish(blockIdx.x, red);  // padding blocks of the XCD-aware grid contribute zero
}

template <int NA, int TY, typename T, class In, class Out, int D = 2>
__global__ void __launch_bounds__(kWave *TY) zmarch(Geom g, In in, Out out) {
    zmarch_launch<NA, TY, T, In, Out, D, false>(g, in, out);
}

// The same sweep marching every chunk from its top plane down.  A sweep that follows an
// upward one starts on the planes that one touched last, which the last-level cache may
// still hold.
template <int NA, int TY, typename T, class In, class Out, int D = 2>
__global__ void __launch_bounds__(kWave *TY) zmarch_down(Geom g, In in, Out out) {
    zmarch_launch<NA, TY, T, In, Out, D, true>(g, in, out);
}

// ------------------------------------------------------------------ epilogues

template <typename T>
struct OutApply {           // y = A x
    T *y;
    __device__ bool skip() const { return false; }
    __device__ void centre(i64, const double *) {}
    __device__ void emit(i64 idx, const double *v, const double *) { y[idx] = (T)v[0]; }
    __device__ void finish(int, Pair *) {}
};

template <typename T>
struct OutResidual {        // r = b - A x, partial of r.r
    const double *b;
    T *r;
    Pair *partials;
    Pair acc;
    struct Pre {
        double b;
    };
    __device__ bool skip() const { return false; }
    __device__ void centre(i64, const double *) {}
    __device__ Pre pre(i64 idx) const { return Pre{b[idx]}; }
    __device__ void emit(i64 idx, const double *v, const double *, const Pre &pr) {
        double rv = pr.b - v[0];
        r[idx] = (T)rv;
        dot2_acc(acc, rv, rv);
    }
    __device__ void finish(int block, Pair *sh) {
        Pair v[1] = {acc};
        block_merge<1>(v, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) partials[block] = v[0];
    }
};

// Outer residual of iterative refinement: r64 = b - A u in FP64 (u FP64), stored rounded
// to FP32 twice (the inner Bi-CG's r_0 and r*_0), partial of r64.r64.
struct OutResidualCast {
    const double *b;
    float *r32;
    float *rs32;
    Pair *partials;
    Pair acc;
    struct Pre {
        double b;
    };
    __device__ bool skip() const { return false; }
    __device__ void centre(i64, const double *) {}
    __device__ Pre pre(i64 idx) const { return Pre{b[idx]}; }
    __device__ void emit(i64 idx, const double *v, const double *, const Pre &pr) {
        const double rv = pr.b - v[0];
        const float rf = (float)rv;
        r32[idx] = rf;
        rs32[idx] = rf;
        dot2_acc(acc, rv, rv);
    }
    __device__ void finish(int block, Pair *sh) {
        Pair v[1] = {acc};
        block_merge<1>(v, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) partials[block] = v[0];
    }
};

// CG sweep A (the symmetric specialisation of Bi-CG: with r*_0 = r_0 the shadow sequence equals
// the primal one): p_new = r + beta p (staged), q = A p_new, partial of p_new . q.  Stores
// p_new (centres) and q.  Accumulates the same products in the same order as OutPairApply.
template <typename T>
struct OutDirApply {
    T *p_new;
    T *q;
    Pair *partials;
    const int *status;
    Pair acc;
    __device__ bool skip() const { return *status != 0; }
    __device__ void centre(i64 idx, const double *c) { p_new[idx] = (T)c[0]; }
    __device__ void emit(i64 idx, const double *v, const double *c) {
        const T q0 = (T)v[0];
        q[idx] = q0;
        dot2_acc(acc, (double)(T)c[0], (double)q0);
    }
    __device__ void finish(int block, Pair *sh) {
        Pair v[1] = {acc};
        block_merge<1>(v, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) partials[block] = v[0];
    }
};

// Bi-CG sweep A: p_new = r + beta p (staged), q = A p_new, qs = A ps_new, partial of
// sigma = ps_new . q.  Stores p_new, ps_new (centres) and q, qs.
template <typename T>
struct OutPairApply {
    T *p_new[2];
    T *q[2];
    Pair *partials;
    const int *status;
    Pair acc;
    __device__ bool skip() const { return *status != 0; }
    __device__ void centre(i64 idx, const double *c) {
        p_new[0][idx] = (T)c[0];
        p_new[1][idx] = (T)c[1];
    }
    __device__ void emit(i64 idx, const double *v, const double *c) {
        T q0 = (T)v[0], q1 = (T)v[1];
        q[0][idx] = q0;
        q[1][idx] = q1;
        dot2_acc(acc, (double)(T)c[1], (double)q0);
    }
    __device__ void finish(int block, Pair *sh) {
        Pair v[1] = {acc};
        block_merge<1>(v, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) partials[block] = v[0];
    }
};

// Sweep A that also applies the previous iteration's update of the iterate, x += alpha p
// (alpha and p of iteration j-1, which sweep B then leaves to it): the streams of x and p
// move from the update sweep into this one, where p is read anyway.  The arithmetic is the
// update sweep's; x and p of an output are requested with the march's loads.  When the run
// stops at the start of the launch, the update is applied on its own.
template <typename T>
struct OutPairApplyX : OutPairApply<T> {
    double *x;
    const T *pold;               // p of iteration j-1 (the direction sweep A reads)
    const double *alpha_dev;     // alpha of iteration j-1
    double alpha;
    struct Pre {
        double x;
        T p;
    };
    __device__ void prepare() { alpha = wave_uniform(*alpha_dev); }
    // 0: running; 2: the run stops in this launch (a workgroup already decided it); 1: stopped
    // before this launch (nothing owed)
    __device__ int gate() const {
        const int s = *this->status;
        return s == kRunning ? 0 : (s == kStopping ? 2 : 1);
    }
    __device__ Pre pre(i64 idx) const { return Pre{x[idx], pold[idx]}; }
    __device__ void emit(i64 idx, const double *v, const double *c, const Pre &pr) {
        x[idx] = pr.x + alpha * (double)pr.p;
        OutPairApply<T>::emit(idx, v, c);
    }
    __device__ void finish_output(i64 idx) { x[idx] = x[idx] + alpha * (double)pold[idx]; }
};

// The recomputing form of a Bi-CG iteration (FP32 vectors on large 3D grids): q = A p and
// q* = A^T p* are not stored but formed again where they are used, which saves their
// stream (a pair of stores and a pair of loads per unknown) for a second pass of the
// stencil, whose arithmetic does not limit these memory-bound sweeps.
//
// Sweep A: p_new = r + beta p is marched (one array) for q = A p_new, which here only feeds
// sigma = p*_new . q; p*_new = r* + beta p* is formed at the output from r* and p* requested
// with the march's loads.  Stores p_new and p*_new.  Same values, roundings and products as
// OutPairApply.
template <typename T>
struct OutDirSigma {
    T *p_new;
    T *ps_new;
    const T *rs;         // r*
    const T *ps_old;     // p* of the previous iteration
    Pair *partials;
    const int *status;
    double beta;
    int first;
    Pair acc;
    struct Pre {
        T r, p;
    };
    template <class In>
    __device__ void bind(const In &in) {
        beta = in.beta;
        first = in.first;
    }
    __device__ bool skip() const { return *status != 0; }
    __device__ void centre(i64, const double *) {}
    __device__ Pre pre(i64 idx) const { return Pre{rs[idx], ps_old[idx]}; }
    __device__ void emit(i64 idx, const double *v, const double *c, const Pre &pr) {
        p_new[idx] = (T)c[0];
        const double rv = (double)pr.r;
        const T psn = (T)(first ? rv : (double)(T)(rv + beta * (double)pr.p));
        ps_new[idx] = psn;
        dot2_acc(acc, (double)psn, (double)(T)v[0]);
    }
    __device__ void finish(int block, Pair *sh) {
        Pair w[1] = {acc};
        block_merge<1>(w, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) partials[block] = w[0];
    }
};

// Sweep A of the recomputing form that owes the iterate the update of the previous
// iteration (paired updates, see OutPairUpdate): while the run goes on the next sweep B
// applies it; when the run stops at the start of this launch, x += alpha p_old is applied
// here on its own, with the update sweep's arithmetic.
template <typename T>
struct OutDirSigmaX : OutDirSigma<T> {
    double *x;
    const T *pold;               // p of iteration j-1 (the direction this sweep reads)
    const double *alpha_dev;     // alpha of iteration j-1
    double alpha_owed;
    __device__ void prepare() { alpha_owed = wave_uniform(*alpha_dev); }
    // 0: running; 2: the run stops in this launch (a workgroup already decided it); 1: stopped
    // before this launch (nothing owed)
    __device__ int gate() const {
        const int s = *this->status;
        return s == kRunning ? 0 : (s == kStopping ? 2 : 1);
    }
    __device__ void finish_output(i64 idx) { x[idx] = x[idx] + alpha_owed * (double)pold[idx]; }
};

// Sweep B: p and p* (stored by sweep A) are marched for q = A p and q* = A^T p*, then
// x += alpha p, r -= alpha q, r* -= alpha q*, and the partials of r*.r and r.r: the
// arithmetic of the update sweep, element by element, with q and q* rounded as if stored.
// XM selects the iterate's update, so that two iterations can share one pass over x:
//   0  x += alpha p;
//   1  none (the next sweep B applies it);
//   2  x += alpha' p' and then x += alpha p, alpha' and p' those of the previous iteration,
//      each rounded as its own sweep of mode 0 would round it.
template <typename T, int XM = 0>
struct OutPairUpdate {
    double *x;
    T *r;
    T *rs;
    Pair *partials;
    const int *status;
    double alpha;
    Pair acc[2];
    const T *p_prev;             // XM 2: p of the previous iteration
    double alpha_prev;           // XM 2: its alpha
    struct Pre {
        double x;
        T r, rs, p;
    };
    template <class In>
    __device__ void bind(const In &in) { alpha = in.alpha; }
    __device__ bool skip() const { return *status != 0; }
    __device__ void centre(i64, const double *) {}
    __device__ Pre pre(i64 idx) const {
        Pre v{};
        if constexpr (XM != 1) v.x = x[idx];
        if constexpr (XM == 2) v.p = p_prev[idx];
        v.r = r[idx];
        v.rs = rs[idx];
        return v;
    }
    __device__ void emit(i64 idx, const double *v, const double *c, const Pre &pr) {
        const T q0 = (T)v[0], q1 = (T)v[1];
        if constexpr (XM == 0) x[idx] = pr.x + alpha * c[0];
        if constexpr (XM == 2) {
            const double xp = pr.x + alpha_prev * (double)pr.p;
            x[idx] = xp + alpha * c[0];
        }
        const double ri = (double)pr.r - alpha * (double)q0;
        const double si = (double)pr.rs - alpha * (double)q1;
        const T rt = (T)ri, st = (T)si;
        r[idx] = rt;
        rs[idx] = st;
        dot2_acc(acc[0], (double)st, (double)rt);
        dot2_acc(acc[1], (double)rt, (double)rt);
    }
    __device__ void finish(int block, Pair *sh) {
        block_merge<2>(acc, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) {
            partials[block] = acc[0];
            partials[gridDim.x + block] = acc[1];
        }
    }
};

// Sweep B of mode 2 with its gate: the previous iteration's update is owed, so a breakdown
// found at the start of this launch (alpha undefined) still applies x += alpha' p' (the
// breakdown is published in poll_status only, see link_alpha); after a sweep A that stopped
// the run (and applied the update itself) the final status replaces kStopping.
template <typename T>
struct OutPairUpdate2 : OutPairUpdate<T, 2> {
    BicgState *state;            // the run's state (NULL without folded finalisations)
    const double *alpha_prev_dev;
    __device__ void prepare() { this->alpha_prev = wave_uniform(*alpha_prev_dev); }
    __device__ int gate() const {
        const int s = *this->status;
        if (s == kRunning) return 0;
        if (s == kStopping && state && blockIdx.x == 0) state->status = state->poll_status;
        return 1;
    }
    __device__ void finish_output(i64 idx) {
        double *x = this->x;
        x[idx] = x[idx] + this->alpha_prev * (double)this->p_prev[idx];
    }
};

}  // namespace excmg
