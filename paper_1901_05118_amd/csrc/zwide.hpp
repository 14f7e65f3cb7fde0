// The recomputing form's Bi-CG sweeps (see OutDirSigma and OutPairUpdate in zmarch.hpp) with
// two adjacent points per lane, for FP32 vectors on padded rows (an even row stride, so that
// the two points' elements form one aligned 8-byte pair).
//
// Why: the single-point sweeps of this form are limited by how many bytes one memory
// instruction moves, not by their arithmetic (cutting a quarter of their vector
// instructions left their time unchanged; FP64 vectors, with twice the bytes per access,
// reach a higher fraction of the HBM peak).  Here every global access of a lane is an
// 8-byte pair (16 bytes for the FP64 iterate), a workgroup of 64 x TY lanes owns a
// 128 x TY column tile, and the two points' column pipelines interleave, so each wave has
// twice the independent work between its waits.
//
// Addressing: buffer loads and stores.  The descriptor of each array is rebased once per
// tile to the first plane the tile touches, and the plane offset of each access is a scalar
// (byte offsets in 32 bits), so no lane computes a 64-bit address in the plane loop; an
// offset beyond the descriptor's size reads 0 and writes nothing.
//
// Arithmetic: per point exactly that of the single-point sweeps (the same column pipeline
// of eq. (method1), the same roundings to FP32); only the partition of the compensated
// partial sums differs (per tile), which the Dot2 sums absorb.
#pragma once

#include "zmarch.hpp"

namespace excmg {

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Buffer descriptor of `bytes` bytes from p (raw, no stride; the fourth word selects the
// 32-bit data format).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wide_rsrc(const void *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ __forceinline__ f32x2 wide_load2(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
}
__device__ __forceinline__ void wide_store2(f32x2 x, __amdgpu_buffer_rsrc_t r, unsigned v,
                                           unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, v, s, 0);
}
__device__ __forceinline__ void wide_store1(float x, __amdgpu_buffer_rsrc_t r, unsigned v,
                                           unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, v, s, 0);
}
struct D2 {
    double x, y;
};
__device__ __forceinline__ D2 wide_load2d(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, v, s, 0);
    u32x2 a, b;
    a.x = w.x;
    a.y = w.y;
    b.x = w.z;
    b.y = w.w;
    return D2{__builtin_bit_cast(double, a), __builtin_bit_cast(double, b)};
}
__device__ __forceinline__ void wide_store2d(D2 d, __amdgpu_buffer_rsrc_t r, unsigned v,
                                            unsigned s) {
    const u32x2 a = __builtin_bit_cast(u32x2, d.x), b = __builtin_bit_cast(u32x2, d.y);
    u32x4 w;
    w.x = a.x;
    w.y = a.y;
    w.z = b.x;
    w.w = b.y;
    __builtin_amdgcn_raw_buffer_store_b128(w, r, v, s, 0);
}
__device__ __forceinline__ void wide_store1d(double d, __amdgpu_buffer_rsrc_t r, unsigned v,
                                            unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, d), r, v, s, 0);
}

// Byte count from element offset `from` to the end of an array of `total` elements of
// `size` bytes (at most 2^32 - 1: the descriptor's limit).
__device__ __forceinline__ unsigned wide_span(i64 total, i64 from, int size) {
    const i64 b = (total - from) * size;
    return b > 0xffffffffLL ? 0xffffffffu : (unsigned)b;
}

// ------------------------------------------------------------------ input policies
// load(a, v, s, raw): the R raw pairs of marched array a at byte offsets v (lane) + s
// (plane); combine(raw, e): the staged value of element e (0 or 1) of the pair.

struct WideDirection {      // p_new = r + beta p_old (p_new = r on the first iteration)
    static constexpr int R = 2;
    const float *r;
    const float *p;
    const double *beta_dev;
    int first;
    double beta;
    StepLink link;
    __amdgpu_buffer_rsrc_t rr, rp;
    __device__ __forceinline__ void rebase(i64 total, i64 from) {
        const unsigned nb = wide_span(total, from, 4);
        rr = wide_rsrc(r + from, nb);
        rp = wide_rsrc(p + from, nb);
    }
    __device__ __forceinline__ bool begin(Pair *sh) {
        if (first || link.state == nullptr) {
            beta = first ? 0.0 : *beta_dev;
            return true;
        }
        return link_step(link, beta, sh);
    }
    __device__ __forceinline__ void load(int, unsigned v, unsigned s, f32x2 (&raw)[R]) const {
        raw[0] = wide_load2(rr, v, s);
        raw[1] = wide_load2(rp, v, s);
    }
    __device__ __forceinline__ float combine(const f32x2 (&raw)[R], int e) const {
        const double rv = (double)(e ? raw[0].y : raw[0].x);
        const double pv = (double)(e ? raw[1].y : raw[1].x);
        const double pn = (double)(float)(rv + beta * pv);
        return (float)(first ? rv : pn);
    }
};

struct WidePlainAlpha {     // the stored directions p, p*; alpha from sweep A's partials
    static constexpr int R = 1;
    const float *x[2];
    const double *alpha_dev;
    StepLink link;
    double alpha;
    __amdgpu_buffer_rsrc_t rx[2];
    __device__ __forceinline__ void rebase(i64 total, i64 from) {
        const unsigned nb = wide_span(total, from, 4);
        rx[0] = wide_rsrc(x[0] + from, nb);
        rx[1] = wide_rsrc(x[1] + from, nb);
    }
    __device__ __forceinline__ bool begin(Pair *sh) {
        if (link.state == nullptr) {
            alpha = wave_uniform(*alpha_dev);
            return true;
        }
        return link_alpha(link, alpha, sh);
    }
    __device__ __forceinline__ void load(int a, unsigned v, unsigned s, f32x2 (&raw)[R]) const {
        raw[0] = wide_load2(rx[a], v, s);
    }
    __device__ __forceinline__ float combine(const f32x2 (&raw)[R], int e) const {
        return e ? raw[0].y : raw[0].x;
    }
};

// ------------------------------------------------------------------ epilogues
// pre(v, s): the per-output data of a lane's two outputs; emit(v, s, y, c, pre, two): the
// outputs (y[e][a], c[e][a]: operator value and centre of array a at element e; two: the
// second point lies inside the grid).

struct WideDirSigma {       // sweep A: store p, form p* at the outputs, sigma = p* . A p
    float *p_new;
    float *ps_new;
    const float *rs;
    const float *ps_old;
    Pair *partials;
    const int *status;
    double beta;
    int first;
    Pair acc;
    __amdgpu_buffer_rsrc_t rpn, rpsn, rrs, rpso;
    struct Pre {
        f32x2 r, p;
    };
    __device__ __forceinline__ void rebase(i64 total, i64 from) {
        const unsigned nb = wide_span(total, from, 4);
        rpn = wide_rsrc(p_new + from, nb);
        rpsn = wide_rsrc(ps_new + from, nb);
        rrs = wide_rsrc(rs + from, nb);
        rpso = wide_rsrc(ps_old + from, nb);
    }
    __device__ void bind(const WideDirection &in) {
        beta = in.beta;
        first = in.first;
    }
    __device__ bool skip() const { return *status != 0; }
    __device__ __forceinline__ Pre pre(unsigned v, unsigned s) const {
        return Pre{wide_load2(rrs, v, s), wide_load2(rpso, v, s)};
    }
    __device__ __forceinline__ float psnew(float r, float p) const {
        const double rv = (double)r;
        return (float)(first ? rv : (double)(float)(rv + beta * (double)p));
    }
    __device__ __forceinline__ void emit(unsigned v, unsigned s, const double (&y)[2][1],
                                         const double (&c)[2][1], const Pre &pr, bool two) {
        const float s0 = psnew(pr.r.x, pr.p.x);
        if (two) {
            const float s1 = psnew(pr.r.y, pr.p.y);
            f32x2 pn, sn;
            pn.x = (float)c[0][0];
            pn.y = (float)c[1][0];
            sn.x = s0;
            sn.y = s1;
            wide_store2(pn, rpn, v, s);
            wide_store2(sn, rpsn, v, s);
            dot2_acc(acc, (double)s0, (double)(float)y[0][0]);
            dot2_acc(acc, (double)s1, (double)(float)y[1][0]);
        } else {
            wide_store1((float)c[0][0], rpn, v, s);
            wide_store1(s0, rpsn, v, s);
            dot2_acc(acc, (double)s0, (double)(float)y[0][0]);
        }
    }
    __device__ void finish(int block, Pair *sh) {
        Pair w[1] = {acc};
        block_merge<1>(w, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) partials[block] = w[0];
    }
};

struct WidePairUpdate {     // sweep B: q, q* formed again; x += alpha p, r -= alpha q, ...
    double *x;
    float *r;
    float *rs;
    Pair *partials;
    const int *status;
    double alpha;
    Pair acc[2];
    __amdgpu_buffer_rsrc_t rx, rr, rrs;
    struct Pre {
        D2 x;
        f32x2 r, rs;
    };
    __device__ __forceinline__ void rebase(i64 total, i64 from) {
        rx = wide_rsrc(x + from, wide_span(total, from, 8));
        const unsigned nb = wide_span(total, from, 4);
        rr = wide_rsrc(r + from, nb);
        rrs = wide_rsrc(rs + from, nb);
    }
    __device__ void bind(const WidePlainAlpha &in) { alpha = in.alpha; }
    __device__ bool skip() const { return *status != 0; }
    // x's byte offsets are twice those of the FP32 arrays (same element offsets)
    __device__ __forceinline__ Pre pre(unsigned v, unsigned s) const {
        return Pre{wide_load2d(rx, 2 * v, 2 * s), wide_load2(rr, v, s), wide_load2(rrs, v, s)};
    }
    __device__ __forceinline__ void point(double xo, float ro, float so, double ya, double yb,
                                          double c, double &xn, float &rt, float &st) {
        const float q0 = (float)ya, q1 = (float)yb;
        xn = xo + alpha * c;
        rt = (float)((double)ro - alpha * (double)q0);
        st = (float)((double)so - alpha * (double)q1);
        dot2_acc(acc[0], (double)st, (double)rt);
        dot2_acc(acc[1], (double)rt, (double)rt);
    }
    __device__ __forceinline__ void emit(unsigned v, unsigned s, const double (&y)[2][2],
                                         const double (&c)[2][2], const Pre &pr, bool two) {
        double x0, x1;
        float r0, r1, s0, s1;
        point(pr.x.x, pr.r.x, pr.rs.x, y[0][0], y[0][1], c[0][0], x0, r0, s0);
        if (two) {
            point(pr.x.y, pr.r.y, pr.rs.y, y[1][0], y[1][1], c[1][0], x1, r1, s1);
            wide_store2d(D2{x0, x1}, rx, 2 * v, 2 * s);
            f32x2 rv, sv;
            rv.x = r0;
            rv.y = r1;
            sv.x = s0;
            sv.y = s1;
            wide_store2(rv, rr, v, s);
            wide_store2(sv, rrs, v, s);
        } else {
            wide_store1d(x0, rx, 2 * v, 2 * s);
            wide_store1(r0, rr, v, s);
            wide_store1(s0, rrs, v, s);
        }
    }
    __device__ void finish(int block, Pair *sh) {
        block_merge<2>(acc, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) {
            partials[block] = acc[0];
            partials[block + gridDim.x] = acc[1];
        }
    }
};

// ------------------------------------------------------------------ the march
// One 128 x TY column tile through its chunk of planes: each lane owns the points ix and
// ix + 1 of one row.  Staging: a plane of the tile with its 2-wide halo is (128 + 4) x
// (TY + 4) elements, requested as aligned pairs (slot e: pair e % 66 of row e / 66) and
// stored in LDS as pairs.  A pair of the halo may hold a fictitious point, a boundary node
// or a point beyond the grid: its source pair is the aligned pair holding the first
// element that has a source, each element picks its half and is multiplied by 0 or +-1
// (bit masks).  Everything else follows zmarch_tile: D planes of loads in flight, whole
// groups of D planes per loop trip, the per-output data requested with the plane that
// completes the output.
template <int NA, int TY, class In, class Out, class Begin, int D>
__device__ __forceinline__ bool zwide_tile(const Geom &g, int tile, In &in, Out &out,
                                           Begin begin) {
    constexpr int TX = 2 * kWave;
    constexpr int LS = TX + 4;          // LDS row stride (even: pairs stay aligned)
    constexpr int LR = TY + 4;
    constexpr int NP = LS / 2;          // pairs per staged row
    constexpr int LP = NP * LR;         // pairs per staged plane
    constexpr int NT = kWave * TY;
    constexpr int NL = (LP + NT - 1) / NT;
    constexpr int R = In::R;
    __shared__ __attribute__((aligned(16))) float buf[2][NA][LS * LR];
    const int n = g.n;
    const int tx = tile % g.tiles_x;
    const int ty = (tile / g.tiles_x) % g.tiles_y;
    const int tz = tile / (g.tiles_x * g.tiles_y);
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = ly * kWave + lx;
    const int ix = tx * TX + 2 * lx, iy = ty * TY + ly;
    const bool valid = ix < n && iy < n, two = ix + 1 < n;
    const int k0 = tz * g.zc, k1 = min(k0 + g.zc, n);
    const i64 plane = g.ps;
    // descriptors start at the first plane the tile touches: plane offsets stay small
    const int base = max(k0 - 2, 0);
    const i64 total = plane * n;
    in.rebase(total, (i64)base * plane);
    out.rebase(total, (i64)base * plane);
    unsigned soff[NL];
    unsigned flip[NL][2], keep[NL][2];
    bool hi[NL][2];
#pragma unroll
    for (int q = 0; q < NL; q++) {
        const int e = tid + q * NT;
        soff[q] = 0;
        hi[q][0] = false;
        hi[q][1] = true;
        flip[q][0] = flip[q][1] = 0u;
        keep[q][0] = keep[q][1] = 0u;
        if (e < LP) {
            const int row = e / NP, j = e % NP;
            int sy, s0, s1;
            const double my = reflect(ty * TY + row - 2, n, g.sgn, sy);
            const int x0 = tx * TX + 2 * j - 2;
            const double m0 = reflect(x0, n, g.sgn, s0) * my;
            const double m1 = reflect(x0 + 1, n, g.sgn, s1) * my;
            const int b = (m0 != 0.0 ? s0 : s1) & ~1;
            soff[q] = (unsigned)(sy * g.ld + b) * 4u;
            hi[q][0] = s0 - b == 1;
            hi[q][1] = s1 - b == 1;
            flip[q][0] = m0 < 0.0 ? 0x80000000u : 0u;
            flip[q][1] = m1 < 0.0 ? 0x80000000u : 0u;
            keep[q][0] = m0 != 0.0 ? 0xffffffffu : 0u;
            keep[q][1] = m1 != 0.0 ? 0xffffffffu : 0u;
        }
    }
    using PreT = typename Out::Pre;
    const int mbeg = k0 - 2, mend = k1 + 1;
    // the lane's pair (clamped into the grid, so idle lanes request valid addresses)
    const unsigned col_off = (unsigned)(min(iy, n - 1) * g.ld + min(ix, (n - 1) & ~1)) * 4u;
    struct Stage {
        f32x2 raw[NL][NA][R];
        float mz;
        PreT pre;
    };
    auto plane_bytes = [&](int p) { return (unsigned)((i64)(p - base) * plane * 4); };
    auto fetch = [&](int p, Stage &st) {
        int sz;
        st.mz = (float)reflect(min(p, mend), n, g.sgn, sz);
        const unsigned s = plane_bytes(max(sz, base));
#pragma unroll
        for (int q = 0; q < NL; q++) {
#pragma unroll
            for (int a = 0; a < NA; a++) in.load(a, soff[q], s, st.raw[q][a]);
        }
        st.pre = out.pre(col_off, plane_bytes(min(max(p - 3, k0), k1 - 1)));
    };
    auto stash = [&](int bsel, const Stage &st) {
        const unsigned fz = st.mz < 0.0f ? 0x80000000u : 0u;
        const unsigned kz = st.mz != 0.0f ? 0xffffffffu : 0u;
#pragma unroll
        for (int q = 0; q < NL; q++) {
            const int e = tid + q * NT;
            if (e < LP) {
#pragma unroll
                for (int a = 0; a < NA; a++) {
                    const float lo = in.combine(st.raw[q][a], 0);
                    const float up = in.combine(st.raw[q][a], 1);
                    const float v0 = hi[q][0] ? up : lo, v1 = hi[q][1] ? up : lo;
                    f32x2 o;
                    o.x = __uint_as_float((__float_as_uint(v0) ^ flip[q][0] ^ fz) & keep[q][0] & kz);
                    o.y = __uint_as_float((__float_as_uint(v1) ^ flip[q][1] ^ fz) & keep[q][1] & kz);
                    *(f32x2 *)&buf[bsel][a][2 * e] = o;
                }
            }
        }
    };
    Column col[2][NA];
#pragma unroll
    for (int e = 0; e < 2; e++)
#pragma unroll
        for (int a = 0; a < NA; a++) column_init(col[e][a]);
    Stage stage[D], stage0;
    fetch(mbeg, stage0);
#pragma unroll
    for (int k = 0; k < D; k++) fetch(mbeg + 1 + k, stage[k]);
    if (!begin()) return false;
    stash(0, stage0);
    __syncthreads();
    int cur = 0;
    const int centre = (ly + 2) * LS + 2 * lx + 2;
    auto body = [&](int m, Stage &st) {
        double y[2][NA], c[2][NA];
#pragma unroll
        for (int e = 0; e < 2; e++)
#pragma unroll
            for (int a = 0; a < NA; a++) {
                double c0;
                c[e][a] = col[e][a].c2;    // centre of plane m-2 (the output's plane)
                y[e][a] = column_step<LS, float>(col[e][a], &buf[cur][a][centre + e], c0);
            }
        const int k = m - 2;
        if (valid && k >= k0 && k < k1) out.emit(col_off, plane_bytes(k), y, c, st.pre, two);
        stash(cur ^ 1, st);
        fetch(m + 1 + D, st);
        __syncthreads();
        cur ^= 1;
    };
    const int groups = (mend - mbeg + 1) / D;
    int m = mbeg;
    for (int grp = 0; grp < groups; grp++, m += D) {
#pragma unroll
        for (int u = 0; u < D; u++) body(m + u, stage[u]);
    }
#pragma unroll
    for (int u = 0; u < D - 1; u++)
        if (m + u <= mend) body(m + u, stage[u]);
    return true;
}

// One workgroup of 64 x TY lanes per 128 x TY tile (XCD-aware order), then the epilogue's
// block-level reduction.
template <int NA, int TY, class In, class Out, int D>
__global__ void __launch_bounds__(kWave *TY) zwide(Geom g, In in_arg, Out out) {
    __shared__ Pair red[4 * TY];
    __shared__ int s_skip;
    In in = in_arg;
    auto start = [&]() {
        if (threadIdx.x == 0 && threadIdx.y == 0) s_skip = out.skip() ? 1 : 0;
        __syncthreads();
        if (s_skip) return false;
        const bool run = in.begin(red);
        if (run) out.bind(in);
        return run;
    };
    const int tile = xcd_tile(blockIdx.x, g.ntiles);
    const bool go = tile < g.ntiles ? zwide_tile<NA, TY, In, Out, decltype(start), D>(
                                          g, tile, in, out, start)
                                    : start();
    if (!go) return;
    out.finish(blockIdx.x, red);
}

}  // namespace excmg
