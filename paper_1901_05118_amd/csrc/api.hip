// Host driver and C ABI of the EXCMG library: the cascade of Algorithm 1, the level loop,
// the device-resident Bi-CG iteration of Algorithm 2 and the entry points of excmg.h.
//
// Control stays on the device inside a Bi-CG run: the scalars (rho, sigma, alpha, beta,
// r.r) and the run status live in device memory, every kernel of an iteration returns
// immediately once the run has stopped, and the host only reads the 64-byte state every few
// iterations to decide whether to launch more.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/excmg.h"
#include "common.hpp"
#include "internal.hpp"

using namespace excmg;

namespace {

char g_err[512] = "";
hipStream_t g_stream = nullptr;

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define CKH(expr)                                                                            \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(EXCMG_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),  \
                        __FILE__, __LINE__);                                                 \
    } while (0)

#define CKR(expr)                                                                            \
    do {                                                                                     \
        int r_ = (expr);                                                                     \
        if (r_ != EXCMG_OK) return r_;                                                       \
    } while (0)

// ------------------------------------------------------------------ device buffers

struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    int ensure(size_t nb) {
        if (nb <= bytes && p) return EXCMG_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (hipMalloc(&p, nb ? nb : 8) != hipSuccess) {
            (void)hipGetLastError();
            return fail(EXCMG_ENOMEM, "device allocation of %zu bytes failed", nb);
        }
        bytes = nb;
        return EXCMG_OK;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *as() const { return (T *)p; }
};

bool is_device_ptr(const void *p) {
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.isManaged;
}

// An array argument: device pointers are used in place, host arrays are staged.
struct Arg {
    const void *user;
    void *dev = nullptr;
    size_t bytes;
    bool staged = false;
    Arg(const void *u, size_t nb) : user(u), bytes(nb) {}
    int in() {  // input: copy to the device if needed
        if (is_device_ptr(user)) {
            dev = const_cast<void *>(user);
            return EXCMG_OK;
        }
        CKH(hipMalloc(&dev, bytes));
        staged = true;
        CKH(hipMemcpyAsync(dev, user, bytes, hipMemcpyHostToDevice, g_stream));
        return EXCMG_OK;
    }
    int out() {  // output: device scratch if the user's pointer is host memory
        if (is_device_ptr(user)) {
            dev = const_cast<void *>(user);
            return EXCMG_OK;
        }
        CKH(hipMalloc(&dev, bytes));
        staged = true;
        return EXCMG_OK;
    }
    int back() {  // copy an output back to host memory
        if (staged) CKH(hipMemcpyAsync(const_cast<void *>(user), dev, bytes,
                                       hipMemcpyDeviceToHost, g_stream));
        return EXCMG_OK;
    }
    ~Arg() {
        if (staged && dev) {
            (void)hipStreamSynchronize(g_stream);
            (void)hipFree(dev);
        }
    }
    template <typename T>
    T *p() const { return (T *)dev; }
};

// ------------------------------------------------------------------ context

struct Level {
    int index = 0;    // level number (0 = coarsest)
    int N = 0;        // cells per axis
    int n = 0;        // unknowns per axis
    long long nu = 0; // unknowns
    long long nodes = 0;
    Geom g1{}, g2{}, g2f{};  // launch shapes: one-array kernels, sweep A FP64, sweep A FP32
    // Rows of the FP32 Bi-CG vectors (and of the FP64 iterate and right-hand side they are
    // solved with): ld elements apart, nflat elements of storage; g1p is g1 on that layout
    // (g2f always is).  ld = n: contiguous, as every other vector of the level.  The vector
    // kernels walk the nu unknowns in the contiguous order whatever the layout, so results
    // do not depend on it.
    int ld = 0;
    long long nflat = 0;
    Geom g1p{};
    // The recomputing form's FP32 sweeps with two points per lane (128-wide tiles) on padded
    // rows: g2w (tw = 0 where the grid cannot take them), used when `wide` is set.
    Geom g2w{};
    bool wide = false;
    DBuf b, x, u;     // right-hand side, unknowns, node array (solution or EXP_finite guess)
    DBuf diag;        // diag(A_h), made when a Jacobi-preconditioned solve first needs it
    Rows rows() const { return ld == n ? Rows{} : Rows{n, ld}; }
};

void release_graphs();

struct Ctx {
    bool ready = false;
    int n_finest = 0, n_levels = 0, bc = 0;
    int dim = 3;                // 3: the 3D equation (eq. bvp); 2: the 2D one (eq. bvp2d)
    std::vector<Level> lv;
    // Bi-CG workspace (sized for the finest level)
    DBuf r, rs, p[2], ps[2], q, qs;
    DBuf ubest;                 // best FP64 iterate of a level solved with residual replacement
    DBuf xp, bp;                // FP64 iterate and right-hand side of a level with padded rows
    DBuf part_a, part_b;        // Dot2 partials of the two sweeps
    DBuf state;                 // BicgState
    DBuf scal;                  // misc device scalars
    DBuf chol[2];               // banded Cholesky factors of levels 0 and 1
    int chol_w[2] = {0, 0};     // their lower bandwidths
    DBuf info;
    DBuf vz1;                   // EXP_finite Z1 scratch
    BicgState *host_state = nullptr;  // pinned; 3 slots (synchronous reads, pipelined polls)
    double *host_scal = nullptr;      // pinned
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    void release() {
        release_graphs();
        for (auto &L : lv) {
            L.b.release();
            L.x.release();
            L.u.release();
            L.diag.release();
        }
        lv.clear();
        r.release(); rs.release();
        p[0].release(); p[1].release(); ps[0].release(); ps[1].release();
        q.release(); qs.release(); ubest.release(); xp.release(); bp.release();
        part_a.release(); part_b.release(); state.release(); scal.release();
        chol[0].release(); chol[1].release(); info.release(); vz1.release();
        if (host_state) (void)hipHostFree(host_state);
        for (hipEvent_t &e : poll_ev) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
        if (host_scal) (void)hipHostFree(host_scal);
        host_state = nullptr;
        host_scal = nullptr;
        ready = false;
    }
};

Ctx g_ctx;

// Optional per-launch timing of the two Bi-CG sweeps (device events on the library stream),
// accumulated per level: [level][0] sweep A, [level][1] sweep B.
bool g_timing = false;
// [0] sweep A, [1] sweep B, [2] sweep A with the deferred update of the iterate, [3] sweep B
// leaving the iterate to the next one, [4] sweep B applying two iterations' updates
double g_time_ms[EXCMG_MAX_LEVELS][5];
long long g_time_n[EXCMG_MAX_LEVELS][5];
std::vector<hipEvent_t> g_events;

int ensure_events(size_t count) {
    while (g_events.size() < count) {
        hipEvent_t e;
        CKH(hipEventCreate(&e));
        g_events.push_back(e);
    }
    return EXCMG_OK;
}

// Tile shapes chosen by the autotuner (or a caller) per grid size and kernel kind.
struct ShapeOverride {
    int N, kind, ty, zc;
};
std::vector<ShapeOverride> g_shapes;

// Default launch shape: 64 x TY column tiles, and the longest z chunk that still gives
// every CU a tile (measured on MI355X: fewer, longer marches beat more, shorter ones,
// because each chunk re-reads four halo planes).  kind 0: one marched array (operator,
// residual); kind 1 / 2: Bi-CG sweep A on FP64 / FP32 vectors (two marched arrays, twice the
// column state, TY <= 8 to keep its registers below 256).
Geom choose_shape(int N, int bc, int kind) {
    const int n = N - 1;
    for (const ShapeOverride &o : g_shapes)
        if (o.N == N && o.kind == kind) return make_geom(n, bc, o.ty, std::max(1, std::min(o.zc, n)));
    // Shapes the autotuner picks on MI355X, per grid-size band and kind {operator/residual,
    // FP64 sweep A, FP32 sweep A}: {ty, zc}.  Grids up to 64^3 are launch-latency bound and
    // want the most workgroups; larger grids want long z-marches.  FP32 sweep A: timed in the
    // form mixed solves run on these grids (128^3: the stored form with the deferred update
    // of the iterate; from 256^3 the recomputing pair of sweeps, which shares the shape).
    // From 256^3 both pairs take 64x8 tiles of 128 planes (one 512-thread workgroup per CU;
    // its update sweep keeps three planes in flight); from 512^3 the mixed pair marches the
    // whole depth (511 planes) on 64x16 tiles, one per CU, and the FP64 pair on 64x8.
    static const int kTuned[6][3][2] = {
        {{4, 2}, {4, 2}, {4, 2}},          // N < 48
        {{8, 2}, {8, 2}, {8, 2}},          // 48 <= N < 96
        {{4, 8}, {8, 16}, {4, 8}},         // 96 <= N < 128
        {{8, 16}, {8, 16}, {8, 16}},       // 128 <= N < 256
        {{8, 64}, {8, 128}, {8, 128}},     // 256 <= N < 512
        {{16, 512}, {8, 512}, {16, 512}},  // N >= 512
    };
    const int band = N < 48 ? 0 : N < 96 ? 1 : N < 128 ? 2 : N < 256 ? 3 : N < 512 ? 4 : 5;
    const int ty = kTuned[band][kind][0];
    const int zc = std::max(1, std::min(kTuned[band][kind][1], n));
    return make_geom(n, bc, ty, zc);
}

// Row stride of padded vectors: a multiple of 32 elements (every row starts on a 128-byte
// line in FP32 and FP64) plus one more line, which keeps the stride off powers of two
// (rows a power of two apart fall into the same cache sets).
int padded_ld(int n) { return (n + 31) / 32 * 32 + 32; }

void set_rows(Level &L, int ld, int dim) {
    if (dim == 2) ld = L.n;
    L.ld = ld;
    L.nflat = dim == 2 ? L.nu : (long long)L.n * L.n * ld;
    L.g1p = with_rows(L.g1, ld);
    L.g2f = with_rows(L.g2f, ld);
}

int level_ld(int n, int row_pad) { return row_pad > 0 ? padded_ld(n) : n; }

// z-chunk of the two-point sweeps: 64 planes (four chunks on 256^3: one workgroup per CU
// with 128 x 8 tiles), the whole depth from 384 unknowns per axis.
int wide_zc(int n) { return n >= 384 ? n : 64; }

void choose_shapes(Level &L, int bc, int dim = 3) {
    if (dim == 2) {  // one pass per tile: more rows per workgroup on large planes
        const int n = L.N - 1;
        const int ty = n >= 1024 ? 16 : (n >= 96 ? 8 : 4);
        L.g1 = L.g2 = L.g2f = make_geom_2d(n, bc, ty);
    } else {
        L.g1 = choose_shape(L.N, bc, 0);
        L.g2 = choose_shape(L.N, bc, 1);
        L.g2f = choose_shape(L.N, bc, 2);
        const int n = L.N - 1;
        L.g2w = make_geom_wide(n, bc, 8, std::min(wide_zc(n), n), padded_ld(n));
    }
    set_rows(L, L.ld > 0 ? L.ld : L.n, dim);
}

int check_sizes(int n_finest, int n_levels, int bc, int dim = 3) {
    if (bc != 1 && bc != 2) return fail(EXCMG_EINVAL, "bc_kind must be 1 or 2 (got %d)", bc);
    if (n_levels < 3 || n_levels > EXCMG_MAX_LEVELS)
        return fail(EXCMG_EINVAL, "n_levels must be in 3..%d (got %d)", EXCMG_MAX_LEVELS,
                    n_levels);
    if (n_finest < 8 || n_finest > (dim == 2 ? 16384 : 2048))
        return fail(EXCMG_EINVAL, "n_finest out of range");
    const int N0 = n_finest >> (n_levels - 1);
    if (N0 < 2 || (N0 << (n_levels - 1)) != n_finest)
        return fail(EXCMG_EINVAL, "n_finest (%d) must be N0 * 2^(n_levels-1) with N0 >= 2",
                    n_finest);
    const int maxN0 = dim == 2 ? 32 : 8;
    if (N0 > maxN0)
        return fail(EXCMG_EINVAL, "coarsest grid of %d cells is too large for DSOLVE (max %d)",
                    N0, maxN0);
    return EXCMG_OK;
}

// Banded Cholesky factor of a direct level into C (nu x (band_width + 1) doubles); info
// holds at least two ints of device scratch.
int factor_band(int N, int bc, int dim, double *C, int *info, hipStream_t st) {
    const int w = band_width(N, dim);
    const int nu = dim == 2 ? (N - 1) * (N - 1) : (N - 1) * (N - 1) * (N - 1);
    CKH(hipMemsetAsync(info, 0, 2 * sizeof(int), st));
    CKH(band_assemble(N, bc, dim, w, C, info + 1, st));
    CKH(band_cholesky(nu, w, C, info, st));
    int h[2] = {0, 0};
    CKH(hipMemcpyAsync(h, info, sizeof(h), hipMemcpyDeviceToHost, st));
    CKH(hipStreamSynchronize(st));
    if (h[1] != 0) return fail(EXCMG_EHIP, "operator of %d cells wider than its band", N);
    if (h[0] != 0)
        return fail(EXCMG_EBREAKDOWN, "Cholesky pivot %d of the %d-cell level not positive", h[0],
                    N);
    return EXCMG_OK;
}

int setup_levels(int n_finest, int n_levels, int bc, int dim);

// Make the context the given hierarchy (kept if it already is).  A failed set-up (for
// instance device memory exhausted) frees whatever it had allocated.
int setup(int n_finest, int n_levels, int bc, int dim = 3) {
    CKR(check_sizes(n_finest, n_levels, bc, dim));
    Ctx &c = g_ctx;
    if (c.ready && c.n_finest == n_finest && c.n_levels == n_levels && c.bc == bc &&
        c.dim == dim)
        return EXCMG_OK;
    c.release();
    const int rc = setup_levels(n_finest, n_levels, bc, dim);
    if (rc != EXCMG_OK) c.release();
    return rc;
}

int setup_levels(int n_finest, int n_levels, int bc, int dim) {
    Ctx &c = g_ctx;
    c.n_finest = n_finest;
    c.n_levels = n_levels;
    c.bc = bc;
    c.dim = dim;
    const int N0 = n_finest >> (n_levels - 1);
    c.lv.resize(n_levels);
    for (int l = 0; l < n_levels; l++) {
        Level &L = c.lv[l];
        L.index = l;
        L.N = N0 << l;
        L.n = L.N - 1;
        L.nu = (long long)L.n * L.n * (dim == 2 ? 1 : L.n);
        L.nodes = (long long)(L.N + 1) * (L.N + 1) * (dim == 2 ? 1 : (L.N + 1));
        L.ld = 0;
        choose_shapes(L, bc, dim);
        CKR(L.b.ensure(L.nu * 8));
        CKR(L.x.ensure(L.nu * 8));
        CKR(L.u.ensure(L.nodes * 8));
    }
    const Level &F = c.lv.back();
    // FP32 vectors with padded rows (row_pad) fit in the FP64 vectors' room, except on
    // grids of under 64 unknowns per axis
    long long flat = F.nu;
    if (dim == 3)
        for (const Level &L : c.lv) flat = std::max(flat, (long long)L.n * L.n * padded_ld(L.n));
    const size_t vb = std::max((size_t)F.nu * 8, (size_t)flat * 4);
    CKR(c.r.ensure(vb));
    CKR(c.rs.ensure(vb));
    CKR(c.p[0].ensure(vb));
    CKR(c.p[1].ensure(vb));
    CKR(c.ps[0].ensure(vb));
    CKR(c.ps[1].ensure(vb));
    CKR(c.q.ensure(vb));
    CKR(c.qs.ensure(vb));
    CKR(c.ubest.ensure((size_t)F.nu * 8));
    int maxblk = 4096 * 2;
    for (auto &L : c.lv)
        maxblk = std::max({maxblk, stencil_blocks(L.g1), stencil_blocks(L.g2), stencil_blocks(L.g2f),
                           stencil_blocks(L.g2w)});
    CKR(c.part_a.ensure((size_t)maxblk * sizeof(Pair)));
    // two values per partial: the update kernels (at most 4096) or the recomputing update
    // sweep (one per tile)
    CKR(c.part_b.ensure((size_t)2 * std::max(4096, maxblk) * sizeof(Pair)));
    CKR(c.state.ensure(sizeof(BicgState)));
    CKR(c.scal.ensure(64 * sizeof(double)));
    CKR(c.info.ensure(64));
    const long long nz1 =
        (long long)(n_finest / 2 + 1) * (n_finest / 2 + 1) * (dim == 2 ? 1 : (n_finest / 2 + 1));
    CKR(c.vz1.ensure((size_t)nz1 * 8));
    CKH(hipHostMalloc((void **)&c.host_state, 3 * sizeof(BicgState), hipHostMallocDefault));
    for (hipEvent_t &e : c.poll_ev) CKH(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    CKH(hipHostMalloc((void **)&c.host_scal, 64 * sizeof(double), hipHostMallocDefault));
    // Cholesky factors of the two direct levels (depend only on the grid and bc kind)
    for (int l = 0; l < 2; l++) {
        Level &L = c.lv[l];
        c.chol_w[l] = band_width(L.N, dim);
        CKR(c.chol[l].ensure((size_t)L.nu * (c.chol_w[l] + 1) * 8));
        CKR(factor_band(L.N, bc, dim, c.chol[l].as<double>(), c.info.as<int>(), g_stream));
    }
    c.ready = true;
    return EXCMG_OK;
}

int need_ctx(int level) {
    if (!g_ctx.ready) return fail(EXCMG_ENOCTX, "no context: call excmg_setup first");
    if (level < 0 || level >= g_ctx.n_levels)
        return fail(EXCMG_EINVAL, "level %d outside 0..%d", level, g_ctx.n_levels - 1);
    return EXCMG_OK;
}

// ------------------------------------------------------------------ reductions

int device_dot(long long n, const double *x, const double *y, double *out_dev, int slot,
               Rows rows = Rows{}) {
    Ctx &c = g_ctx;
    const int nb = vec_blocks(n);
    CKH(dot_partials<double>(n, x, y, c.part_b.as<Pair>(), nb, g_stream, rows));
    CKH(reduce_to(out_dev, c.part_b.as<Pair>(), nb, slot, g_stream));
    return EXCMG_OK;
}

int read_state(BicgState &s) {
    Ctx &c = g_ctx;
    CKH(hipMemcpyAsync(c.host_state, c.state.p, sizeof(BicgState), hipMemcpyDeviceToHost,
                       g_stream));
    CKH(hipStreamSynchronize(g_stream));
    s = *c.host_state;
    return EXCMG_OK;
}

// The relative-residual floor of FP64 arithmetic for the iterate x of level L (the reading of
// Algorithm 1's while loop): about 22 u ||x||_2 / ||b||_2 with u = 2^-53, the constant fitted
// to the floors measured on 128^3 grids with zero and with smooth boundary data.
constexpr double kFloorConst = 22.0 * 0x1p-53;
int level_floor(const Level &L, const double *x, Rows rows, double bb, double *floor) {
    Ctx &c = g_ctx;
    double *sc = c.scal.as<double>();
    CKR(device_dot(L.nu, x, x, sc, 3, rows));
    CKH(hipMemcpyAsync(c.host_scal + 3, sc + 3, sizeof(double), hipMemcpyDeviceToHost, g_stream));
    CKH(hipStreamSynchronize(g_stream));
    *floor = bb > 0 ? kFloorConst * std::sqrt(c.host_scal[3] / bb) : 0.0;
    return EXCMG_OK;
}

// Why a level stopped, from its status, tolerance and floor.
int level_exit(int status, double eps, double floor) {
    if (status == EXCMG_OK) return EXCMG_EXIT_TOL;
    if (status == EXCMG_EBREAKDOWN) return EXCMG_EXIT_BREAKDOWN;
    return eps < 10.0 * floor ? EXCMG_EXIT_FLOOR : EXCMG_EXIT_CAP;
}

// r = b - A x on the level, and r.r into scal[slot]
int true_residual(const Level &L, const double *b, const double *x, double *r, int slot) {
    Ctx &c = g_ctx;
    CKH(stencil_residual<double>(L.g1, L.g1.ty, b, x, r, c.part_a.as<Pair>(), g_stream));
    CKH(reduce_to(c.scal.as<double>(), c.part_a.as<Pair>(), stencil_blocks(L.g1), slot,
                  g_stream));
    return EXCMG_OK;
}

// ------------------------------------------------------------------ Bi-CG (Algorithm 2)

// Iterations launched between two reads of the device state.  At least 16 on 3D grids below
// 2^26 unknowns: each window adds a closing check and a state copy, which cost more than the
// no-op launches queued after a stop (512^3 solve, one box: mixed 572 / 567 / 563 ms and
// FP64 814 / 805 / 803 ms with at least 4 / 8 / 16).  At least 4 on larger grids and in 2D,
// whose largest levels run a few iterations each and whose no-op launches cost more (2D
// 4096^2 solve: 85.6 ms with 4, 89.6 ms with 16).
int poll_interval(long long nu, int dim) {
    long long k = (1LL << 21) / (nu > 0 ? nu : 1);
    if (k < 16) k = (dim == 3 && nu < (1LL << 26)) ? 16 : 4;
    if (k > 64) k = 64;
    return (int)k;
}

// Iterations of Algorithm 2 on level L after bicg_start: the Bi-CG vectors r, r*, p, p*, q, q*
// have type T, the iterate x type TX.  Sweep A forms p, p* and their products with A (and
// sigma), sweep B updates x, r, r* (and rho, r.r).  Every kernel returns at once when the
// run has stopped, so the host launches K iterations between two polls of the state.
bool g_cg = false;          // current solve uses the CG specialisation (opts.method)
bool g_graphs = false;      // replay iteration windows from captured hipGraphs (solves only)
hipStream_t g_capture = nullptr;

// Captured windows of K iterations, per level, vector type, method and iterate pointer.
// Options of Algorithm 2 for the run in progress (FP64 Bi-CG only): the diagonal of a
// preconditioner M, and the dual iterate x* (updated with the shadow directions).
struct RunVariant {
    const double *d = nullptr;
    double *xs = nullptr;
};
RunVariant g_var;

// Bi-CG on large 3D grids (plain Algorithm 2, folded finalisations, an FP64 iterate) takes
// the recomputing form: its update sweep marches p and p* again for q and q* instead of
// reading them back (mixed: 64 instead of 72 bytes per unknown and iteration, 58 with the
// paired x updates; FP64: 112 instead of 136, 106 paired).  The CG specialisation keeps the stored form: its streaming update sweep
// is cheap, and a second march cost more than the 16 bytes it saves (measured at 512^3:
// FP64 CG 704 -> 807 ms, mixed 480 -> 477 ms).  Smaller grids keep the stored form (mixed: x's update deferred to the
// next sweep A from 2^17 unknowns up): there a second march per iteration costs more
// latency than the bytes it saves (measured, mixed: 128^3 level 81.9 ms stored, 88.0 ms
// recomputing; 256^3: 532.0 and 513.7 ms; FP64 256^3: 874.7 and 843.9 ms).  With the paired
// x updates and the alternating march directions FP64 vectors gain from 2^20 unknowns on
// (128^3 level of the 512^3 solve: 102.6 ms stored, 89.1 ms recomputing; 64^3: 22.8 and
// 23.5 ms), FP32 vectors still from 2^22 (128^3: 77.7 and 80.1 ms).
constexpr long long kRecomputeMin = 1LL << 22;     // FP32 vectors
constexpr long long kRecomputeMin64 = 1LL << 20;   // FP64 vectors
long long g_rq_min = 0;   // opts.recompute_min_unknowns of the solve in progress (0: defaults)

inline long long recompute_min(bool fp64) {
    return g_rq_min > 0 ? g_rq_min : (fp64 ? kRecomputeMin64 : kRecomputeMin);
}

template <typename TX, typename T>
bool recompute_q(const Level &L) {
    return sizeof(TX) == 8 && !g_cg && !g_var.d && !g_var.xs && g_ctx.dim == 3 &&
           L.nu >= recompute_min(sizeof(T) == 8);
}

// Partials (per value) that the update sweep of level L leaves for the next sweep A.
// The geometry of the FP32 recomputing sweeps of level L (two points per lane when the
// level takes them).
inline const Geom &rq_geom_f32(const Level &L) { return L.wide ? L.g2w : L.g2f; }

template <typename TX, typename T>
int b_partials(const Level &L) {
    return recompute_q<TX, T>(L) ? stencil_blocks(sizeof(T) == 4 ? rq_geom_f32(L) : L.g2)
                                 : update_blocks(L.nu);
}

struct GraphEntry {
    int level, tsize, cg, K, defer, ld, rq, wide;
    const void *x, *d, *xs;
    hipGraph_t graph;
    hipGraphExec_t exec;
};
std::vector<GraphEntry> g_graph_cache;

void release_graphs() {
    for (GraphEntry &e : g_graph_cache) {
        (void)hipGraphExecDestroy(e.exec);
        (void)hipGraphDestroy(e.graph);
    }
    g_graph_cache.clear();
}

// The launches of iteration j of a run: sweep A (direction update + products + sigma) and
// sweep B (updates + rho, r.r); the finalisations (alpha, beta, the stopping checks) are
// folded into the sweeps, so two launches.  Forms: the recomputing
// one on large 3D grids (recompute_q: sweep A stores p, p* only, sweep B forms q, q* again),
// else the stored one (q, q* written by sweep A, read by sweep B).  ev >= 0 brackets the
// sweeps with timing events.
// defer (stored form): 0 = sweep B updates x; 1 = x's update is left to the next sweep A
// (deferred), this sweep A has none pending (first launch of a run or of a resumed run);
// 2 = deferred, and this sweep A applies the pending update of iteration j-1.  Deferral:
// FP32 vectors, FP64 iterate, Bi-CG with folded finalisations and no options.
// defer (recomputing form, single-point sweeps): paired updates of x.  Sweep B of an odd
// iteration leaves x alone and sweep B of the next (even) one applies both updates, so x
// streams once per two iterations (plus the previous direction); a sweep A of an even
// iteration that stops the run applies the update owed.  0 = x += alpha p in every sweep B;
// 1 = the first launch of a run or of a resumed run (at even j: x += alpha p, nothing owed
// before it); 2 = steady state.
template <typename TX, typename T>
int launch_iteration(const Level &L, TX *x, long long j, int ev, hipStream_t st, int defer = 0) {
    Ctx &c = g_ctx;
    BicgState *S = c.state.as<BicgState>();
    T *r = c.r.as<T>(), *rs = c.rs.as<T>(), *q = c.q.as<T>(), *qs = c.qs.as<T>();
    // the recomputing form's FP32 sweeps may take two points per lane; every other sweep
    // keeps the level's single-point FP32 or FP64 shape
    const Geom &G = sizeof(T) == 4 ? (recompute_q<TX, T>(L) ? rq_geom_f32(L) : L.g2f) : L.g2;
    // FP32 vectors (and the iterate solved with them) have the level's row layout
    const Rows rows = sizeof(T) == 4 ? L.rows() : Rows{};
    const int nsb = stencil_blocks(G);
    const int nvb = b_partials<TX, T>(L);
    const int cur = (int)(j & 1), nxt = cur ^ 1;
    T *pn = c.p[nxt].as<T>(), *psn = c.ps[nxt].as<T>();
    // sweep A merges the previous sweep B's partials (rho, r.r, beta, stopping checks),
    // sweep B merges sweep A's (sigma, alpha)
    StepLink la{S, c.part_b.as<Pair>(), nvb, g_cg ? 1 : 2, cur};
    StepLink lb{S, c.part_a.as<Pair>(), nsb, 1, cur};
    if (ev >= 0) CKH(hipEventRecord(g_events[4 * ev], st));
    if constexpr (sizeof(TX) == 8) {
        if (recompute_q<TX, T>(L)) {
            const int xm = defer == 0 ? 0 : ((j & 1) ? 1 : (defer == 2 ? 2 : 0));
            la.defer = xm == 2 ? 1 : 0;
            lb.defer = xm == 2 ? 1 : 0;
            CKH(stencil_dir_sigma<T>(G, G.ty, r, rs, c.p[cur].as<T>(), c.ps[cur].as<T>(),
                                     &S->beta, j == 0 ? 1 : 0, pn, psn, c.part_a.as<Pair>(),
                                     &S->status, st, la, xm == 2 ? x : nullptr,
                                     xm == 2 ? &S->alpha : nullptr, sizeof(T) == 4 && !L.wide));
            if (ev >= 0) CKH(hipEventRecord(g_events[4 * ev + 1], st));
            if (ev >= 0) CKH(hipEventRecord(g_events[4 * ev + 2], st));
            CKH(stencil_pair_update<T>(G, G.ty, pn, psn, x, r, rs, c.part_b.as<Pair>(),
                                       &S->status, &S->alpha, st, lb, xm,
                                       xm == 2 ? c.p[cur].as<T>() : nullptr,
                                       xm == 2 ? &S->alpha_slot[cur ^ 1] : nullptr,
                                       sizeof(T) == 8 && L.nu < kDownMaxUnknowns));
            if (ev >= 0) CKH(hipEventRecord(g_events[4 * ev + 3], st));
            return EXCMG_OK;
        }
    }
    if constexpr (sizeof(T) == 8 && sizeof(TX) == 8) {
        if (g_var.d || g_var.xs) {  // Algorithm 2 with its options
            if (g_var.d)
                CKH(stencil_pair_direction_m(G, G.ty, r, rs, c.p[cur].as<T>(), c.ps[cur].as<T>(),
                                             g_var.d, &S->beta, j == 0 ? 1 : 0, pn, psn, q, qs,
                                             c.part_a.as<Pair>(), &S->status, st, la));
            else
                CKH(stencil_pair_direction<T>(G, G.ty, r, rs, c.p[cur].as<T>(), c.ps[cur].as<T>(),
                                              &S->beta, j == 0 ? 1 : 0, pn, psn, q, qs,
                                              c.part_a.as<Pair>(), &S->status, st, la));
            if (ev >= 0) CKH(hipEventRecord(g_events[4 * ev + 1], st));
            if (ev >= 0) CKH(hipEventRecord(g_events[4 * ev + 2], st));
            CKH(bicg_update_ex(L.nu, S, x, pn, r, q, rs, qs, g_var.d, g_var.xs, psn,
                               c.part_b.as<Pair>(), st, lb));
            if (ev >= 0) CKH(hipEventRecord(g_events[4 * ev + 3], st));
            return EXCMG_OK;
        }
    }
    if (defer == 2) {
        la.defer = 1;
        if constexpr (sizeof(T) == 4 && sizeof(TX) == 8)
            CKH(stencil_pair_direction_x(G, G.ty, r, rs, c.p[cur].as<T>(), c.ps[cur].as<T>(),
                                         &S->beta, pn, psn, q, qs, c.part_a.as<Pair>(),
                                         &S->status, x, &S->alpha, st, la));
        else
            return fail(EXCMG_EINVAL, "deferred update needs FP32 vectors and an FP64 iterate");
    } else if (g_cg)
        CKH(stencil_direction<T>(G, G.ty, r, c.p[cur].as<T>(), &S->beta, j == 0 ? 1 : 0, pn, q,
                                 c.part_a.as<Pair>(), &S->status, st, la));
    else
        CKH(stencil_pair_direction<T>(G, G.ty, r, rs, c.p[cur].as<T>(), c.ps[cur].as<T>(),
                                      &S->beta, j == 0 ? 1 : 0, pn, psn, q, qs,
                                      c.part_a.as<Pair>(), &S->status, st, la));
    if (ev >= 0) CKH(hipEventRecord(g_events[4 * ev + 1], st));
    if (ev >= 0) CKH(hipEventRecord(g_events[4 * ev + 2], st));
    if (g_cg)
        CKH((cg_update<TX, T>(L.nu, S, x, pn, r, q, c.part_b.as<Pair>(), st, lb, rows)));
    else
        CKH((bicg_update<TX, T>(L.nu, S, defer ? nullptr : x, pn, r, q, rs, qs,
                                c.part_b.as<Pair>(), st, lb, rows)));
    if (ev >= 0) CKH(hipEventRecord(g_events[4 * ev + 3], st));
    return EXCMG_OK;
}

// The folded steps leave the end-of-iteration checks of iteration j to the next sweep A; before
// the host reads the state, run them on their own (the next sweep A repeats them with the
// same result).
// With a deferred update pending the check only publishes its decision (poll_status): the
// next sweep A stops the run after applying the update.
template <typename T>
int close_window(const Level &L, long long j_next, hipStream_t st, int defer = 0) {
    Ctx &c = g_ctx;
    const StepLink l{c.state.as<BicgState>(), c.part_b.as<Pair>(), b_partials<double, T>(L), g_cg ? 1 : 2,
                     (int)(j_next & 1), defer ? 1 : 0};
    CKH(step_check(l, st));
    return EXCMG_OK;
}

// Graph of iterations j = 1..K (K even, so the p / p* buffer parity repeats).  defer: 0
// none, 1 the stored form's deferred update, 2 the recomputing form's paired updates (a
// window ends at an even iteration, where x owes nothing, so its closing check stops the
// run itself).
template <typename TX, typename T>
int window_graph(const Level &L, TX *x, int K, hipGraphExec_t *out, int defer = 0) {
    for (GraphEntry &e : g_graph_cache)
        if (e.level == L.index && e.tsize == (int)sizeof(T) && e.cg == (int)g_cg &&
            e.K == K && e.defer == defer && e.ld == L.ld &&
            e.rq == (int)recompute_q<TX, T>(L) && e.wide == (int)L.wide &&
            e.x == (const void *)x &&
            e.d == g_var.d && e.xs == g_var.xs) {
            *out = e.exec;
            return EXCMG_OK;
        }
    if (!g_capture) CKH(hipStreamCreateWithFlags(&g_capture, hipStreamNonBlocking));
    CKH(hipStreamBeginCapture(g_capture, hipStreamCaptureModeRelaxed));
    int rc = EXCMG_OK;
    for (int t = 0; t < K && rc == EXCMG_OK; t++)
        rc = launch_iteration<TX, T>(L, x, 1 + t, -1, g_capture, defer ? 2 : 0);
    if (rc == EXCMG_OK) rc = close_window<T>(L, K + 1, g_capture, defer == 1 ? 1 : 0);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(g_capture, &graph);
    if (rc != EXCMG_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    CKH(e);
    hipGraphExec_t exec = nullptr;
    CKH(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    g_graph_cache.push_back(GraphEntry{L.index, (int)sizeof(T), (int)g_cg, K, defer,
                                       L.ld, (int)recompute_q<TX, T>(L), (int)L.wide,
                                       (const void *)x, g_var.d, g_var.xs, graph, exec});
    *out = exec;
    return EXCMG_OK;
}

// Iterations of Algorithm 2 on level L after bicg_start: the Bi-CG vectors r, r*, p, p*, q, q*
// have type T, the iterate x type TX.  Every kernel returns at once when the run has stopped,
// so the host issues K iterations between two polls of the state: directly, or (in solves)
// as the replay of a captured K-iteration graph after the first iteration.  j is the index
// of the next iteration (0 starts the run; a run resumed after its residuals were replaced
// continues at the j it stopped at, with its search directions).
template <typename TX, typename T>
int bicg_iterate(const Level &L, TX *x, BicgState &hs, long long &j) {
    int K = poll_interval(L.nu, g_ctx.dim);
    K += K & 1;
    if (g_timing) CKR(ensure_events(4 * (size_t)(K + 1)));
    const bool graphs = g_graphs && !g_timing;
    // x += alpha p deferred to the next sweep A (large grids, FP32 vectors, plain Bi-CG):
    // sweep B then streams r, q, r*, q* only
    const int defer = (!recompute_q<TX, T>(L) && (graphs || g_timing) && K <= 16 && sizeof(T) == 4 &&
                       sizeof(TX) == 8 && !g_cg && !g_var.d && !g_var.xs &&
                       g_ctx.dim == 3) ? 1 : 0;
    // the recomputing form's paired updates of x (single-point sweeps); windows of
    // iterations start at odd j, so each ends at an even one with x up to date
    const int paired = (recompute_q<TX, T>(L) && (graphs || g_timing) &&
                        (sizeof(T) == 8 || !L.wide)) ? 1 : 0;
    hipGraphExec_t exec = nullptr;
    if (graphs) CKR((window_graph<TX, T>(L, x, K, &exec, defer ? 1 : (paired ? 2 : 0))));
    if (graphs && K <= 16 && hs.status == kRunning) {
        // Short windows (large grids): queue window w+1 before reading the state of window
        // w, so the device never waits for the host.  The window after the one that stopped
        // the run consists of no-op launches (with a deferred update, its first sweep A
        // applies the update and stops the run).
        Ctx &c = g_ctx;
        if (defer) {
            // the first sweep A of a run, or of a resumed run, has no update pending
            CKR((launch_iteration<TX, T>(L, x, j, -1, g_stream, 1)));
            j++;
            if ((j & 1) == 0) {   // the captured window starts at an odd iteration
                CKR((launch_iteration<TX, T>(L, x, j, -1, g_stream, 2)));
                j++;
            }
        } else if (j == 0 || (j & 1) == 0) {
            CKR((launch_iteration<TX, T>(L, x, j, -1, g_stream)));
            j++;
        }
        auto queue_window = [&](int slot) -> int {
            CKH(hipGraphLaunch(exec, g_stream));
            CKH(hipMemcpyAsync(c.host_state + 1 + slot, c.state.p, sizeof(BicgState),
                               hipMemcpyDeviceToHost, g_stream));
            CKH(hipEventRecord(c.poll_ev[slot], g_stream));
            j += K;
            return EXCMG_OK;
        };
        CKR(queue_window(0));
        for (int w = 0;; w++) {
            CKR(queue_window((w + 1) & 1));
            CKH(hipEventSynchronize(c.poll_ev[w & 1]));
            if (c.host_state[1 + (w & 1)].poll_status != kRunning) break;
        }
        CKR(read_state(hs));
        if (hs.status == kStopping) hs.status = hs.poll_status;  // (a sweep B always follows)
        return EXCMG_OK;
    }
    bool seg_first = true;
    while (hs.status == kRunning) {
        const int it0 = hs.iter;
        if (graphs) {
            // the captured window holds iterations of odd index first
            if (j == 0 || (j & 1) == 0) {
                CKR((launch_iteration<TX, T>(L, x, j, -1, g_stream)));
                j++;
            }
            CKH(hipGraphLaunch(exec, g_stream));
            j += K;
        }
        int plain_first = 0;   // timed window starting with a sweep A that owes no update
        int Kw = K;            // iterations in this window
        const long long j0 = j;
        if (!graphs) {
            plain_first = ((defer || paired) && seg_first) ? 1 : 0;
            // paired updates: a window that starts at an even iteration takes one more, so
            // that it ends at an even one
            if (paired && (j & 1) == 0) Kw = K + 1;
            for (int t = 0; t < Kw; t++, j++) {
                // with a deferred update, the first sweep A of the call has none pending
                const int dm = (defer || paired) ? (seg_first ? 1 : 2) : 0;
                seg_first = false;
                CKR((launch_iteration<TX, T>(L, x, j, g_timing ? t : -1, g_stream, dm)));
            }
            CKR(close_window<T>(L, j, g_stream, defer));
        }
        CKR(read_state(hs));
        if (defer && hs.status == kRunning && hs.poll_status != kRunning) {
            // the closing check found the stop: one more sweep A applies the owed update
            CKR((launch_iteration<TX, T>(L, x, j, -1, g_stream, 2)));
            j++;
            CKR(read_state(hs));
        }
        if (hs.status == kStopping) hs.status = hs.poll_status;
        if (g_timing && L.index < EXCMG_MAX_LEVELS) {
            const int active = std::min(Kw, hs.iter - it0);  // launches that did work
            for (int t = 0; t < active; t++) {
                float a = 0.f, b2 = 0.f;
                CKH(hipEventElapsedTime(&a, g_events[4 * t], g_events[4 * t + 1]));
                CKH(hipEventElapsedTime(&b2, g_events[4 * t + 2], g_events[4 * t + 3]));
                const bool lead = (t == 0 && plain_first);
                const int ka = (defer && !lead) ? 2 : 0;
                // paired updates: odd iterations leave x, even ones (but a leading one) apply two
                const int kb = !paired ? 1 : (((j0 + t) & 1) ? 3 : (lead ? 1 : 4));
                g_time_ms[L.index][ka] += a;
                g_time_ms[L.index][kb] += b2;
                g_time_n[L.index][ka]++;
                g_time_n[L.index][kb]++;
            }
        }
    }
    return EXCMG_OK;
}

// One Bi-CG run from x (in place) on level L with right-hand side b.
// One run of Algorithm 2 from x (in place) on level L with right-hand side b.  Options: d,
// the diagonal of a preconditioner M (NULL: M = I); the shadow system, either bstar and
// xstar (r*_0 = b* - A^T x*_0, x* updated in place) or shadow (r*_0 = shadow), else
// r*_0 = r_0.  A^T is applied as A (A_h is exactly symmetric).
int bicg_run(const Level &L, const double *b, double *x, double eps, int maxit, int *iters,
             double *rr_out, int *status_out, const double *d = nullptr,
             const double *shadow = nullptr, const double *bstar = nullptr,
             double *xstar = nullptr) {
    Ctx &c = g_ctx;
    BicgState *S = c.state.as<BicgState>();
    double *r = c.r.as<double>(), *rs = c.rs.as<double>();
    // b.b and r_0 = b - A x_0
    CKR(device_dot(L.nu, b, b, (double *)&S->bb, 0));
    CKH(stencil_residual<double>(L.g1, L.g1.ty, b, x, r, c.part_a.as<Pair>(), g_stream));
    if (!d && !shadow && !bstar) {
        // r*_0 = r_0 and rho_0 = r_0.r_0
        CKH((copy_convert<double, double>(L.nu, r, rs, g_stream)));
        CKH(bicg_start(S, c.part_a.as<Pair>(), stencil_blocks(L.g1), eps, maxit, g_stream));
    } else {
        if (bstar)
            CKH(stencil_residual<double>(L.g1, L.g1.ty, bstar, xstar, rs, c.part_b.as<Pair>(),
                                         g_stream));
        else
            CKH((copy_convert<double, double>(L.nu, shadow ? shadow : r, rs, g_stream)));
        // rho_0 = r*_0 . M^-1 r_0
        CKH(rho_partials<double>(L.nu, r, rs, c.part_b.as<Pair>(), g_stream, d));
        CKH(bicg_start2(S, c.part_b.as<Pair>(), update_blocks(L.nu), eps, maxit, g_stream));
    }
    BicgState hs;
    CKR(read_state(hs));
    long long j = 0;
    g_var = RunVariant{d, bstar ? xstar : nullptr};
    const int rc = bicg_iterate<double, double>(L, x, hs, j);
    g_var = RunVariant{};
    CKR(rc);
    if (iters) *iters = hs.iter;
    if (rr_out) *rr_out = hs.rr;
    if (status_out) *status_out = hs.status;
    return EXCMG_OK;
}

// diag(A_h) of level L (the Jacobi choice of M), made once per context
const double *level_diagonal(Level &L) {
    if (!L.diag.p) {
        if (L.diag.ensure((size_t)L.nu * 8) != EXCMG_OK) return nullptr;
        if (operator_diagonal(L.n, g_ctx.bc == 1 ? 1.0 : -1.0, L.diag.as<double>(), g_stream,
                              g_ctx.dim) != hipSuccess)
            return nullptr;
    }
    return L.diag.as<double>();
}

// Algorithm 1's while loop on one level.
int level_solve(const Level &L, const double *b, double *x, double eps, int maxit, int max_runs,
                excmg_level_stats *st, const double *d = nullptr) {
    Ctx &c = g_ctx;
    double *sc = c.scal.as<double>();
    CKR(device_dot(L.nu, b, b, sc, 1));
    CKR(true_residual(L, b, x, c.r.as<double>(), 2));
    CKH(hipMemcpyAsync(c.host_scal, sc, 3 * sizeof(double), hipMemcpyDeviceToHost, g_stream));
    CKH(hipStreamSynchronize(g_stream));
    const double bb = c.host_scal[1];
    double rr = c.host_scal[2];
    const double thr = (eps * eps) * bb;
    int total = 0, runs = 0, status = EXCMG_OK;
    double floor = 0.0;
    while (!(rr <= thr)) {
        if (runs >= max_runs) {
            status = EXCMG_ENOCONV;
            break;
        }
        int it = 0, bst = 0;
        double rrr = 0.0;
        CKR(bicg_run(L, b, x, eps, maxit, &it, &rrr, &bst, d));
        total += it;
        runs++;
        const double prev = rr;
        CKR(true_residual(L, b, x, c.r.as<double>(), 2));
        CKH(hipMemcpyAsync(c.host_scal + 2, sc + 2, sizeof(double), hipMemcpyDeviceToHost,
                           g_stream));
        CKH(hipStreamSynchronize(g_stream));
        rr = c.host_scal[2];
        if (bst == kBreakdown) {
            status = EXCMG_EBREAKDOWN;
            break;
        }
        // a tolerance near the FP64 floor: stop once a run no longer halves the residual
        if (!(rr <= thr)) {
            CKR(level_floor(L, x, Rows{}, bb, &floor));
            if (eps < 10.0 * floor && !(rr < 0.5 * prev)) {
                status = EXCMG_ENOCONV;
                break;
            }
        }
    }
    if (st) {
        st->n = L.N;
        st->iterations = total;
        st->runs = runs;
        st->status = status;
        st->eps = eps;
        st->rel_residual = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
        if (floor == 0.0) CKR(level_floor(L, x, Rows{}, bb, &floor));
        st->floor = floor;
        st->exit = level_exit(status, eps, floor);
    }
    return EXCMG_OK;
}

// ------------------------------------------------------------------ mixed precision

// One FP32 Bi-CG run for A e = r32 (r32 = r*32 already written by the outer residual), e
// starting at 0 and accumulated directly into the FP64 iterate u (u + e is the refined
// solution).  Vectors FP32, scalars and dot products FP64.  Stops at the relative
// recurrence residual inner_tol.
int bicg_inner_fp32(const Level &L, double *u, double inner_tol, int maxit, int *iters,
                    int *status_out) {
    Ctx &c = g_ctx;
    BicgState *S = c.state.as<BicgState>();
    float *r = c.r.as<float>();
    const int nvb = vec_blocks(L.nu);
    CKH(dot_partials<float>(L.nu, r, r, c.part_b.as<Pair>(), nvb, g_stream, L.rows()));
    CKH(reduce_to((double *)&S->bb, c.part_b.as<Pair>(), nvb, 0, g_stream));
    CKH(bicg_start(S, c.part_b.as<Pair>(), nvb, inner_tol, maxit, g_stream));
    BicgState hs;
    CKR(read_state(hs));
    long long j = 0;
    CKR((bicg_iterate<double, float>(L, u, hs, j)));
    if (iters) *iters = hs.iter;
    if (status_out) *status_out = hs.status;
    return EXCMG_OK;
}

// The mixed-precision solvers work on the level's row layout (L.ld): b and u are padded
// into the context's copies first when the rows are padded, and u is copied back after.
template <class Solve>
int with_level_rows(const Level &L, const double *b, double *u, Solve solve) {
    if (L.ld == L.n) return solve(b, u);
    Ctx &c = g_ctx;
    double *bp = c.bp.as<double>(), *xp = c.xp.as<double>();
    CKH(pad_rows(L.n, L.ld, b, bp, g_stream));
    CKH(pad_rows(L.n, L.ld, u, xp, g_stream));
    CKR(solve(bp, xp));
    CKH(unpad_rows(L.n, L.ld, xp, u, g_stream));
    return EXCMG_OK;
}

// Iterative refinement on one level: r = b - A u in FP64 (rounded to FP32 for the inner
// solve), FP32 Bi-CG correction added to u in FP64, until ||b - A u||_2 <= eps ||b||_2 in
// FP64.  Stops early (EXCMG_ENOCONV) if an outer step fails to reduce the FP64 residual.
// b and u have the level's row layout.
int level_solve_mixed(const Level &L, const double *b, double *u, double eps, int maxit,
                      int max_outer, double inner_tol, excmg_level_stats *st) {
    Ctx &c = g_ctx;
    double *sc = c.scal.as<double>();
    CKR(device_dot(L.nu, b, b, sc, 1, L.rows()));
    const int nrb = stencil_blocks(L.g1p);
    int total = 0, outer = 0, status = EXCMG_OK;
    double bb = 0.0, rr = 0.0, prev = INFINITY;
    for (;;) {
        CKH(stencil_residual_cast(L.g1p, L.g1p.ty, b, u, c.r.as<float>(), c.rs.as<float>(),
                                  c.part_a.as<Pair>(), g_stream));
        CKH(reduce_to(sc, c.part_a.as<Pair>(), nrb, 2, g_stream));
        CKH(hipMemcpyAsync(c.host_scal, sc, 3 * sizeof(double), hipMemcpyDeviceToHost, g_stream));
        CKH(hipStreamSynchronize(g_stream));
        bb = c.host_scal[1];
        rr = c.host_scal[2];
        if (rr <= (eps * eps) * bb) break;
        if (outer >= max_outer || !(rr < prev)) {
            status = EXCMG_ENOCONV;
            break;
        }
        prev = rr;
        // no need to solve the correction much more accurately than the outer target
        double it = std::max(inner_tol, 0.3 * eps * std::sqrt(bb / rr));
        if (it > 0.5) it = 0.5;
        int its = 0, bst = 0;
        CKR(bicg_inner_fp32(L, u, it, maxit, &its, &bst));
        total += its;
        outer++;
        if (bst == kBreakdown) {
            status = EXCMG_EBREAKDOWN;
            break;
        }
    }
    if (st) {
        double floor = 0.0;
        CKR(level_floor(L, u, L.rows(), bb, &floor));
        st->n = L.N;
        st->iterations = total;
        st->runs = outer;
        st->status = status;
        st->eps = eps;
        st->rel_residual = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
        st->floor = floor;
        st->exit = level_exit(status, eps, floor);
    }
    return EXCMG_OK;
}

// Mixed precision with residual replacement (reliable updates).  An FP32 Bi-CG run for
// A e = r adds its correction directly into the FP64 iterate u (sweep B).  Whenever the
// run's recurrence residual has fallen by the factor delta since the last replacement (or
// below half the target), the FP64 residual b - A u replaces r and r* (rounded to FP32),
// rho is taken from the new vectors and the run goes on with its search directions:
// unlike restarted refinement, the Krylov space built so far is kept.  The best iterate so
// far is kept aside: if a stretch of the run made the FP64 residual larger (or a run that
// has been replaced into breaks down), u goes back to it and a fresh run starts from there
// (a breakdown of a fresh run is reported).  Stops when ||b - A u||_2 <= eps ||b||_2 in FP64,
// when two replacements in a row fail to halve the squared residual, or at the caps.
// b and u have the level's row layout.
int level_solve_reliable(const Level &L, const double *b, double *u, double eps, int maxit,
                         int max_outer, double delta, excmg_level_stats *st) {
    Ctx &c = g_ctx;
    BicgState *S = c.state.as<BicgState>();
    double *sc = c.scal.as<double>(), *ub = c.ubest.as<double>();
    float *r = c.r.as<float>(), *rs = c.rs.as<float>();
    const Rows rows = L.rows();
    const int nrb = stencil_blocks(L.g1p), nvb = vec_blocks(L.nu);
    const size_t ubytes = (size_t)L.nflat * 8;
    CKR(device_dot(L.nu, b, b, sc, 1, rows));
    // FP64 residual of u (rounded into r and r*), its square norm, and b.b
    auto true_residual = [&](double &bb, double &rr) -> int {
        CKH(stencil_residual_cast(L.g1p, L.g1p.ty, b, u, r, rs, c.part_a.as<Pair>(), g_stream));
        CKH(reduce_to(sc, c.part_a.as<Pair>(), nrb, 2, g_stream));
        CKH(hipMemcpyAsync(c.host_scal, sc, 3 * sizeof(double), hipMemcpyDeviceToHost, g_stream));
        CKH(hipStreamSynchronize(g_stream));
        bb = c.host_scal[1];
        rr = c.host_scal[2];
        return EXCMG_OK;
    };
    double bb = 0.0, rr = 0.0;
    CKR(true_residual(bb, rr));
    const double target = (eps * eps) * bb;
    int status = EXCMG_OK, replaced = 0, iters = 0, done = 0, weak = 0;
    BicgState hs;
    long long j = 0;
    int since_start = 0;  // replacements in the current run
    // fresh run on the current residual: rho_0 = r.r of the FP32 copy
    auto start_run = [&]() -> int {
        CKH(dot_partials<float>(L.nu, r, r, c.part_b.as<Pair>(), nvb, g_stream, rows));
        CKH(reduce_to((double *)&S->bb, c.part_b.as<Pair>(), nvb, 0, g_stream));
        CKH(bicg_start(S, c.part_b.as<Pair>(), nvb, delta, std::max(1, maxit - done), g_stream));
        CKH(state_resume(S, std::max((delta * delta) * rr, 0.25 * target), g_stream));
        CKR(read_state(hs));
        j = 0;
        since_start = 0;
        return EXCMG_OK;
    };
    if (!(rr <= target)) {
        CKH(hipMemcpyAsync(ub, u, ubytes, hipMemcpyDeviceToDevice, g_stream));
        CKR(start_run());
        double best = rr;
        for (;;) {
            CKR((bicg_iterate<double, float>(L, u, hs, j)));
            iters = done + hs.iter;
            const bool broke = (hs.status == kBreakdown);
            CKR(true_residual(bb, rr));
            if (rr <= target) break;
            const bool better = std::isfinite(rr) && rr < best;
            weak = (better && rr < 0.5 * best) ? 0 : weak + 1;
            if (better) {
                best = rr;
                CKH(hipMemcpyAsync(ub, u, ubytes, hipMemcpyDeviceToDevice, g_stream));
            } else {
                // back to the best iterate; r and r* again hold its residual
                CKH(hipMemcpyAsync(u, ub, ubytes, hipMemcpyDeviceToDevice, g_stream));
                CKR(true_residual(bb, rr));
                if (broke && since_start == 0) {
                    status = EXCMG_EBREAKDOWN;
                    break;
                }
            }
            if ((!broke && hs.status == kNoConv) || iters >= maxit || replaced >= max_outer ||
                weak >= 2) {
                status = EXCMG_ENOCONV;
                break;
            }
            replaced++;
            if (broke || !better) {
                done = iters;
                CKR(start_run());
                continue;
            }
            since_start++;
            CKH(rho_partials<float>(L.nu, r, rs, c.part_b.as<Pair>(), g_stream, nullptr, rows,
                                    b_partials<double, float>(L)));
            CKH(state_resume(S, std::max((delta * delta) * rr, 0.25 * target), g_stream));
            CKR(read_state(hs));
            // the run stopped inside the last window: go on from the iteration it reached
            // (that index selects the direction buffers and the rho slots)
            j = hs.iter;
        }
    }
    if (st) {
        double floor = 0.0;
        CKR(level_floor(L, u, rows, bb, &floor));
        st->n = L.N;
        st->iterations = iters;
        st->runs = replaced;
        st->status = status;
        st->eps = eps;
        st->rel_residual = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
        st->floor = floor;
        st->exit = level_exit(status, eps, floor);
    }
    return EXCMG_OK;
}

double level_tolerance(double tol, int i, int L) {
    double p = 1.0;
    for (int t = 0; t < L - i; t++) p *= 10.0;
    return tol / p;
}

// Algorithm 1.  f, g1, g2 are device node arrays of the finest grid.  Bi-CG levels run in
// FP64 or as FP32 Bi-CG inside FP64 iterative refinement (opts.precision, opts.refine).
int solve_cascade(const excmg_opts &o, const double *f, const double *g1, const double *g2,
                  double *u_out, double *ut_out, excmg_stats *st) {
    Ctx &c = g_ctx;
    const int nl = o.n_levels, Nf = o.n_finest;
    const int L = nl - 2;
    const int maxit = o.max_iters > 0 ? o.max_iters : 100000;
    const int max_runs = o.max_runs > 0 ? o.max_runs : 5;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 60;
    const bool reliable = o.refine == EXCMG_RELIABLE;
    const bool jacobi = (o.precond == EXCMG_PRECOND_JACOBI);
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : (reliable ? 0.1 : 1e-4);
    const bool mixed = (o.precision == EXCMG_MIXED);
    if (c.dim == 3) {
        // padded rows: the FP64 copies of b and u they are solved with, made on first use
        long long flat = 0;
        for (Level &Lv : c.lv) {
            // row_pad 2: padded rows and two-point sweeps on the levels that take the
            // recomputing form
            Lv.wide = mixed && o.row_pad == 2 && Lv.nu >= recompute_min(false) && Lv.g2w.tw != 0;
            set_rows(Lv, level_ld(Lv.n, mixed && (o.row_pad == 1 || Lv.wide) ? 1 : 0), c.dim);
            if (Lv.ld != Lv.n) flat = std::max(flat, Lv.nflat);
        }
        if (flat > 0) {
            CKR(c.xp.ensure((size_t)flat * 8));
            CKR(c.bp.ensure((size_t)flat * 8));
            CKR(c.ubest.ensure((size_t)std::max(flat, c.lv.back().nu) * 8));
        }
    }
    hipEvent_t ev0, ev1, evl0, evl1;
    CKH(hipEventCreate(&ev0));
    CKH(hipEventCreate(&ev1));
    CKH(hipEventCreate(&evl0));
    CKH(hipEventCreate(&evl1));
    CKH(hipEventRecord(ev0, g_stream));
    int worst = EXCMG_OK;
    for (int l = 0; l < nl; l++) {
        Level &Lv = c.lv[l];
        const int s = 1 << (nl - 1 - l);
        excmg_level_stats ls{};
        ls.n = Lv.N;
        CKH(hipEventRecord(evl0, g_stream));
        if (c.dim == 2) CKH(rhs_assemble_2d(Lv.N, c.bc, s, Nf, f, g1, g2, Lv.b.as<double>(), g_stream));
        else CKH(rhs_assemble(Lv.N, c.bc, s, Nf, f, g1, g2, Lv.b.as<double>(), g_stream));
        if (l <= 1) {
            CKH(band_solve((int)Lv.nu, c.chol_w[l], c.chol[l].as<double>(), Lv.b.as<double>(),
                           Lv.x.as<double>(), g_stream));
            ls.status = EXCMG_OK;
        } else {
            if (c.dim == 2) {
                CKH(exp_finite_2d(Lv.N, c.lv[l - 1].u.as<double>(), c.lv[l - 2].u.as<double>(),
                                  c.vz1.as<double>(), Lv.u.as<double>(), g_stream));
                CKH(from_nodes_2d(Lv.N, Lv.u.as<double>(), Lv.x.as<double>(), g_stream));
            } else {
                CKH(exp_finite(Lv.N, c.lv[l - 1].u.as<double>(), c.lv[l - 2].u.as<double>(),
                               c.vz1.as<double>(), Lv.u.as<double>(), g_stream));
                CKH(from_nodes(Lv.N, Lv.u.as<double>(), Lv.x.as<double>(), g_stream));
            }
            const double eps = level_tolerance(o.tol, l - 1, L);
            // small levels run FP64 Bi-CG: they are bound by launch latency, so FP32 vectors
            // save nothing and the refinement costs extra (default: with residual
            // replacement below 2^18 unknowns; restarted refinement on every level)
            const long long fp32_min = o.fp32_min_unknowns > 0 ? o.fp32_min_unknowns
                                                               : (reliable ? (1LL << 18) : 1);
            const bool lmixed = mixed && Lv.nu >= fp32_min;
            if (lmixed && reliable)
                CKR(with_level_rows(Lv, Lv.b.as<double>(), Lv.x.as<double>(),
                                    [&](const double *b, double *u) {
                                        return level_solve_reliable(Lv, b, u, eps, maxit,
                                                                    max_outer, inner_tol, &ls);
                                    }));
            else if (lmixed)
                CKR(with_level_rows(Lv, Lv.b.as<double>(), Lv.x.as<double>(),
                                    [&](const double *b, double *u) {
                                        return level_solve_mixed(Lv, b, u, eps, maxit, max_outer,
                                                                 inner_tol, &ls);
                                    }));
            else
                CKR(level_solve(Lv, Lv.b.as<double>(), Lv.x.as<double>(), eps, maxit, max_runs,
                                &ls, jacobi ? level_diagonal(Lv) : nullptr));
            if (ls.status != EXCMG_OK && worst == EXCMG_OK) worst = ls.status;
        }
        if (c.dim == 2)
            CKH(to_nodes_2d<double>(Lv.N, s, Nf, Lv.x.as<double>(), g1, Lv.u.as<double>(), g_stream));
        else
            CKH(to_nodes<double>(Lv.N, s, Nf, Lv.x.as<double>(), g1, Lv.u.as<double>(), g_stream));
        CKH(hipEventRecord(evl1, g_stream));
        CKH(hipEventSynchronize(evl1));
        float ms = 0.f;
        CKH(hipEventElapsedTime(&ms, evl0, evl1));
        ls.ms = ms;
        if (st && l < EXCMG_MAX_LEVELS) st->level[l] = ls;
    }
    const Level &F = c.lv[nl - 1];
    if (ut_out) {
        if (c.dim == 2)
            CKH(exp_true_2d(Nf, F.u.as<double>(), c.lv[nl - 2].u.as<double>(), ut_out, g_stream));
        else
            CKH(exp_true(Nf, F.u.as<double>(), c.lv[nl - 2].u.as<double>(), ut_out, g_stream));
    }
    if (u_out) CKH(hipMemcpyAsync(u_out, F.u.p, F.nodes * 8, hipMemcpyDeviceToDevice, g_stream));
    CKH(hipEventRecord(ev1, g_stream));
    CKH(hipEventSynchronize(ev1));
    float ms = 0.f;
    CKH(hipEventElapsedTime(&ms, ev0, ev1));
    if (st) {
        st->n_levels = nl;
        st->total_ms = ms;
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    (void)hipEventDestroy(evl0);
    (void)hipEventDestroy(evl1);
    if (worst != EXCMG_OK)
        return fail(worst, "a level stopped before its tolerance (status %d)", worst);
    return EXCMG_OK;
}


// ================================================================== batched solves

// Cholesky factors of direct-solve levels, shared by the problems of a batch.
struct FactorCache {
    std::vector<std::pair<long long, DBuf>> f;
    int get(int N, int bc, hipStream_t st, double **out) {
        const long long key = (long long)N * 4 + bc;
        for (auto &e : f)
            if (e.first == key) {
                *out = e.second.as<double>();
                return EXCMG_OK;
            }
        f.emplace_back(key, DBuf{});
        DBuf &b = f.back().second;
        const size_t n = (size_t)(N - 1) * (N - 1) * (N - 1);
        CKR(b.ensure(n * (band_width(N, 3) + 1) * 8));
        DBuf info;
        CKR(info.ensure(64));
        const int rc = factor_band(N, bc, 3, b.as<double>(), info.as<int>(), st);
        info.release();
        if (rc != EXCMG_OK) return rc;
        *out = b.as<double>();
        return EXCMG_OK;
    }
    void release() {
        for (auto &e : f) e.second.release();
        f.clear();
    }
};

enum { kPhaseCheck = 0, kPhaseRun = 1, kPhaseDone = 2 };

// Launch shape of the batched sweep A: one tile height for the whole batch (a launch has
// one workgroup shape; 4 or 8 rows) and a z-chunk per grid size and vector precision,
// chosen by excmg_autotune_batch on the batch's own work list; sizes it has not tuned take
// the single-problem table's z-chunk.
struct BatchZc {
    int N;
    bool f32;
    int zc;
};
int g_batch_ty = kBatchTY;
std::vector<BatchZc> g_batch_zc;

int batch_zc(int N, int bc, bool f32) {
    for (const auto &e : g_batch_zc)
        if (e.N == N && e.f32 == f32) return std::max(1, std::min(e.zc, N - 1));
    return choose_shape(N, bc, f32 ? 2 : 1).zc;
}

// Sweep-A tiles of a grid of n unknowns per axis for the smallest batch tile (4 rows, 2
// planes): the size of the per-system work lists and partials whatever shape is tuned.
long long batch_max_tiles(int n) {
    return (long long)((n + kWave - 1) / kWave) * ((n + 3) / 4) * ((n + 1) / 2);
}

struct BProb {
    int N = 0, nl = 0, bc = 0, L = 0;
    std::vector<Level> lv;
    DBuf r, rs, p[2], ps[2], q, qs, part_a, part_b, ubuf;
    Arg *af = nullptr, *a1 = nullptr, *a2 = nullptr, *au = nullptr, *at = nullptr;
    int level = 0, phase = kPhaseCheck;
    bool f32 = false;           // the current level runs FP32 Bi-CG inside FP64 refinement
    int runs = 0, iters = 0, outer = 0, worst = EXCMG_OK;
    int iter_base = 0;          // the run's iteration count when it was last (re)started
    int broke = 0;              // the last run broke down (Algorithm 2's denominators)
    double eps = 0.0, prev = INFINITY, last_bb = 0.0;
    double level_bb[EXCMG_MAX_LEVELS] = {};   // b.b of each finished level
    excmg_stats stats{};
    ~BProb() {
        for (auto &l : lv) { l.b.release(); l.x.release(); l.u.release(); }
        r.release(); rs.release(); p[0].release(); p[1].release(); ps[0].release();
        ps[1].release(); q.release(); qs.release(); part_a.release(); part_b.release();
        ubuf.release();
        delete af; delete a1; delete a2; delete au; delete at;
    }
};

// The systems of a batch whose current level has vectors of one precision, advanced by
// their own step launches (work list, control block, captured graph).
struct StepSet {
    bool f32 = false;
    DBuf items, ctl;
    int2 *h_items = nullptr;
    int *h_hdr = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int grid = 0, ni = 0;
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~StepSet() {
        drop_graph();
        items.release();
        ctl.release();
        if (h_items) (void)hipHostFree(h_items);
        if (h_hdr) (void)hipHostFree(h_hdr);
    }
};

struct BatchSolver {
    bool mixed = false;
    bool reliable = true;     // FP32 levels: residual replacement (else restarted refinement)
    long long fp32_min = 1LL << 18;  // mixed: levels with fewer unknowns run FP64 Bi-CG
    bool persistent = false;  // one persistent launch per step instead of four phase launches
    int ty = kBatchTY;        // tile height of the batched sweep A
    int maxit = 100000, max_runs = 5, max_outer = 60;
    double tol = 0.0, inner_tol = 1e-5;
    hipStream_t st = nullptr;
    std::vector<BProb *> pb;
    FactorCache fc;
    DBuf states, runs, scal, xx;
    BatchRun *h_runs = nullptr;
    double *h_scal = nullptr;
    BicgState *h_states = nullptr;
    StepSet set[2];           // systems with FP64 vectors, with FP32 vectors
    // while both kinds run, the FP32 systems' steps go to a second stream (forked from and
    // joined to st by events) and run beside the FP64 systems' steps
    hipStream_t st2 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // Bi-CG steps per captured graph between two reads of the states (64 problems of
    // 32^3-128^3, one box: 4 / 8 / 16 steps, FP64 1279 / 1252 / 1237 ms, mixed 1180 / 1128 /
    // 1112 ms; another: 16 / 32 steps, FP64 1240 / 1233 ms, mixed 1117 / 1102 ms)
    int steps_per_graph = 32;
    long long launches = 0;

    ~BatchSolver() {
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (st2) (void)hipStreamDestroy(st2);
        for (BProb *b : pb) delete b;
        states.release(); runs.release(); scal.release();
        xx.release();
        fc.release();
        if (h_runs) (void)hipHostFree(h_runs);
        if (h_scal) (void)hipHostFree(h_scal);
        if (h_states) (void)hipHostFree(h_states);
    }

    bool level_f32(const BProb &b, int l) const { return mixed && b.lv[l].nu >= fp32_min; }

    BicgState *S(int j) { return states.as<BicgState>() + j; }
    double *sc(int j) { return scal.as<double>() + 4 * j; }

    int init(int nprob, const excmg_problem *probs, const excmg_opts &o) {
        mixed = (o.precision == EXCMG_MIXED);
        reliable = (o.refine == EXCMG_RELIABLE);
        fp32_min = o.fp32_min_unknowns > 0 ? o.fp32_min_unknowns : (1LL << 18);
        persistent = (o.batch_mode == 1);
        ty = g_batch_ty;
        tol = o.tol;
        maxit = o.max_iters > 0 ? o.max_iters : 100000;
        max_runs = o.max_runs > 0 ? o.max_runs : 5;
        max_outer = o.max_outer > 0 ? o.max_outer : 60;
        inner_tol = o.inner_tol > 0 ? o.inner_tol : (reliable ? 0.1 : 1e-5);
        CKR(states.ensure((size_t)nprob * sizeof(BicgState)));
        CKR(runs.ensure((size_t)nprob * sizeof(BatchRun)));
        CKR(scal.ensure((size_t)nprob * 4 * sizeof(double)));
        const int one = 1;
        for (int k = 0; k < 2; k++) {
            StepSet &S = set[k];
            S.f32 = (k == 1);
            CKR(S.ctl.ensure(sizeof(BatchCtl)));
            // epoch starts at 1: alpha_epoch[] = 0 must not read as "published" in launch 1
            CKH(hipMemsetAsync(S.ctl.p, 0, sizeof(BatchCtl), st));
            CKH(hipMemcpyAsync((char *)S.ctl.p + offsetof(BatchCtl, epoch), &one, sizeof(int),
                               hipMemcpyHostToDevice, st));
            CKH(hipHostMalloc((void **)&S.h_hdr, (4 + kMaxRuns) * sizeof(int), hipHostMallocDefault));
        }
        CKH(hipHostMalloc((void **)&h_runs, (size_t)nprob * sizeof(BatchRun), hipHostMallocDefault));
        CKH(hipHostMalloc((void **)&h_scal, (size_t)nprob * 4 * sizeof(double), hipHostMallocDefault));
        CKH(hipHostMalloc((void **)&h_states, (size_t)nprob * sizeof(BicgState), hipHostMallocDefault));
        long long max_items = 0;
        for (int j = 0; j < nprob; j++) {
            const excmg_problem &P = probs[j];
            CKR(check_sizes(P.n_finest, P.n_levels, P.bc_kind));
            if (!P.f || !P.g1 || !P.g2 || !P.u_out) return fail(EXCMG_EINVAL, "problem %d: NULL array", j);
            BProb *b = new BProb();
            pb.push_back(b);
            b->N = P.n_finest;
            b->nl = P.n_levels;
            b->bc = P.bc_kind;
            b->L = P.n_levels - 2;
            const size_t nb = (size_t)(b->N + 1) * (b->N + 1) * (b->N + 1) * 8;
            b->af = new Arg(P.f, nb);
            b->a1 = new Arg(P.g1, nb);
            b->a2 = new Arg(P.g2, nb);
            b->au = new Arg(P.u_out, nb);
            CKR(b->af->in());
            CKR(b->a1->in());
            CKR(b->a2->in());
            CKR(b->au->out());
            if (P.ut_out) {
                b->at = new Arg(P.ut_out, nb);
                CKR(b->at->out());
            }
            const int N0 = b->N >> (b->nl - 1);
            b->lv.resize(b->nl);
            size_t max_pa = 1, max_pb = 1;
            for (int l = 0; l < b->nl; l++) {
                Level &Lv = b->lv[l];
                Lv.index = l;
                Lv.N = N0 << l;
                Lv.n = Lv.N - 1;
                Lv.nu = (long long)Lv.n * Lv.n * Lv.n;
                Lv.nodes = (long long)(Lv.N + 1) * (Lv.N + 1) * (Lv.N + 1);
                Lv.g1 = choose_shape(Lv.N, b->bc, 0);
                Lv.g2 = make_geom(Lv.n, b->bc, ty, batch_zc(Lv.N, b->bc, level_f32(*b, l)));
                CKR(Lv.b.ensure(Lv.nu * 8));
                CKR(Lv.x.ensure(Lv.nu * 8));
                CKR(Lv.u.ensure(Lv.nodes * 8));
                const long long nch = (Lv.nu + kChunkGraph - 1) / kChunkGraph;
                const long long mt = batch_max_tiles(Lv.n);
                max_pa = std::max({max_pa, (size_t)stencil_blocks(Lv.g1), (size_t)mt});
                max_pb = std::max({max_pb, (size_t)(2 * nch), (size_t)(2 * vec_blocks(Lv.nu))});
                if (l >= 2) max_items += mt + nch;
            }
            const size_t vb = (size_t)b->lv.back().nu * 8;
            CKR(b->r.ensure(vb)); CKR(b->rs.ensure(vb));
            CKR(b->p[0].ensure(vb)); CKR(b->p[1].ensure(vb));
            CKR(b->ps[0].ensure(vb)); CKR(b->ps[1].ensure(vb));
            CKR(b->q.ensure(vb)); CKR(b->qs.ensure(vb));
            CKR(b->part_a.ensure(max_pa * sizeof(Pair)));
            CKR(b->part_b.ensure(max_pb * sizeof(Pair)));
            const long long m1 = b->N / 2 + 1;
            CKR(b->ubuf.ensure((size_t)m1 * m1 * m1 * 8));
            b->stats.n_levels = b->nl;
        }
        for (StepSet &S : set) {
            CKR(S.items.ensure((size_t)std::max(1LL, max_items) * sizeof(int2)));
            CKH(hipHostMalloc((void **)&S.h_items, (size_t)std::max(1LL, max_items) * sizeof(int2),
                              hipHostMallocDefault));
        }
        CKH(batch_step_grid<double>(ty, &set[0].grid));
        CKH(batch_step_grid<float>(ty, &set[1].grid));
        return EXCMG_OK;
    }

    // Levels 0 and 1 (direct), then the first Bi-CG level's guess.
    int start(int j) {
        BProb &b = *pb[j];
        const double *f = b.af->p<double>(), *g1 = b.a1->p<double>(), *g2 = b.a2->p<double>();
        for (int l = 0; l < 2; l++) {
            Level &Lv = b.lv[l];
            const int s = 1 << (b.nl - 1 - l);
            CKH(rhs_assemble(Lv.N, b.bc, s, b.N, f, g1, g2, Lv.b.as<double>(), st));
            double *Lf = nullptr;
            CKR(fc.get(Lv.N, b.bc, st, &Lf));
            CKH(band_solve((int)Lv.nu, band_width(Lv.N, 3), Lf, Lv.b.as<double>(),
                           Lv.x.as<double>(), st));
            CKH(to_nodes<double>(Lv.N, s, b.N, Lv.x.as<double>(), g1, Lv.u.as<double>(), st));
            b.stats.level[l].n = Lv.N;
        }
        return enter_level(j, 2);
    }

    int enter_level(int j, int l) {
        BProb &b = *pb[j];
        Level &Lv = b.lv[l];
        const int s = 1 << (b.nl - 1 - l);
        CKH(rhs_assemble(Lv.N, b.bc, s, b.N, b.af->p<double>(), b.a1->p<double>(),
                         b.a2->p<double>(), Lv.b.as<double>(), st));
        CKH(exp_finite(Lv.N, b.lv[l - 1].u.as<double>(), b.lv[l - 2].u.as<double>(),
                       b.ubuf.as<double>(), Lv.u.as<double>(), st));
        CKH(from_nodes(Lv.N, Lv.u.as<double>(), Lv.x.as<double>(), st));
        // b.b: into the run state (FP64 runs) and the host-visible slot
        const int nvb = vec_blocks(Lv.nu);
        CKH(dot_partials<double>(Lv.nu, Lv.b.as<double>(), Lv.b.as<double>(),
                                 b.part_b.as<Pair>(), nvb, st));
        CKH(reduce_to(sc(j), b.part_b.as<Pair>(), nvb, 1, st));
        CKH(reduce_to((double *)&S(j)->bb, b.part_b.as<Pair>(), nvb, 0, st));
        b.level = l;
        b.f32 = level_f32(b, l);
        b.phase = kPhaseCheck;
        b.runs = b.iters = b.outer = 0;
        b.prev = INFINITY;
        b.eps = level_tolerance(tol, l - 1, b.L);
        return EXCMG_OK;
    }

    // Launch the true (FP64) residual of the current iterate; r.r lands in slot 2.
    int launch_check(int j) {
        BProb &b = *pb[j];
        Level &Lv = b.lv[b.level];
        if (b.f32)
            CKH(stencil_residual_cast(Lv.g1, Lv.g1.ty, Lv.b.as<double>(), Lv.x.as<double>(),
                                      b.r.as<float>(), b.rs.as<float>(), b.part_a.as<Pair>(), st));
        else
            CKH(stencil_residual<double>(Lv.g1, Lv.g1.ty, Lv.b.as<double>(), Lv.x.as<double>(),
                                         b.r.as<double>(), b.part_a.as<Pair>(), st));
        CKH(reduce_to(sc(j), b.part_a.as<Pair>(), stencil_blocks(Lv.g1), 2, st));
        return EXCMG_OK;
    }

    int finish_level(int j, int status, double rr, double bb) {
        BProb &b = *pb[j];
        Level &Lv = b.lv[b.level];
        const int s = 1 << (b.nl - 1 - b.level);
        excmg_level_stats &ls = b.stats.level[b.level];
        ls.n = Lv.N;
        ls.iterations = b.iters;
        ls.runs = b.f32 ? b.outer : b.runs;
        ls.status = status;
        ls.eps = b.eps;
        ls.rel_residual = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
        if (b.level < EXCMG_MAX_LEVELS) b.level_bb[b.level] = bb;
        if (status != EXCMG_OK && b.worst == EXCMG_OK) b.worst = status;
        CKH(to_nodes<double>(Lv.N, s, b.N, Lv.x.as<double>(), b.a1->p<double>(), Lv.u.as<double>(), st));
        if (b.level == b.nl - 1) {
            if (b.at) CKH(exp_true(b.N, Lv.u.as<double>(), b.lv[b.nl - 2].u.as<double>(),
                                   b.at->p<double>(), st));
            CKH(hipMemcpyAsync(b.au->p<double>(), Lv.u.p, Lv.nodes * 8, hipMemcpyDeviceToDevice, st));
            b.phase = kPhaseDone;
            return EXCMG_OK;
        }
        return enter_level(j, b.level + 1);
    }

    // Decide after a check: converged level, give up, or start a (new) Bi-CG run.
    int decide(int j) {
        BProb &b = *pb[j];
        Level &Lv = b.lv[b.level];
        const double bb = h_scal[4 * j + 1], rr = h_scal[4 * j + 2];
        const double thr = (b.eps * b.eps) * bb;
        if (b.broke) {
            // a breakdown ends the level, as in a single solve: FP64 reports the residual of
            // the iterate after the broken run, mixed precision the residual it was started on
            b.broke = 0;
            if (b.f32) return finish_level(j, EXCMG_EBREAKDOWN, b.prev, b.last_bb);
            return finish_level(j, EXCMG_EBREAKDOWN, rr, bb);
        }
        if (rr <= thr) return finish_level(j, EXCMG_OK, rr, bb);
        BicgState *Sj = S(j);
        if (!b.f32) {
            if (b.runs >= max_runs) return finish_level(j, EXCMG_ENOCONV, rr, bb);
            CKH((copy_convert<double, double>(Lv.nu, b.r.as<double>(), b.rs.as<double>(), st)));
            CKH(bicg_start(Sj, b.part_a.as<Pair>(), stencil_blocks(Lv.g1), b.eps, maxit, st));
            b.iter_base = 0;
        } else {
            if (b.outer >= max_outer || !(rr < b.prev)) return finish_level(j, EXCMG_ENOCONV, rr, bb);
            // a run of this level stopped at its threshold: with residual replacement it goes
            // on from the new residual with its search directions
            const bool resume = reliable && b.outer > 0 && h_states[j].status == kConverged;
            b.prev = rr;
            b.last_bb = bb;
            const int nvb = vec_blocks(Lv.nu);
            CKH(dot_partials<float>(Lv.nu, b.r.as<float>(), b.r.as<float>(), b.part_b.as<Pair>(), nvb, st));
            if (reliable) {
                // the run stops when its recurrence residual has fallen by inner_tol since the
                // replacement, or below half the level's target residual
                const double rthr = std::max((inner_tol * inner_tol) * rr, 0.25 * thr);
                if (resume) {
                    CKH(batch_resume(Sj, b.part_b.as<Pair>(), nvb, rthr, st));
                    b.iter_base = h_states[j].iter;
                } else {
                    CKH(reduce_to((double *)&Sj->bb, b.part_b.as<Pair>(), nvb, 0, st));
                    CKH(bicg_start(Sj, b.part_b.as<Pair>(), nvb, std::sqrt(rthr / rr), maxit, st));
                    b.iter_base = 0;
                }
            } else {
                double it = std::max(inner_tol, 0.3 * b.eps * std::sqrt(bb / rr));
                if (it > 0.5) it = 0.5;
                CKH(reduce_to((double *)&Sj->bb, b.part_b.as<Pair>(), nvb, 0, st));
                CKH(bicg_start(Sj, b.part_b.as<Pair>(), nvb, it, maxit, st));
                b.iter_base = 0;
            }
            b.outer++;
        }
        b.phase = kPhaseRun;
        return EXCMG_OK;
    }

    // Work lists of the running systems, one per vector precision: all sweep-A tiles, then
    // all sweep-B chunks.
    int build_items() {
        const int np = (int)pb.size();
        for (int j = 0; j < np; j++) {
            BProb &b = *pb[j];
            Level &Lv = b.lv[b.level];
            BatchRun &R = h_runs[j];
            R.g = Lv.g2;
            R.nu = Lv.nu;
            R.a_count = Lv.g2.ntiles;
            R.chunk = persistent ? kChunkPersistent : kChunkGraph;
            R.b_count = (int)((Lv.nu + R.chunk - 1) / R.chunk);
            R.r = b.r.p; R.rs = b.rs.p;
            R.p[0] = b.p[0].p; R.p[1] = b.p[1].p; R.ps[0] = b.ps[0].p; R.ps[1] = b.ps[1].p;
            R.q = b.q.p; R.qs = b.qs.p;
            R.x = Lv.x.as<double>();
            R.state = S(j);
            R.part_a = b.part_a.as<Pair>();
            R.part_b = b.part_b.as<Pair>();
        }
        CKH(hipMemcpyAsync(runs.p, h_runs, (size_t)np * sizeof(BatchRun), hipMemcpyHostToDevice, st));
        for (StepSet &K : set) {
            auto in_set = [&](int j) { return pb[j]->phase == kPhaseRun && pb[j]->f32 == K.f32; };
            int na = 0;
            for (int j = 0; j < np; j++)
                if (in_set(j))
                    for (int t = 0; t < h_runs[j].a_count; t++) K.h_items[na++] = make_int2(j, t);
            int ni = na;
            for (int j = 0; j < np; j++)
                if (in_set(j))
                    for (int c = 0; c < h_runs[j].b_count; c++) K.h_items[ni++] = make_int2(j, c);
            K.ni = ni;
            if (ni == 0) continue;
            CKH(hipMemcpyAsync(K.items.p, K.h_items, (size_t)ni * sizeof(int2),
                               hipMemcpyHostToDevice, st));
            // header: n_a, n_items, n_runs, n_active, active[]
            K.h_hdr[0] = na;
            K.h_hdr[1] = ni;
            K.h_hdr[2] = np;
            int nact = 0;
            for (int j = 0; j < np; j++)
                if (in_set(j)) K.h_hdr[4 + nact++] = j;
            K.h_hdr[3] = nact;
            CKH(hipMemcpyAsync((char *)K.ctl.p + offsetof(BatchCtl, n_a), K.h_hdr,
                               (4 + kMaxRuns) * sizeof(int), hipMemcpyHostToDevice, st));
        }
        return EXCMG_OK;
    }

    // steps_per_graph Bi-CG steps of every running system: each precision's steps are
    // captured once in a graph (the launches read their work list from the control block)
    // and replayed while it has systems.
    int launch_steps() {
        for (StepSet &K : set) {
            if (K.ni == 0 || K.exec) continue;
            BatchCtl *ctl = K.ctl.as<BatchCtl>();
            const int2 *items = K.items.as<int2>();
            const BatchRun *rn = runs.as<BatchRun>();
            CKH(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
            for (int t = 0; t < steps_per_graph; t++) {
                hipError_t e;
                if (persistent)
                    e = K.f32 ? batch_step<float>(ty, K.grid, rn, items, ctl, st)
                              : batch_step<double>(ty, K.grid, rn, items, ctl, st);
                else
                    e = K.f32 ? batch_step_phases<float>(ty, rn, items, ctl, st)
                              : batch_step_phases<double>(ty, rn, items, ctl, st);
                if (e != hipSuccess) {
                    hipGraph_t g;
                    (void)hipStreamEndCapture(st, &g);
                    return fail(EXCMG_EHIP, "batch step launch: %s", hipGetErrorString(e));
                }
            }
            CKH(hipStreamEndCapture(st, &K.graph));
            CKH(hipGraphInstantiate(&K.exec, K.graph, nullptr, nullptr, 0));
        }
        // the phase launches never wait for other workgroups, so the two kinds can share
        // the GPU; the persistent kernel needs all its workgroups resident, so its two
        // kinds run one after the other
        const bool side = !persistent && set[0].ni > 0 && set[1].ni > 0;
        if (side && !st2) {
            CKH(hipStreamCreateWithFlags(&st2, hipStreamNonBlocking));
            CKH(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
            CKH(hipEventCreateWithFlags(&join, hipEventDisableTiming));
        }
        if (side) {
            CKH(hipEventRecord(fork, st));
            CKH(hipStreamWaitEvent(st2, fork, 0));
        }
        for (StepSet &K : set)
            if (K.ni > 0) CKH(hipGraphLaunch(K.exec, side && K.f32 ? st2 : st));
        if (side) {
            CKH(hipEventRecord(join, st2));
            CKH(hipStreamWaitEvent(st, join, 0));
        }
        launches += steps_per_graph;
        return EXCMG_OK;
    }

    int run() {
        const int np = (int)pb.size();
        for (int j = 0; j < np; j++) CKR(start(j));
        for (;;) {
            // checks of every system that is between runs
            bool any_check = false;
            for (int j = 0; j < np; j++)
                if (pb[j]->phase == kPhaseCheck) {
                    CKR(launch_check(j));
                    any_check = true;
                }
            if (any_check) {
                CKH(hipMemcpyAsync(h_scal, scal.p, (size_t)np * 4 * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
                CKH(hipStreamSynchronize(st));
                for (int j = 0; j < np; j++)
                    if (pb[j]->phase == kPhaseCheck) CKR(decide(j));
                continue;  // newly entered levels need their first check
            }
            bool running = false;
            for (int j = 0; j < np; j++) running |= (pb[j]->phase == kPhaseRun);
            if (!running) break;
            CKR(build_items());
            // advance every running system until one of them stops
            for (;;) {
                CKR(launch_steps());
                CKH(hipMemcpyAsync(h_states, states.p, (size_t)np * sizeof(BicgState),
                                   hipMemcpyDeviceToHost, st));
                CKH(hipStreamSynchronize(st));
                bool changed = false;
                for (int j = 0; j < np; j++) {
                    BProb &b = *pb[j];
                    if (b.phase != kPhaseRun || h_states[j].status == kRunning) continue;
                    b.iters += h_states[j].iter - b.iter_base;
                    b.runs++;
                    changed = true;
                    b.phase = kPhaseCheck;
                    if (h_states[j].status == kBreakdown) b.broke = 1;
                }
                int err[2] = {0, 0};
                for (int k = 0; k < 2; k++)
                    CKH(hipMemcpyAsync(&err[k], (char *)set[k].ctl.p + offsetof(BatchCtl, error),
                                       sizeof(int), hipMemcpyDeviceToHost, st));
                CKH(hipStreamSynchronize(st));
                if (err[0] || err[1]) return fail(EXCMG_EHIP, "batched step: a bounded wait expired");
                if (changed) break;
            }
        }
        CKR(level_floors());
        for (BProb *b : pb) {
            CKR(b->au->back());
            if (b->at) CKR(b->at->back());
        }
        CKH(hipStreamSynchronize(st));
        return EXCMG_OK;
    }

    // ------------------------------------------------------------ shape tuning
    // The finest level of every problem of `only_n` cells (0: of every problem) as a running
    // Bi-CG system (from x = 0, with a tolerance it never reaches), the other problems idle,
    // so that their steps can be timed with any shape.
    int tune_prepare(int only_n) {
        for (int j = 0; j < (int)pb.size(); j++) {
            BProb &b = *pb[j];
            if (only_n && b.N != only_n) {
                b.phase = kPhaseDone;
                continue;
            }
            b.level = b.nl - 1;
            b.f32 = level_f32(b, b.level);
            Level &Lv = b.lv[b.level];
            CKH(rhs_assemble(Lv.N, b.bc, 1, b.N, b.af->p<double>(), b.a1->p<double>(),
                             b.a2->p<double>(), Lv.b.as<double>(), st));
            CKH(hipMemsetAsync(Lv.x.p, 0, (size_t)Lv.nu * 8, st));
            const int nvb = vec_blocks(Lv.nu);
            if (b.f32) {
                CKH((copy_convert<float, double>(Lv.nu, Lv.b.as<double>(), b.r.as<float>(), st)));
                CKH((copy_convert<float, double>(Lv.nu, Lv.b.as<double>(), b.rs.as<float>(), st)));
                CKH(dot_partials<float>(Lv.nu, b.r.as<float>(), b.r.as<float>(),
                                        b.part_b.as<Pair>(), nvb, st));
            } else {
                CKH((copy_convert<double, double>(Lv.nu, Lv.b.as<double>(), b.r.as<double>(), st)));
                CKH((copy_convert<double, double>(Lv.nu, Lv.b.as<double>(), b.rs.as<double>(), st)));
                CKH(dot_partials<double>(Lv.nu, b.r.as<double>(), b.r.as<double>(),
                                         b.part_b.as<Pair>(), nvb, st));
            }
            CKH(reduce_to((double *)&S(j)->bb, b.part_b.as<Pair>(), nvb, 0, st));
            CKH(bicg_start(S(j), b.part_b.as<Pair>(), nvb, 0.0, 1 << 30, st));
            b.phase = kPhaseRun;
        }
        return EXCMG_OK;
    }

    // The finest levels take tile height `ty` and the z-chunk of their grid in `zc`.
    void tune_apply(const std::vector<BatchZc> &zc) {
        for (BProb *b : pb) {
            Level &Lv = b->lv[b->nl - 1];
            int z = 1;
            for (const auto &e : zc)
                if (e.N == b->N) z = e.zc;
            Lv.g2 = make_geom(Lv.n, b->bc, ty, std::max(1, std::min(z, Lv.n)));
        }
    }

    // Mean ms of one Bi-CG step of the systems of `only_n` cells (0: of the whole batch;
    // phase launches replayed from a graph), every system restarted first.
    int tune_time(int reps, int only_n, double *ms) {
        CKR(tune_prepare(only_n));
        CKR(build_items());
        for (StepSet &K : set) K.drop_graph();
        CKR(launch_steps());  // captures the graphs; warm-up
        hipEvent_t e0 = nullptr, e1 = nullptr;
        CKH(hipEventCreate(&e0));
        hipError_t e = hipEventCreate(&e1);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        int rc = EXCMG_OK;
        for (int t = 0; t < reps && e == hipSuccess && rc == EXCMG_OK; t++) rc = launch_steps();
        if (e == hipSuccess && rc == EXCMG_OK) e = hipEventRecord(e1, st);
        if (e == hipSuccess && rc == EXCMG_OK) e = hipEventSynchronize(e1);
        float f = 0.f;
        if (e == hipSuccess && rc == EXCMG_OK) e = hipEventElapsedTime(&f, e0, e1);
        (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        CKR(rc);
        CKH(e);
        *ms = (double)f / ((double)reps * steps_per_graph);
        return EXCMG_OK;
    }

    // For each tile height (4 and 8 rows) and each of the batch's grid sizes, z-chunks of 2,
    // 4, ... planes and the whole depth are timed on steps of the systems of that size alone
    // (in a whole-batch step the largest systems hide the others' shapes); the height with
    // the smallest sum of the sizes' best steps is kept, with their chunks, for later batches.
    int tune(int reps, int *ty_out, double *ms_out) {
        persistent = false;
        std::vector<int> sizes;
        for (BProb *b : pb)
            if (std::find(sizes.begin(), sizes.end(), b->N) == sizes.end()) sizes.push_back(b->N);
        std::sort(sizes.begin(), sizes.end());
        int best_ty = ty;
        double best = INFINITY;
        std::vector<BatchZc> best_zc;
        for (int cand : {4, 8}) {
            ty = cand;
            CKH(batch_step_grid<double>(ty, &set[0].grid));
            CKH(batch_step_grid<float>(ty, &set[1].grid));
            std::vector<BatchZc> zc;
            for (int N : sizes) {
                const bool f32 = mixed && (long long)(N - 1) * (N - 1) * (N - 1) >= fp32_min;
                zc.push_back({N, f32, batch_zc(N, 1, f32)});
            }
            double total = 0.0;
            for (auto &e : zc) {
                const int n = e.N - 1;
                tune_apply(zc);
                double cur = 0.0;
                CKR(tune_time(reps, e.N, &cur));
                int keep = e.zc;
                for (int z : {2, 4, 8, 16, 32, 64, 128, n}) {
                    if (z > n || z == keep) continue;
                    e.zc = z;
                    tune_apply(zc);
                    double t = 0.0;
                    CKR(tune_time(reps, e.N, &t));
                    if (t < cur) {
                        cur = t;
                        keep = z;
                    }
                }
                e.zc = keep;
                total += cur;
            }
            if (total < best) {
                best = total;
                best_ty = cand;
                best_zc = zc;
            }
        }
        ty = best_ty;
        g_batch_ty = best_ty;
        for (const auto &e : best_zc) {
            bool found = false;
            for (auto &g : g_batch_zc)
                if (g.N == e.N && g.f32 == e.f32) {
                    g.zc = e.zc;
                    found = true;
                }
            if (!found) g_batch_zc.push_back(e);
        }
        *ty_out = best_ty;
        *ms_out = best;
        return EXCMG_OK;
    }

    // The FP64 residual floor of every Bi-CG level's solution (22 u ||x||_2 / ||b||_2) and why
    // each level stopped.
    int level_floors() {
        const int np = (int)pb.size();
        CKR(xx.ensure((size_t)np * EXCMG_MAX_LEVELS * sizeof(double)));
        for (int j = 0; j < np; j++) {
            BProb &b = *pb[j];
            for (int l = 2; l < b.nl && l < EXCMG_MAX_LEVELS; l++) {
                const Level &Lv = b.lv[l];
                const int nb = vec_blocks(Lv.nu);
                CKH(dot_partials<double>(Lv.nu, Lv.x.as<double>(), Lv.x.as<double>(),
                                         b.part_b.as<Pair>(), nb, st));
                CKH(reduce_to(xx.as<double>(), b.part_b.as<Pair>(), nb, j * EXCMG_MAX_LEVELS + l, st));
            }
        }
        std::vector<double> h((size_t)np * EXCMG_MAX_LEVELS);
        CKH(hipMemcpyAsync(h.data(), xx.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        CKH(hipStreamSynchronize(st));
        for (int j = 0; j < np; j++) {
            BProb &b = *pb[j];
            for (int l = 2; l < b.nl && l < EXCMG_MAX_LEVELS; l++) {
                excmg_level_stats &ls = b.stats.level[l];
                const double bb = b.level_bb[l];
                ls.floor = bb > 0 ? kFloorConst * std::sqrt(h[(size_t)j * EXCMG_MAX_LEVELS + l] / bb) : 0.0;
                ls.exit = level_exit(ls.status, ls.eps, ls.floor);
            }
        }
        return EXCMG_OK;
    }
};

}  // namespace

// ================================================================== fixed scratch

// The intermediate grid of EXP_finite for callers that cannot allocate (excmg_exp_finite
// without allocation): a fixed device array of the library, one per GPU, held until the
// process ends.  Its largest use is the (n/2 + 1)^3 Z1 grid of n = kStaticExpFiniteMaxN.
constexpr int kStaticExpFiniteMaxN = 256;
constexpr size_t kStaticScratchDoubles =
    (size_t)(kStaticExpFiniteMaxN / 2 + 1) * (kStaticExpFiniteMaxN / 2 + 1) *
    (kStaticExpFiniteMaxN / 2 + 1);
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

// Device address of `scratch` on each GPU (the array's name in host code is not a device
// address).  Looked up once per device, with that device current, on its first use.
constexpr int kMaxDevices = 64;
double *g_scratch_ptr[kMaxDevices] = {};

int static_scratch(double **out) {
    int dev = 0;
    CKH(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(EXCMG_EINVAL, "device %d out of range", dev);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        CKH(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return EXCMG_OK;
}

// ================================================================== C ABI

extern "C" {

int excmg_set_stream(void *stream) {
    g_stream = (hipStream_t)stream;
    return EXCMG_OK;
}

int excmg_setup(int n_finest, int n_levels, int bc_kind) {
    g_err[0] = 0;
    return setup(n_finest, n_levels, bc_kind);
}

int excmg_apply_stencil(int level, int transpose, const double *x, double *y) {
    (void)transpose;  // A_h is exactly symmetric: A_h^T x = A_h x
    g_err[0] = 0;
    CKR(need_ctx(level));
    if (!x || !y) return fail(EXCMG_EINVAL, "NULL array");
    const Level &L = g_ctx.lv[level];
    Arg ax(x, L.nu * 8), ay(y, L.nu * 8);
    CKR(ax.in());
    CKR(ay.out());
    CKH(stencil_apply<double>(L.g1, L.g1.ty, ax.p<double>(), ay.p<double>(), g_stream));
    CKR(ay.back());
    CKH(hipStreamSynchronize(g_stream));
    return EXCMG_OK;
}

int excmg_apply_operator(int n, int bc_kind, int transpose, const double *x, double *y) {
    (void)transpose;  // A_h is exactly symmetric
    g_err[0] = 0;
    if (n < 2 || n > 4096) return fail(EXCMG_EINVAL, "n must be in 2..4096");
    if (bc_kind != 1 && bc_kind != 2) return fail(EXCMG_EINVAL, "bc_kind must be 1 or 2");
    if (!x || !y) return fail(EXCMG_EINVAL, "NULL array");
    Level L;
    L.N = n;
    L.n = n - 1;
    L.nu = (long long)L.n * L.n * L.n;
    choose_shapes(L, bc_kind);
    Arg ax(x, L.nu * 8), ay(y, L.nu * 8);
    CKR(ax.in());
    CKR(ay.out());
    CKH(stencil_apply<double>(L.g1, L.g1.ty, ax.p<double>(), ay.p<double>(), g_stream));
    CKR(ay.back());
    CKH(hipStreamSynchronize(g_stream));
    return EXCMG_OK;
}

int excmg_rhs(int level, const double *f, const double *g1, const double *g2, double *b) {
    g_err[0] = 0;
    CKR(need_ctx(level));
    if (!f || !g1 || !g2 || !b) return fail(EXCMG_EINVAL, "NULL array");
    const Ctx &c = g_ctx;
    const Level &L = c.lv[level];
    const size_t nb = (size_t)(c.n_finest + 1) * (c.n_finest + 1) *
                      (c.dim == 2 ? 1 : (c.n_finest + 1)) * 8;
    Arg af(f, nb), a1(g1, nb), a2(g2, nb), ab(b, L.nu * 8);
    CKR(af.in());
    CKR(a1.in());
    CKR(a2.in());
    CKR(ab.out());
    if (c.dim == 2)
        CKH(rhs_assemble_2d(L.N, c.bc, 1 << (c.n_levels - 1 - level), c.n_finest, af.p<double>(),
                            a1.p<double>(), a2.p<double>(), ab.p<double>(), g_stream));
    else
        CKH(rhs_assemble(L.N, c.bc, 1 << (c.n_levels - 1 - level), c.n_finest, af.p<double>(),
                         a1.p<double>(), a2.p<double>(), ab.p<double>(), g_stream));
    CKR(ab.back());
    CKH(hipStreamSynchronize(g_stream));
    return EXCMG_OK;
}

int excmg_dsolve(int level, const double *b, double *x) {
    g_err[0] = 0;
    CKR(need_ctx(level));
    if (level > 1) return fail(EXCMG_EINVAL, "DSOLVE is for levels 0 and 1");
    if (!b || !x) return fail(EXCMG_EINVAL, "NULL array");
    Ctx &c = g_ctx;
    const Level &L = c.lv[level];
    Arg ab(b, L.nu * 8), ax(x, L.nu * 8);
    CKR(ab.in());
    CKR(ax.out());
    CKH(band_solve((int)L.nu, c.chol_w[level], c.chol[level].as<double>(), ab.p<double>(),
                   ax.p<double>(), g_stream));
    CKR(ax.back());
    CKH(hipStreamSynchronize(g_stream));
    return EXCMG_OK;
}

int excmg_bicg(int level, const double *b, double *x, double eps, int max_iters, int *iters,
               double *rr) {
    g_err[0] = 0;
    CKR(need_ctx(level));
    if (!b || !x) return fail(EXCMG_EINVAL, "NULL array");
    if (!(eps >= 0.0) || max_iters < 0) return fail(EXCMG_EINVAL, "bad eps or max_iters");
    const Level &L = g_ctx.lv[level];
    Arg ab(b, L.nu * 8), ax(x, L.nu * 8);
    CKR(ab.in());
    CKR(ax.in());
    int it = 0, status = 0;
    double r2 = 0.0;
    g_cg = false;
    CKR(bicg_run(L, ab.p<double>(), ax.p<double>(), eps, max_iters, &it, &r2, &status));
    CKR(ax.back());
    CKH(hipStreamSynchronize(g_stream));
    if (iters) *iters = it;
    if (rr) *rr = r2;
    if (status == kBreakdown) return fail(EXCMG_EBREAKDOWN, "Bi-CG breakdown");
    if (status == kNoConv) return fail(EXCMG_ENOCONV, "Bi-CG reached %d iterations", max_iters);
    return EXCMG_OK;
}

int excmg_bicg_ex(int level, const double *b, double *x, const double *shadow,
                  const double *bstar, double *xstar, const double *mdiag, double eps,
                  int max_iters, int *iters, double *rr) {
    g_err[0] = 0;
    CKR(need_ctx(level));
    if (!b || !x) return fail(EXCMG_EINVAL, "NULL array");
    if ((bstar == nullptr) != (xstar == nullptr))
        return fail(EXCMG_EINVAL, "bstar and xstar go together");
    if (bstar && shadow) return fail(EXCMG_EINVAL, "give either shadow or (bstar, xstar)");
    if (!(eps >= 0.0) || max_iters < 0) return fail(EXCMG_EINVAL, "bad eps or max_iters");
    Level &L = g_ctx.lv[level];
    const size_t vb = (size_t)L.nu * 8;
    Arg ab(b, vb), ax(x, vb), ash(shadow, vb), abs_(bstar, vb), axs(xstar, vb), amd(mdiag, vb);
    CKR(ab.in());
    CKR(ax.in());
    if (shadow) CKR(ash.in());
    if (bstar) {
        CKR(abs_.in());
        CKR(axs.in());
    }
    if (mdiag) CKR(amd.in());
    int it = 0, status = 0;
    double r2 = 0.0;
    g_cg = false;
    CKR(bicg_run(L, ab.p<double>(), ax.p<double>(), eps, max_iters, &it, &r2, &status,
                 mdiag ? amd.p<double>() : nullptr, shadow ? ash.p<double>() : nullptr,
                 bstar ? abs_.p<double>() : nullptr, bstar ? axs.p<double>() : nullptr));
    CKR(ax.back());
    if (bstar) CKR(axs.back());
    CKH(hipStreamSynchronize(g_stream));
    if (iters) *iters = it;
    if (rr) *rr = r2;
    if (status == kBreakdown) return fail(EXCMG_EBREAKDOWN, "Bi-CG breakdown");
    if (status == kNoConv) return fail(EXCMG_ENOCONV, "Bi-CG reached %d iterations", max_iters);
    return EXCMG_OK;
}

int excmg_diagonal(int level, double *d) {
    g_err[0] = 0;
    CKR(need_ctx(level));
    if (!d) return fail(EXCMG_EINVAL, "NULL array");
    Level &L = g_ctx.lv[level];
    const double *dd = level_diagonal(L);
    if (!dd) return fail(EXCMG_EHIP, "diagonal of level %d", level);
    Arg ad(d, (size_t)L.nu * 8);
    CKR(ad.out());
    CKH(hipMemcpyAsync(ad.p<double>(), dd, (size_t)L.nu * 8, hipMemcpyDeviceToDevice, g_stream));
    CKR(ad.back());
    CKH(hipStreamSynchronize(g_stream));
    return EXCMG_OK;
}

int excmg_level_solve(int level, const double *b, double *x, double eps, int max_iters,
                      int max_runs, excmg_level_stats *st) {
    g_err[0] = 0;
    CKR(need_ctx(level));
    if (!b || !x) return fail(EXCMG_EINVAL, "NULL array");
    if (!(eps >= 0.0) || max_iters < 0 || max_runs < 0)
        return fail(EXCMG_EINVAL, "bad eps, max_iters or max_runs");
    const Level &L = g_ctx.lv[level];
    Arg ab(b, L.nu * 8), ax(x, L.nu * 8);
    CKR(ab.in());
    CKR(ax.in());
    excmg_level_stats ls{};
    g_cg = false;
    CKR(level_solve(L, ab.p<double>(), ax.p<double>(), eps, max_iters, max_runs, &ls));
    CKR(ax.back());
    CKH(hipStreamSynchronize(g_stream));
    if (st) *st = ls;
    if (ls.status != EXCMG_OK) return fail(ls.status, "level solve stopped early");
    return EXCMG_OK;
}

int excmg_get_level_solution(int level, double *u) {
    g_err[0] = 0;
    CKR(need_ctx(level));
    if (!u) return fail(EXCMG_EINVAL, "NULL array");
    const Level &L = g_ctx.lv[level];
    Arg au(u, L.nodes * 8);
    CKR(au.out());
    CKH(hipMemcpyAsync(au.p<double>(), L.u.p, L.nodes * 8, hipMemcpyDeviceToDevice, g_stream));
    CKR(au.back());
    CKH(hipStreamSynchronize(g_stream));
    return EXCMG_OK;
}

int excmg_exp_finite(int n, const double *u1, const double *u0, double *w) {
    g_err[0] = 0;
    if (n < 4 || n % 4 != 0 || n > 4096) return fail(EXCMG_EINVAL, "n must be a multiple of 4");
    if (!u1 || !u0 || !w) return fail(EXCMG_EINVAL, "NULL array");
    const size_t m1 = (size_t)(n / 2 + 1), m0 = (size_t)(n / 4 + 1), m = (size_t)(n + 1);
    Arg a1(u1, m1 * m1 * m1 * 8), a0(u0, m0 * m0 * m0 * 8), aw(w, m * m * m * 8);
    CKR(a1.in());
    CKR(a0.in());
    CKR(aw.out());
    DBuf v;
    CKR(v.ensure(m1 * m1 * m1 * 8));
    hipError_t e = exp_finite(n, a1.p<double>(), a0.p<double>(), v.as<double>(), aw.p<double>(),
                              g_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g_stream);
    v.release();
    CKH(e);
    CKR(aw.back());
    CKH(hipStreamSynchronize(g_stream));
    return EXCMG_OK;
}

int excmg_exp_finite_noalloc(int n, const double *u1, const double *u0, double *w) {
    g_err[0] = 0;
    if (n < 4 || n % 4 != 0 || n > kStaticExpFiniteMaxN)
        return fail(EXCMG_EINVAL, "n must be a multiple of 4 in 4..%d (got %d)",
                    kStaticExpFiniteMaxN, n);
    if (!u1 || !u0 || !w) return fail(EXCMG_EINVAL, "NULL array");
    if (!is_device_ptr(u1) || !is_device_ptr(u0) || !is_device_ptr(w))
        return fail(EXCMG_EINVAL, "u1, u0 and w must be device arrays (nothing is staged)");
    double *v = nullptr;
    CKR(static_scratch(&v));
    // every node of the Z1 grid is written by the first kernel before the second reads it,
    // so the array needs no clearing between calls
    CKH(exp_finite(n, u1, u0, v, w, g_stream));
    return EXCMG_OK;
}

int excmg_exp_true(int n, const double *uh, const double *u2h, double *ut) {
    g_err[0] = 0;
    if (n < 2 || n % 2 != 0 || n > 4096) return fail(EXCMG_EINVAL, "n must be even");
    if (!uh || !u2h || !ut) return fail(EXCMG_EINVAL, "NULL array");
    const size_t m = (size_t)(n + 1), mc = (size_t)(n / 2 + 1);
    Arg ah(uh, m * m * m * 8), ac(u2h, mc * mc * mc * 8), at(ut, m * m * m * 8);
    CKR(ah.in());
    CKR(ac.in());
    CKR(at.out());
    CKH(exp_true(n, ah.p<double>(), ac.p<double>(), at.p<double>(), g_stream));
    CKR(at.back());
    CKH(hipStreamSynchronize(g_stream));
    return EXCMG_OK;
}

int solve_ex_dim(const excmg_opts *opts, const double *f, const double *g1, const double *g2,
                 double *u_out, double *ut_out, excmg_stats *st, int dim) {
    g_err[0] = 0;
    if (!opts) return fail(EXCMG_EINVAL, "NULL options");
    const excmg_opts o = *opts;
    if (!f || !g1 || !g2 || !u_out) return fail(EXCMG_EINVAL, "NULL array");
    if (!(o.tol > 0.0)) return fail(EXCMG_EINVAL, "tol must be positive");
    if (o.precision != EXCMG_FP64 && o.precision != EXCMG_MIXED)
        return fail(EXCMG_EINVAL, "precision %d not supported", o.precision);
    if (o.method != EXCMG_BICG && o.method != EXCMG_CG)
        return fail(EXCMG_EINVAL, "method %d not supported", o.method);
    if (o.refine != EXCMG_RELIABLE && o.refine != EXCMG_RESTART)
        return fail(EXCMG_EINVAL, "refine %d not supported", o.refine);
    if (o.precond != EXCMG_PRECOND_NONE && o.precond != EXCMG_PRECOND_JACOBI)
        return fail(EXCMG_EINVAL, "precond %d not supported", o.precond);
    if (o.fp32_min_unknowns < 0)
        return fail(EXCMG_EINVAL, "fp32_min_unknowns must be >= 0");
    if (o.row_pad < 0 || o.row_pad > 2) return fail(EXCMG_EINVAL, "row_pad must be 0, 1 or 2");
    if (o.recompute_min_unknowns < 0)
        return fail(EXCMG_EINVAL, "recompute_min_unknowns must be >= 0");
    if (o.precond == EXCMG_PRECOND_JACOBI && (o.precision != EXCMG_FP64 || o.method != EXCMG_BICG))
        return fail(EXCMG_EINVAL, "the Jacobi preconditioner runs with FP64 Bi-CG only");
    CKR(setup(o.n_finest, o.n_levels, o.bc_kind, dim));
    const size_t nb = (size_t)(o.n_finest + 1) * (o.n_finest + 1) *
                      (dim == 2 ? 1 : (o.n_finest + 1)) * 8;
    Arg af(f, nb), a1(g1, nb), a2(g2, nb), au(u_out, nb), at(ut_out, nb);
    CKR(af.in());
    CKR(a1.in());
    CKR(a2.in());
    CKR(au.out());
    if (ut_out) CKR(at.out());
    if (st) memset(st, 0, sizeof(*st));
    g_cg = (o.method == EXCMG_CG);
    g_graphs = true;
    g_rq_min = o.recompute_min_unknowns > 0 ? o.recompute_min_unknowns : 0;
    int rc = solve_cascade(o, af.p<double>(), a1.p<double>(), a2.p<double>(), au.p<double>(),
                        ut_out ? at.p<double>() : nullptr, st);
    g_graphs = false;
    g_rq_min = 0;
    if (rc != EXCMG_OK && rc != EXCMG_ENOCONV && rc != EXCMG_EBREAKDOWN) return rc;
    CKR(au.back());
    if (ut_out) CKR(at.back());
    CKH(hipStreamSynchronize(g_stream));
    return rc;
}

int excmg_solve_ex(const excmg_opts *opts, const double *f, const double *g1, const double *g2,
                   double *u_out, double *ut_out, excmg_stats *st) {
    return solve_ex_dim(opts, f, g1, g2, u_out, ut_out, st, 3);
}

int excmg2d_solve_ex(const excmg_opts *opts, const double *f, const double *g1, const double *g2,
                     double *u_out, double *ut_out, excmg_stats *st) {
    return solve_ex_dim(opts, f, g1, g2, u_out, ut_out, st, 2);
}

int excmg2d_setup(int n_finest, int n_levels, int bc_kind) {
    g_err[0] = 0;
    return setup(n_finest, n_levels, bc_kind, 2);
}

int excmg2d_exp_finite(int n, const double *u1, const double *u0, double *w) {
    g_err[0] = 0;
    if (n < 4 || n % 4 != 0 || n > 16384) return fail(EXCMG_EINVAL, "n must be a multiple of 4");
    if (!u1 || !u0 || !w) return fail(EXCMG_EINVAL, "NULL array");
    const size_t m1 = (size_t)(n / 2 + 1), m0 = (size_t)(n / 4 + 1), m = (size_t)(n + 1);
    Arg a1(u1, m1 * m1 * 8), a0(u0, m0 * m0 * 8), aw(w, m * m * 8);
    CKR(a1.in());
    CKR(a0.in());
    CKR(aw.out());
    DBuf v;
    CKR(v.ensure(m1 * m1 * 8));
    CKH(exp_finite_2d(n, a1.p<double>(), a0.p<double>(), v.as<double>(), aw.p<double>(), g_stream));
    CKR(aw.back());
    CKH(hipStreamSynchronize(g_stream));
    return EXCMG_OK;
}

int excmg2d_exp_true(int n, const double *uh, const double *u2h, double *ut) {
    g_err[0] = 0;
    if (n < 2 || n % 2 != 0 || n > 16384) return fail(EXCMG_EINVAL, "n must be even");
    if (!uh || !u2h || !ut) return fail(EXCMG_EINVAL, "NULL array");
    const size_t m = (size_t)(n + 1), mc = (size_t)(n / 2 + 1);
    Arg ah(uh, m * m * 8), ac(u2h, mc * mc * 8), at(ut, m * m * 8);
    CKR(ah.in());
    CKR(ac.in());
    CKR(at.out());
    CKH(exp_true_2d(n, ah.p<double>(), ac.p<double>(), at.p<double>(), g_stream));
    CKR(at.back());
    CKH(hipStreamSynchronize(g_stream));
    return EXCMG_OK;
}

int excmg_solve(int n_finest, int n_levels, int bc_kind, const double *f, const double *g1,
                const double *g2, double tol, double *u_out) {
    excmg_opts o;
    memset(&o, 0, sizeof(o));
    o.n_finest = n_finest;
    o.n_levels = n_levels;
    o.bc_kind = bc_kind;
    o.precision = EXCMG_FP64;
    o.tol = tol;
    return excmg_solve_ex(&o, f, g1, g2, u_out, nullptr, nullptr);
}

int excmg_profile_sweep(int which, int precision, int reps, double *ms_per_launch,
                        double *bytes_per_launch) {
    g_err[0] = 0;
    if (!g_ctx.ready) return fail(EXCMG_ENOCTX, "no context: call excmg_setup first");
    if (which < 0 || which > 10 || reps < 1) return fail(EXCMG_EINVAL, "bad sweep or reps");
    if (precision != EXCMG_FP64 && precision != EXCMG_MIXED)
        return fail(EXCMG_EINVAL, "bad precision");
    if (which >= 5 && g_ctx.dim != 3) return fail(EXCMG_EINVAL, "sweeps 5 to 10 are 3D ones");
    if (which >= 9 && precision == EXCMG_MIXED && g_ctx.lv.back().wide)
        return fail(EXCMG_EINVAL, "sweeps 9 and 10 take single-point tiles (row_pad 2 is set)");
    if ((which == 5 || which == 6) && precision != EXCMG_MIXED)
        return fail(EXCMG_EINVAL, "sweeps 5 and 6 are mixed-precision ones");
    Ctx &c = g_ctx;
    const Level &L = c.lv.back();
    const size_t es = precision == EXCMG_FP64 ? 8 : 4;
    // mixed sweeps run on the row layout of the mixed solve (padded on large grids)
    const bool mixed = precision == EXCMG_MIXED;
    const long long nv = mixed ? L.nflat : L.nu;
    const Rows rows = mixed ? L.rows() : Rows{};
    const bool padded = mixed && L.ld != L.n;
    double *xv = padded ? c.xp.as<double>() : L.x.as<double>();
    double *bv = padded ? c.bp.as<double>() : L.b.as<double>();
    const size_t vb = (size_t)nv * es;
    DBuf *vecs[8] = {&c.r, &c.rs, &c.p[0], &c.p[1], &c.ps[0], &c.ps[1], &c.q, &c.qs};
    for (DBuf *v : vecs) CKH(hipMemsetAsync(v->p, 0, vb, g_stream));
    CKH(hipMemsetAsync(xv, 0, (size_t)nv * 8, g_stream));
    CKH(hipMemsetAsync(bv, 0, (size_t)nv * 8, g_stream));
    BicgState hs{};
    hs.status = kRunning;
    hs.rho = 1.0;
    hs.maxit = 1 << 30;
    CKH(hipMemcpyAsync(c.state.p, &hs, sizeof(hs), hipMemcpyHostToDevice, g_stream));
    BicgState *S = c.state.as<BicgState>();
    // algorithmic bytes per unknown of each sweep
    const double fp64_bytes[11] = {16, 24, 64, 72, 16, 0, 0, 48, 64, 48, 72};
    const double mixed_bytes[11] = {8, 24, 32, 44, 8, 48, 24, 24, 40, 24, 44};
    auto launch_once = [&]() -> hipError_t {
        if (precision == EXCMG_FP64) {
            double *r = c.r.as<double>(), *rs = c.rs.as<double>();
            switch (which) {
                case 0: return stencil_apply<double>(L.g1, L.g1.ty, r, c.q.as<double>(), g_stream);
                case 1: return stencil_residual<double>(L.g1, L.g1.ty, L.b.as<double>(), r,
                                                        c.q.as<double>(), c.part_a.as<Pair>(),
                                                        g_stream);
                case 2: return stencil_pair_direction<double>(
                            L.g2, L.g2.ty, r, rs, c.p[0].as<double>(), c.ps[0].as<double>(),
                            &S->beta, 0, c.p[1].as<double>(), c.ps[1].as<double>(),
                            c.q.as<double>(), c.qs.as<double>(), c.part_a.as<Pair>(), &S->status,
                            g_stream);
                case 3: return bicg_update<double, double>(
                            L.nu, S, L.x.as<double>(), c.p[1].as<double>(), r, c.q.as<double>(),
                            rs, c.qs.as<double>(), c.part_b.as<Pair>(), g_stream);
                case 7: return stencil_dir_sigma<double>(
                            L.g2, L.g2.ty, r, rs, c.p[0].as<double>(), c.ps[0].as<double>(),
                            &S->beta, 0, c.p[1].as<double>(), c.ps[1].as<double>(),
                            c.part_a.as<Pair>(), &S->status, g_stream, StepLink{});
                case 8:
                case 9:
                case 10: return stencil_pair_update<double>(
                            L.g2, L.g2.ty, c.p[1].as<double>(), c.ps[1].as<double>(),
                            L.x.as<double>(), r, rs, c.part_b.as<Pair>(), &S->status, &S->alpha,
                            g_stream, StepLink{}, which - 8, c.p[0].as<double>(), &S->alpha,
                            L.nu < kDownMaxUnknowns);
                default: return copy_convert<double, double>(L.nu, r, c.q.as<double>(), g_stream);
            }
        }
        float *r = c.r.as<float>(), *rs = c.rs.as<float>();
        switch (which) {
            case 0: return stencil_apply<float>(L.g1p, L.g1p.ty, r, c.q.as<float>(), g_stream);
            case 1: return stencil_residual_cast(L.g1p, L.g1p.ty, bv, xv, r, rs,
                                                 c.part_a.as<Pair>(), g_stream);
            case 2: return stencil_pair_direction<float>(
                        L.g2f, L.g2f.ty, r, rs, c.p[0].as<float>(), c.ps[0].as<float>(), &S->beta,
                        0, c.p[1].as<float>(), c.ps[1].as<float>(), c.q.as<float>(),
                        c.qs.as<float>(), c.part_a.as<Pair>(), &S->status, g_stream);
            case 3: return bicg_update<double, float>(L.nu, S, xv, c.p[1].as<float>(), r,
                                                      c.q.as<float>(), rs, c.qs.as<float>(),
                                                      c.part_b.as<Pair>(), g_stream, StepLink{},
                                                      rows);
            case 5: return stencil_pair_direction_x(
                        L.g2f, L.g2f.ty, r, rs, c.p[0].as<float>(), c.ps[0].as<float>(), &S->beta,
                        c.p[1].as<float>(), c.ps[1].as<float>(), c.q.as<float>(),
                        c.qs.as<float>(), c.part_a.as<Pair>(), &S->status, xv, &S->alpha,
                        g_stream, StepLink{});
            case 6: return bicg_update<double, float>(L.nu, S, nullptr, c.p[1].as<float>(), r,
                                                      c.q.as<float>(), rs, c.qs.as<float>(),
                                                      c.part_b.as<Pair>(), g_stream, StepLink{},
                                                      rows);
            case 7: return stencil_dir_sigma<float>(rq_geom_f32(L), rq_geom_f32(L).ty, r, rs, c.p[0].as<float>(),
                                             c.ps[0].as<float>(), &S->beta, 0,
                                             c.p[1].as<float>(), c.ps[1].as<float>(),
                                             c.part_a.as<Pair>(), &S->status, g_stream,
                                             StepLink{}, nullptr, nullptr, !L.wide);
            case 8:
            case 9:
            case 10: return stencil_pair_update<float>(rq_geom_f32(L), rq_geom_f32(L).ty, c.p[1].as<float>(),
                                               c.ps[1].as<float>(), xv, r, rs,
                                               c.part_b.as<Pair>(), &S->status, &S->alpha,
                                               g_stream, StepLink{}, which - 8, c.p[0].as<float>(),
                                               &S->alpha);
            default: return copy_convert<float, float>(L.nu, r, c.q.as<float>(), g_stream);
        }
    };
    CKH(launch_once());  // warm-up
    hipEvent_t e0, e1;
    CKH(hipEventCreate(&e0));
    CKH(hipEventCreate(&e1));
    CKH(hipEventRecord(e0, g_stream));
    for (int t = 0; t < reps; t++) CKH(launch_once());
    CKH(hipEventRecord(e1, g_stream));
    CKH(hipEventSynchronize(e1));
    float ms = 0.f;
    CKH(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms_per_launch) *ms_per_launch = (double)ms / reps;
    if (bytes_per_launch)
        *bytes_per_launch =
            (precision == EXCMG_FP64 ? fp64_bytes[which] : mixed_bytes[which]) * (double)L.nu;
    return EXCMG_OK;
}

int excmg_solve_batch(int nprob, const excmg_problem *probs, const excmg_opts *opts,
                      excmg_stats *stats) {
    g_err[0] = 0;
    if (nprob < 1 || nprob > kMaxRuns) return fail(EXCMG_EINVAL, "nprob must be in 1..%d", kMaxRuns);
    if (!probs || !opts) return fail(EXCMG_EINVAL, "NULL problems or options");
    if (!(opts->tol > 0.0)) return fail(EXCMG_EINVAL, "tol must be positive");
    if (opts->precision != EXCMG_FP64 && opts->precision != EXCMG_MIXED)
        return fail(EXCMG_EINVAL, "precision %d not supported", opts->precision);
    if (opts->fp32_min_unknowns < 0) return fail(EXCMG_EINVAL, "fp32_min_unknowns must be >= 0");
    if (opts->refine != EXCMG_RELIABLE && opts->refine != EXCMG_RESTART)
        return fail(EXCMG_EINVAL, "refine %d not supported", opts->refine);
    for (int j = 0; j < nprob; j++) CKR(check_sizes(probs[j].n_finest, probs[j].n_levels, probs[j].bc_kind));
    // every failure below is recorded in rc and the stream, events and library stream are
    // restored and released on the way out
    int rc = EXCMG_OK;
    auto hip_ok = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && rc == EXCMG_OK)
            rc = fail(EXCMG_EHIP, "%s failed: %s", what, hipGetErrorString(e));
        return rc == EXCMG_OK;
    };
    hipStream_t bs = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr, ein = nullptr;
    float ms = 0.f;
    if (hip_ok(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking), "hipStreamCreate") &&
        hip_ok(hipEventCreate(&e0), "hipEventCreate") && hip_ok(hipEventCreate(&e1), "hipEventCreate") &&
        hip_ok(hipEventCreate(&ein), "hipEventCreate") &&
        hip_ok(hipEventRecord(ein, g_stream), "hipEventRecord") &&
        hip_ok(hipStreamWaitEvent(bs, ein, 0), "hipStreamWaitEvent")) {
        hipStream_t saved = g_stream;
        g_stream = bs;  // host-array staging of the batch goes through the batch stream
        {
            BatchSolver B;
            B.st = bs;
            rc = B.init(nprob, probs, *opts);
            if (rc == EXCMG_OK && hip_ok(hipEventRecord(e0, bs), "hipEventRecord")) {
                rc = B.run();
                if (rc == EXCMG_OK && hip_ok(hipEventRecord(e1, bs), "hipEventRecord") &&
                    hip_ok(hipEventSynchronize(e1), "hipEventSynchronize"))
                    hip_ok(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            }
            if (rc == EXCMG_OK) {
                int worst = EXCMG_OK;
                for (int j = 0; j < nprob; j++) {
                    B.pb[j]->stats.total_ms = ms;
                    if (stats) stats[j] = B.pb[j]->stats;
                    if (B.pb[j]->worst != EXCMG_OK && worst == EXCMG_OK) worst = B.pb[j]->worst;
                }
                if (worst != EXCMG_OK) rc = fail(worst, "a level of a batched problem stopped early");
            }
            (void)hipStreamSynchronize(bs);
        }
        g_stream = saved;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (ein) (void)hipEventDestroy(ein);
    if (bs) (void)hipStreamDestroy(bs);
    return rc;
}

int excmg_autotune_batch(int nprob, const excmg_problem *probs, const excmg_opts *opts, int reps,
                         int *ty_out, double *ms_out) {
    g_err[0] = 0;
    if (nprob < 1 || nprob > kMaxRuns) return fail(EXCMG_EINVAL, "nprob must be in 1..%d", kMaxRuns);
    if (!probs || !opts || reps < 1) return fail(EXCMG_EINVAL, "NULL problems or options, or reps < 1");
    if (opts->precision != EXCMG_FP64 && opts->precision != EXCMG_MIXED)
        return fail(EXCMG_EINVAL, "precision %d not supported", opts->precision);
    if (opts->fp32_min_unknowns < 0) return fail(EXCMG_EINVAL, "fp32_min_unknowns must be >= 0");
    for (int j = 0; j < nprob; j++) CKR(check_sizes(probs[j].n_finest, probs[j].n_levels, probs[j].bc_kind));
    hipStream_t bs = nullptr;
    CKH(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
    hipStream_t saved = g_stream;
    g_stream = bs;
    int rc;
    int ty = 0;
    double ms = 0.0;
    {
        BatchSolver B;
        B.st = bs;
        excmg_opts o = *opts;
        o.batch_mode = 0;
        if (!(o.tol > 0.0)) o.tol = 1e-8;
        rc = B.init(nprob, probs, o);
        if (rc == EXCMG_OK) rc = B.tune(reps, &ty, &ms);
        (void)hipStreamSynchronize(bs);
    }
    g_stream = saved;
    (void)hipStreamDestroy(bs);
    if (rc == EXCMG_OK) {
        if (ty_out) *ty_out = ty;
        if (ms_out) *ms_out = ms;
    }
    return rc;
}

int excmg_get_batch_shape(int n, int precision, int *ty, int *zc) {
    g_err[0] = 0;
    if (n < 3) return fail(EXCMG_EINVAL, "n must be at least 3");
    if (ty) *ty = g_batch_ty;
    if (zc) *zc = batch_zc(n, 1, precision == EXCMG_MIXED);
    return EXCMG_OK;
}

int excmg_autotune(int n, int kind, int precision, int reps, int *ty_out, int *zc_out,
                   double *ms_out) {
    g_err[0] = 0;
    if (n < 4 || n > 4096) return fail(EXCMG_EINVAL, "n must be in 4..4096");
    if (kind != 0 && kind != 1) return fail(EXCMG_EINVAL, "kind must be 0 or 1");
    if (precision != EXCMG_FP64 && precision != EXCMG_MIXED) return fail(EXCMG_EINVAL, "bad precision");
    if (reps < 1) reps = 5;
    const int nn = n - 1;
    const size_t es = precision == EXCMG_FP64 ? 8 : 4;
    const int ld = nn;  // contiguous rows, the solver's default
    const long long nv = (long long)nn * nn * ld;
    // on grids where Bi-CG takes the recomputing form, sweep A is timed with the sweep B it
    // shares its launch shape with (the pair the solver runs; x is FP64 in both precisions)
    const bool rq = kind == 1 && (long long)nn * nn * nn >= recompute_min(es == 8) && !g_var.d &&
                    !g_var.xs;
    DBuf v[8], part, stb, xd;
    for (auto &b : v) {
        CKR(b.ensure((size_t)nv * es));
        CKH(hipMemsetAsync(b.p, 0, (size_t)nv * es, g_stream));
    }
    if (rq) {
        CKR(xd.ensure((size_t)nv * 8));
        CKH(hipMemsetAsync(xd.p, 0, (size_t)nv * 8, g_stream));
    }
    CKR(stb.ensure(sizeof(BicgState)));
    BicgState hs{};
    hs.status = kRunning;
    hs.rho = 1.0;
    hs.maxit = 1 << 30;
    CKH(hipMemcpyAsync(stb.p, &hs, sizeof(hs), hipMemcpyHostToDevice, g_stream));
    BicgState *S = stb.as<BicgState>();
    // FP64 sweep A spills at ty = 16 (1024 threads leave 128 registers per lane)
    std::vector<int> tys = (kind == 1 && es == 8) ? std::vector<int>{4, 8} : std::vector<int>{4, 8, 16};
    double best = INFINITY;
    int bty = 8, bzc = 8;
    hipEvent_t e0, e1;
    CKH(hipEventCreate(&e0));
    CKH(hipEventCreate(&e1));
    int rc = EXCMG_OK;
    int pair_calls = 0;
    for (int ty : tys) {
        // chunks of 2, 4, ... planes and, last, the whole depth in one march
        for (int zp = 2;; zp *= 2) {
            const int zc = std::min(zp, nn);
            Geom g = with_rows(make_geom(nn, 1, ty, zc), ld);
            rc = part.ensure((size_t)stencil_blocks(g) * sizeof(Pair) * (rq ? 2 : 1));
            if (rc) break;
            auto launch = [&]() -> hipError_t {
                if (kind == 0) {
                    if (es == 8) return stencil_apply<double>(g, ty, v[0].as<double>(), v[1].as<double>(), g_stream);
                    return stencil_apply<float>(g, ty, v[0].as<float>(), v[1].as<float>(), g_stream);
                }
                if (rq) {
                    // r, r*, p, p* -> p_new, p*_new (sigma); then p_new, p*_new -> x, r, r*,
                    // the sweeps B alternating as the solver's paired updates do
                    const StepLink nl{};
                    const int xm = 1 + (pair_calls++ & 1);
                    hipError_t e;
                    if (es == 8) {
                        e = stencil_dir_sigma<double>(g, ty, v[0].as<double>(), v[1].as<double>(),
                                                      v[2].as<double>(), v[3].as<double>(), &S->beta, 0,
                                                      v[4].as<double>(), v[5].as<double>(), part.as<Pair>(),
                                                      &S->status, g_stream, nl);
                        if (e != hipSuccess) return e;
                        return stencil_pair_update<double>(g, ty, v[4].as<double>(), v[5].as<double>(),
                                                           xd.as<double>(), v[0].as<double>(),
                                                           v[1].as<double>(), part.as<Pair>(), &S->status,
                                                           &S->alpha, g_stream, nl, xm, v[2].as<double>(),
                                                           &S->alpha,
                                                           (long long)nn * nn * nn < kDownMaxUnknowns);
                    }
                    e = stencil_dir_sigma<float>(g, ty, v[0].as<float>(), v[1].as<float>(), v[2].as<float>(),
                                                 v[3].as<float>(), &S->beta, 0, v[4].as<float>(),
                                                 v[5].as<float>(), part.as<Pair>(), &S->status, g_stream, nl,
                                                 nullptr, nullptr, true);
                    if (e != hipSuccess) return e;
                    return stencil_pair_update<float>(g, ty, v[4].as<float>(), v[5].as<float>(), xd.as<double>(),
                                                      v[0].as<float>(), v[1].as<float>(), part.as<Pair>(),
                                                      &S->status, &S->alpha, g_stream, nl, xm,
                                                      v[2].as<float>(), &S->alpha);
                }
                if (es == 8)
                    return stencil_pair_direction<double>(g, ty, v[0].as<double>(), v[1].as<double>(),
                                                          v[2].as<double>(), v[3].as<double>(), &S->beta, 0,
                                                          v[4].as<double>(), v[5].as<double>(), v[6].as<double>(),
                                                          v[7].as<double>(), part.as<Pair>(), &S->status, g_stream);
                return stencil_pair_direction<float>(g, ty, v[0].as<float>(), v[1].as<float>(),
                                                     v[2].as<float>(), v[3].as<float>(), &S->beta, 0,
                                                     v[4].as<float>(), v[5].as<float>(), v[6].as<float>(),
                                                     v[7].as<float>(), part.as<Pair>(), &S->status, g_stream);
            };
            CKH(launch());
            CKH(hipEventRecord(e0, g_stream));
            for (int t = 0; t < reps; t++) CKH(launch());
            CKH(hipEventRecord(e1, g_stream));
            CKH(hipEventSynchronize(e1));
            float ms = 0.f;
            CKH(hipEventElapsedTime(&ms, e0, e1));
            if (ms / reps < best) {
                best = ms / reps;
                bty = ty;
                bzc = zc;
            }
            if (zc == nn) break;
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (auto &b : v) b.release();
    part.release();
    stb.release();
    xd.release();
    if (rc) return rc;
    CKR(excmg_set_shape(n, (kind == 1 && es == 4) ? 2 : kind, bty, bzc));
    if (ty_out) *ty_out = bty;
    if (zc_out) *zc_out = bzc;
    if (ms_out) *ms_out = best;
    return EXCMG_OK;
}

int excmg_set_timing(int on) {
    g_timing = (on != 0);
    memset(g_time_ms, 0, sizeof(g_time_ms));
    memset(g_time_n, 0, sizeof(g_time_n));
    return EXCMG_OK;
}

int excmg_get_timing(int level, int sweep, double *ms_total, long long *launches) {
    if (level < 0 || level >= EXCMG_MAX_LEVELS || sweep < 0 || sweep > 4)
        return fail(EXCMG_EINVAL, "bad level or sweep");
    if (ms_total) *ms_total = g_time_ms[level][sweep];
    if (launches) *launches = g_time_n[level][sweep];
    return EXCMG_OK;
}

int excmg_set_shape(int n, int kind, int ty, int zc) {
    g_err[0] = 0;
    if (n < 2) return fail(EXCMG_EINVAL, "n must be >= 2");
    if (kind < 0 || kind > 2) return fail(EXCMG_EINVAL, "kind must be 0, 1 or 2");
    if (ty != 0 && ty != 4 && ty != 8 && ty != 16) return fail(EXCMG_EINVAL, "ty must be 4, 8 or 16");
    if (kind == 1 && ty == 16) return fail(EXCMG_EINVAL, "FP64 sweep A supports ty 4 or 8");
    if (ty != 0 && zc < 1) return fail(EXCMG_EINVAL, "zc must be >= 1");
    for (size_t i = 0; i < g_shapes.size(); i++)
        if (g_shapes[i].N == n && g_shapes[i].kind == kind) {
            g_shapes.erase(g_shapes.begin() + i);
            break;
        }
    if (ty != 0) g_shapes.push_back(ShapeOverride{n, kind, ty, zc});
    release_graphs();  // captured iteration windows hold the old launch shapes
    for (Level &L : g_ctx.lv) {
        if (L.N != n) continue;
        choose_shapes(L, g_ctx.bc, g_ctx.dim);
        const size_t need = (size_t)std::max({stencil_blocks(L.g1), stencil_blocks(L.g2),
                                              stencil_blocks(L.g2f), stencil_blocks(L.g2w)}) *
                            sizeof(Pair);
        if (need > g_ctx.part_a.bytes) CKR(g_ctx.part_a.ensure(need));
        if (2 * need > g_ctx.part_b.bytes) CKR(g_ctx.part_b.ensure(2 * need));
    }
    return EXCMG_OK;
}

int excmg_get_shape(int n, int kind, int *ty, int *zc) {
    if (n < 2 || kind < 0 || kind > 2) return fail(EXCMG_EINVAL, "bad n or kind");
    Geom g = choose_shape(n, 1, kind);
    if (ty) *ty = g.ty;
    if (zc) *zc = g.zc;
    return EXCMG_OK;
}

const char *excmg_last_error(void) { return g_err; }

void excmg_finalize(void) {
    (void)hipStreamSynchronize(g_stream);
    g_ctx.release();
}

}  // extern "C"
