// Host driver and C ABI of the EXCMG library: the cascade of Algorithm 1, the level loop,
// the device-resident Bi-CG iteration of Algorithm 2 and the entry points of excmg.h.
//
// Control stays on the device inside a Bi-CG run: the scalars (rho, sigma, alpha, beta,
// r.r) and the run status live in device memory, every kernel of an iteration returns
// immediately once the run has stopped, and the host only reads the 64-byte state every few
// iterations to decide whether to launch more.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
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
    Geom g1{}, g2{};  // launch shapes: single-array kernels, Bi-CG sweep A
    DBuf b, x, u;     // right-hand side, unknowns, node array (solution or EXP_finite guess)
};

struct Ctx {
    bool ready = false;
    int n_finest = 0, n_levels = 0, bc = 0;
    std::vector<Level> lv;
    // Bi-CG workspace (sized for the finest level)
    DBuf r, rs, p[2], ps[2], q, qs;
    DBuf part_a, part_b;        // Dot2 partials of the two sweeps
    DBuf state;                 // BicgState
    DBuf scal;                  // misc device scalars
    DBuf chol[2], chol_y;       // Cholesky factors of levels 0 and 1, solve scratch
    DBuf info;
    DBuf vz1;                   // EXP_finite Z1 scratch
    BicgState *host_state = nullptr;  // pinned
    double *host_scal = nullptr;      // pinned
    void release() {
        for (auto &L : lv) {
            L.b.release();
            L.x.release();
            L.u.release();
        }
        lv.clear();
        r.release(); rs.release();
        p[0].release(); p[1].release(); ps[0].release(); ps[1].release();
        q.release(); qs.release();
        part_a.release(); part_b.release(); state.release(); scal.release();
        chol[0].release(); chol[1].release(); chol_y.release(); info.release(); vz1.release();
        if (host_state) (void)hipHostFree(host_state);
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
double g_time_ms[EXCMG_MAX_LEVELS][2];
long long g_time_n[EXCMG_MAX_LEVELS][2];
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
// because each chunk re-reads four halo planes).  kind 0: one marched array (apply,
// residual); kind 1: two marched arrays (Bi-CG sweep A), which holds twice the column state
// and stays at TY = 8 to keep its registers below 256.
Geom choose_shape(int N, int bc, int kind) {
    const int n = N - 1;
    for (const ShapeOverride &o : g_shapes)
        if (o.N == N && o.kind == kind) return make_geom(n, bc, o.ty, std::max(1, std::min(o.zc, n)));
    const int ty = (kind == 0 && n >= 255) ? 16 : (n >= 24 ? 8 : 4);
    const int tiles_xy = ((n + kWave - 1) / kWave) * ((n + ty - 1) / ty);
    int zc = 4;
    for (int cand = 512; cand >= 4; cand >>= 1) {
        const int tz = (n + cand - 1) / cand;
        if ((long long)tiles_xy * tz >= 256) {
            zc = cand;
            break;
        }
    }
    zc = std::max(1, std::min(zc, n));
    return make_geom(n, bc, ty, zc);
}

void choose_shapes(Level &L, int bc) {
    L.g1 = choose_shape(L.N, bc, 0);
    L.g2 = choose_shape(L.N, bc, 1);
}

int check_sizes(int n_finest, int n_levels, int bc) {
    if (bc != 1 && bc != 2) return fail(EXCMG_EINVAL, "bc_kind must be 1 or 2 (got %d)", bc);
    if (n_levels < 3 || n_levels > EXCMG_MAX_LEVELS)
        return fail(EXCMG_EINVAL, "n_levels must be in 3..%d (got %d)", EXCMG_MAX_LEVELS,
                    n_levels);
    if (n_finest < 8 || n_finest > 2048) return fail(EXCMG_EINVAL, "n_finest out of range");
    const int N0 = n_finest >> (n_levels - 1);
    if (N0 < 2 || (N0 << (n_levels - 1)) != n_finest)
        return fail(EXCMG_EINVAL, "n_finest (%d) must be N0 * 2^(n_levels-1) with N0 >= 2",
                    n_finest);
    if (N0 > 8)
        return fail(EXCMG_EINVAL, "coarsest grid of %d cells is too large for DSOLVE (max 8)",
                    N0);
    return EXCMG_OK;
}

int setup(int n_finest, int n_levels, int bc) {
    CKR(check_sizes(n_finest, n_levels, bc));
    Ctx &c = g_ctx;
    if (c.ready && c.n_finest == n_finest && c.n_levels == n_levels && c.bc == bc)
        return EXCMG_OK;
    c.release();
    c.n_finest = n_finest;
    c.n_levels = n_levels;
    c.bc = bc;
    const int N0 = n_finest >> (n_levels - 1);
    c.lv.resize(n_levels);
    for (int l = 0; l < n_levels; l++) {
        Level &L = c.lv[l];
        L.index = l;
        L.N = N0 << l;
        L.n = L.N - 1;
        L.nu = (long long)L.n * L.n * L.n;
        L.nodes = (long long)(L.N + 1) * (L.N + 1) * (L.N + 1);
        choose_shapes(L, bc);
        CKR(L.b.ensure(L.nu * 8));
        CKR(L.x.ensure(L.nu * 8));
        CKR(L.u.ensure(L.nodes * 8));
    }
    const Level &F = c.lv.back();
    const size_t vb = (size_t)F.nu * 8;
    CKR(c.r.ensure(vb));
    CKR(c.rs.ensure(vb));
    CKR(c.p[0].ensure(vb));
    CKR(c.p[1].ensure(vb));
    CKR(c.ps[0].ensure(vb));
    CKR(c.ps[1].ensure(vb));
    CKR(c.q.ensure(vb));
    CKR(c.qs.ensure(vb));
    int maxblk = 4096 * 2;
    for (auto &L : c.lv) maxblk = std::max({maxblk, stencil_blocks(L.g1), stencil_blocks(L.g2)});
    CKR(c.part_a.ensure((size_t)maxblk * sizeof(Pair)));
    CKR(c.part_b.ensure((size_t)2 * 4096 * sizeof(Pair)));
    CKR(c.state.ensure(sizeof(BicgState)));
    CKR(c.scal.ensure(64 * sizeof(double)));
    CKR(c.info.ensure(64));
    const long long nz1 = (long long)(n_finest / 2 + 1) * (n_finest / 2 + 1) * (n_finest / 2 + 1);
    CKR(c.vz1.ensure((size_t)nz1 * 8));
    CKH(hipHostMalloc((void **)&c.host_state, sizeof(BicgState), hipHostMallocDefault));
    CKH(hipHostMalloc((void **)&c.host_scal, 64 * sizeof(double), hipHostMallocDefault));
    // Cholesky factors of the two direct levels (depend only on the grid and bc kind)
    for (int l = 0; l < 2; l++) {
        Level &L = c.lv[l];
        const int n = (int)L.nu;
        CKR(c.chol[l].ensure((size_t)n * n * 8));
        CKH(dense_assemble(L.N, bc, c.chol[l].as<double>(), g_stream));
        CKH(dense_cholesky(n, c.chol[l].as<double>(), c.info.as<int>(), g_stream));
        int info = 0;
        CKH(hipMemcpyAsync(&info, c.info.p, sizeof(int), hipMemcpyDeviceToHost, g_stream));
        CKH(hipStreamSynchronize(g_stream));
        if (info != 0)
            return fail(EXCMG_EBREAKDOWN, "Cholesky pivot %d of level %d not positive", info, l);
    }
    CKR(c.chol_y.ensure((size_t)c.lv[1].nu * 8));
    c.ready = true;
    return EXCMG_OK;
}

int need_ctx(int level) {
    if (!g_ctx.ready) return fail(EXCMG_EINVAL, "no context: call excmg_setup first");
    if (level < 0 || level >= g_ctx.n_levels)
        return fail(EXCMG_EINVAL, "level %d outside 0..%d", level, g_ctx.n_levels - 1);
    return EXCMG_OK;
}

// ------------------------------------------------------------------ reductions

int device_dot(long long n, const double *x, const double *y, double *out_dev, int slot) {
    Ctx &c = g_ctx;
    const int nb = vec_blocks(n);
    CKH(dot_partials<double>(n, x, y, c.part_b.as<Pair>(), nb, g_stream));
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

// r = b - A x on the level, and r.r into scal[slot]
int true_residual(const Level &L, const double *b, const double *x, double *r, int slot) {
    Ctx &c = g_ctx;
    CKH(stencil_residual<double>(L.g1, L.g1.ty, b, x, r, c.part_a.as<Pair>(), g_stream));
    CKH(reduce_to(c.scal.as<double>(), c.part_a.as<Pair>(), stencil_blocks(L.g1), slot,
                  g_stream));
    return EXCMG_OK;
}

// ------------------------------------------------------------------ Bi-CG (Algorithm 2)

// Iterations launched between two reads of the device state.
int poll_interval(long long nu) {
    long long k = (1LL << 21) / (nu > 0 ? nu : 1);
    if (k < 4) k = 4;
    if (k > 64) k = 64;
    return (int)k;
}

// Iterations of Algorithm 2 on level L after bicg_start: the Bi-CG vectors r, r*, p, p*, q, q*
// have type T, the iterate x type TX.  Sweep A forms p, p* and their products with A (and
// sigma), sweep B updates x, r, r* (and rho, r.r).  Every kernel returns at once when the
// run has stopped, so the host launches K iterations between two polls of the state.
template <typename TX, typename T>
int bicg_iterate(const Level &L, TX *x, BicgState &hs) {
    Ctx &c = g_ctx;
    BicgState *S = c.state.as<BicgState>();
    T *r = c.r.as<T>(), *rs = c.rs.as<T>(), *q = c.q.as<T>(), *qs = c.qs.as<T>();
    const int K = poll_interval(L.nu);
    const int nsb = stencil_blocks(L.g2);
    const int nvb = vec_blocks(L.nu);
    if (g_timing) CKR(ensure_events(4 * (size_t)K));
    long long j = 0;
    while (hs.status == kRunning) {
        const int it0 = hs.iter;
        for (int t = 0; t < K; t++, j++) {
            const int cur = (int)(j & 1), nxt = cur ^ 1;
            T *pn = c.p[nxt].as<T>(), *psn = c.ps[nxt].as<T>();
            if (g_timing) CKH(hipEventRecord(g_events[4 * t], g_stream));
            CKH(stencil_pair_direction<T>(L.g2, L.g2.ty, r, rs, c.p[cur].as<T>(),
                                          c.ps[cur].as<T>(), &S->beta, j == 0 ? 1 : 0, pn, psn,
                                          q, qs, c.part_a.as<Pair>(), &S->status, g_stream));
            if (g_timing) CKH(hipEventRecord(g_events[4 * t + 1], g_stream));
            CKH(bicg_alpha(S, c.part_a.as<Pair>(), nsb, g_stream));
            if (g_timing) CKH(hipEventRecord(g_events[4 * t + 2], g_stream));
            CKH((bicg_update<TX, T>(L.nu, S, x, pn, r, q, rs, qs, c.part_b.as<Pair>(), g_stream)));
            if (g_timing) CKH(hipEventRecord(g_events[4 * t + 3], g_stream));
            CKH(bicg_beta(S, c.part_b.as<Pair>(), nvb, g_stream));
        }
        CKR(read_state(hs));
        if (g_timing && L.index < EXCMG_MAX_LEVELS) {
            const int active = std::min(K, hs.iter - it0);  // launches that did work
            for (int t = 0; t < active; t++) {
                float a = 0.f, b = 0.f;
                CKH(hipEventElapsedTime(&a, g_events[4 * t], g_events[4 * t + 1]));
                CKH(hipEventElapsedTime(&b, g_events[4 * t + 2], g_events[4 * t + 3]));
                g_time_ms[L.index][0] += a;
                g_time_ms[L.index][1] += b;
                g_time_n[L.index][0]++;
                g_time_n[L.index][1]++;
            }
        }
    }
    return EXCMG_OK;
}

// One Bi-CG run from x (in place) on level L with right-hand side b.
int bicg_run(const Level &L, const double *b, double *x, double eps, int maxit, int *iters,
             double *rr_out, int *status_out) {
    Ctx &c = g_ctx;
    BicgState *S = c.state.as<BicgState>();
    double *r = c.r.as<double>(), *rs = c.rs.as<double>();
    // b.b and r_0 = b - A x_0, r*_0 = r_0
    CKR(device_dot(L.nu, b, b, (double *)&S->bb, 0));
    CKH(stencil_residual<double>(L.g1, L.g1.ty, b, x, r, c.part_a.as<Pair>(), g_stream));
    CKH((copy_convert<double, double>(L.nu, r, rs, g_stream)));
    CKH(bicg_start(S, c.part_a.as<Pair>(), stencil_blocks(L.g1), eps, maxit, g_stream));
    BicgState hs;
    CKR(read_state(hs));
    CKR((bicg_iterate<double, double>(L, x, hs)));
    if (iters) *iters = hs.iter;
    if (rr_out) *rr_out = hs.rr;
    if (status_out) *status_out = hs.status;
    return EXCMG_OK;
}

// Algorithm 1's while loop on one level.
int level_solve(const Level &L, const double *b, double *x, double eps, int maxit, int max_runs,
                excmg_level_stats *st) {
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
    while (!(rr <= thr)) {
        if (runs >= max_runs) {
            status = EXCMG_ENOCONV;
            break;
        }
        int it = 0, bst = 0;
        double rrr = 0.0;
        CKR(bicg_run(L, b, x, eps, maxit, &it, &rrr, &bst));
        total += it;
        runs++;
        CKR(true_residual(L, b, x, c.r.as<double>(), 2));
        CKH(hipMemcpyAsync(c.host_scal + 2, sc + 2, sizeof(double), hipMemcpyDeviceToHost,
                           g_stream));
        CKH(hipStreamSynchronize(g_stream));
        rr = c.host_scal[2];
        if (bst == kBreakdown) {
            status = EXCMG_EBREAKDOWN;
            break;
        }
    }
    if (st) {
        st->n = L.N;
        st->iterations = total;
        st->runs = runs;
        st->status = status;
        st->eps = eps;
        st->rel_residual = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
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
    CKH(dot_partials<float>(L.nu, r, r, c.part_b.as<Pair>(), nvb, g_stream));
    CKH(reduce_to((double *)&S->bb, c.part_b.as<Pair>(), nvb, 0, g_stream));
    CKH(bicg_start(S, c.part_b.as<Pair>(), nvb, inner_tol, maxit, g_stream));
    BicgState hs;
    CKR(read_state(hs));
    CKR((bicg_iterate<double, float>(L, u, hs)));
    if (iters) *iters = hs.iter;
    if (status_out) *status_out = hs.status;
    return EXCMG_OK;
}

// Iterative refinement on one level: r = b - A u in FP64 (rounded to FP32 for the inner
// solve), FP32 Bi-CG correction added to u in FP64, until ||b - A u||_2 <= eps ||b||_2 in
// FP64.  Stops early (EXCMG_ENOCONV) if an outer step fails to reduce the FP64 residual.
int level_solve_mixed(const Level &L, const double *b, double *u, double eps, int maxit,
                      int max_outer, double inner_tol, excmg_level_stats *st) {
    Ctx &c = g_ctx;
    double *sc = c.scal.as<double>();
    CKR(device_dot(L.nu, b, b, sc, 1));
    const int nrb = stencil_blocks(L.g1);
    int total = 0, outer = 0, status = EXCMG_OK;
    double bb = 0.0, rr = 0.0, prev = INFINITY;
    for (;;) {
        CKH(stencil_residual_cast(L.g1, L.g1.ty, b, u, c.r.as<float>(), c.rs.as<float>(),
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
        st->n = L.N;
        st->iterations = total;
        st->runs = outer;
        st->status = status;
        st->eps = eps;
        st->rel_residual = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    }
    return EXCMG_OK;
}

double level_tolerance(double tol, int i, int L) {
    double p = 1.0;
    for (int t = 0; t < L - i; t++) p *= 10.0;
    return tol / p;
}

// Algorithm 1.  f, g1, g2 are device node arrays of the finest grid.  Bi-CG levels run in
// FP64 or as FP32 Bi-CG inside FP64 iterative refinement (opts.precision).
int solve_cascade(const excmg_opts &o, const double *f, const double *g1, const double *g2,
                  double *u_out, double *ut_out, excmg_stats *st) {
    Ctx &c = g_ctx;
    const int nl = o.n_levels, Nf = o.n_finest;
    const int L = nl - 2;
    const int maxit = o.max_iters > 0 ? o.max_iters : 100000;
    const int max_runs = o.max_runs > 0 ? o.max_runs : 5;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 60;
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-4;
    const bool mixed = (o.precision == EXCMG_MIXED);
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
        CKH(rhs_assemble(Lv.N, c.bc, s, Nf, f, g1, g2, Lv.b.as<double>(), g_stream));
        if (l <= 1) {
            CKH(dense_solve((int)Lv.nu, c.chol[l].as<double>(), Lv.b.as<double>(),
                            Lv.x.as<double>(), c.chol_y.as<double>(), g_stream));
            ls.status = EXCMG_OK;
        } else {
            CKH(exp_finite(Lv.N, c.lv[l - 1].u.as<double>(), c.lv[l - 2].u.as<double>(),
                           c.vz1.as<double>(), Lv.u.as<double>(), g_stream));
            CKH(from_nodes(Lv.N, Lv.u.as<double>(), Lv.x.as<double>(), g_stream));
            const double eps = level_tolerance(o.tol, l - 1, L);
            if (mixed)
                CKR(level_solve_mixed(Lv, Lv.b.as<double>(), Lv.x.as<double>(), eps, maxit,
                                      max_outer, inner_tol, &ls));
            else
                CKR(level_solve(Lv, Lv.b.as<double>(), Lv.x.as<double>(), eps, maxit, max_runs,
                                &ls));
            if (ls.status != EXCMG_OK && worst == EXCMG_OK) worst = ls.status;
        }
        CKH(to_nodes<double>(Lv.N, s, Nf, Lv.x.as<double>(), g1, Lv.u.as<double>(), g_stream));
        CKH(hipEventRecord(evl1, g_stream));
        CKH(hipEventSynchronize(evl1));
        float ms = 0.f;
        CKH(hipEventElapsedTime(&ms, evl0, evl1));
        ls.ms = ms;
        if (st && l < EXCMG_MAX_LEVELS) st->level[l] = ls;
    }
    const Level &F = c.lv[nl - 1];
    if (ut_out) CKH(exp_true(Nf, F.u.as<double>(), c.lv[nl - 2].u.as<double>(), ut_out, g_stream));
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

}  // namespace

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
    const size_t nb = (size_t)(c.n_finest + 1) * (c.n_finest + 1) * (c.n_finest + 1) * 8;
    Arg af(f, nb), a1(g1, nb), a2(g2, nb), ab(b, L.nu * 8);
    CKR(af.in());
    CKR(a1.in());
    CKR(a2.in());
    CKR(ab.out());
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
    CKH(dense_solve((int)L.nu, c.chol[level].as<double>(), ab.p<double>(), ax.p<double>(),
                    c.chol_y.as<double>(), g_stream));
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
    CKR(bicg_run(L, ab.p<double>(), ax.p<double>(), eps, max_iters, &it, &r2, &status));
    CKR(ax.back());
    CKH(hipStreamSynchronize(g_stream));
    if (iters) *iters = it;
    if (rr) *rr = r2;
    if (status == kBreakdown) return fail(EXCMG_EBREAKDOWN, "Bi-CG breakdown");
    if (status == kNoConv) return fail(EXCMG_ENOCONV, "Bi-CG reached %d iterations", max_iters);
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
    CKR(level_solve(L, ab.p<double>(), ax.p<double>(), eps, max_iters, max_runs, &ls));
    CKR(ax.back());
    CKH(hipStreamSynchronize(g_stream));
    if (st) *st = ls;
    if (ls.status != EXCMG_OK) return fail(ls.status, "level solve stopped early");
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

int excmg_solve_ex(const excmg_opts *opts, const double *f, const double *g1, const double *g2,
                   double *u_out, double *ut_out, excmg_stats *st) {
    g_err[0] = 0;
    if (!opts) return fail(EXCMG_EINVAL, "NULL options");
    const excmg_opts o = *opts;
    if (!f || !g1 || !g2 || !u_out) return fail(EXCMG_EINVAL, "NULL array");
    if (!(o.tol > 0.0)) return fail(EXCMG_EINVAL, "tol must be positive");
    if (o.precision != EXCMG_FP64 && o.precision != EXCMG_MIXED)
        return fail(EXCMG_EINVAL, "precision %d not supported", o.precision);
    CKR(setup(o.n_finest, o.n_levels, o.bc_kind));
    const size_t nb = (size_t)(o.n_finest + 1) * (o.n_finest + 1) * (o.n_finest + 1) * 8;
    Arg af(f, nb), a1(g1, nb), a2(g2, nb), au(u_out, nb), at(ut_out, nb);
    CKR(af.in());
    CKR(a1.in());
    CKR(a2.in());
    CKR(au.out());
    if (ut_out) CKR(at.out());
    if (st) memset(st, 0, sizeof(*st));
    int rc = solve_cascade(o, af.p<double>(), a1.p<double>(), a2.p<double>(), au.p<double>(),
                        ut_out ? at.p<double>() : nullptr, st);
    if (rc != EXCMG_OK && rc != EXCMG_ENOCONV && rc != EXCMG_EBREAKDOWN) return rc;
    CKR(au.back());
    if (ut_out) CKR(at.back());
    CKH(hipStreamSynchronize(g_stream));
    return rc;
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
    if (!g_ctx.ready) return fail(EXCMG_EINVAL, "no context: call excmg_setup first");
    if (which < 0 || which > 4 || reps < 1) return fail(EXCMG_EINVAL, "bad sweep or reps");
    if (precision != EXCMG_FP64 && precision != EXCMG_MIXED)
        return fail(EXCMG_EINVAL, "bad precision");
    Ctx &c = g_ctx;
    const Level &L = c.lv.back();
    const size_t es = precision == EXCMG_FP64 ? 8 : 4;
    const size_t vb = (size_t)L.nu * es;
    DBuf *vecs[8] = {&c.r, &c.rs, &c.p[0], &c.p[1], &c.ps[0], &c.ps[1], &c.q, &c.qs};
    for (DBuf *v : vecs) CKH(hipMemsetAsync(v->p, 0, vb, g_stream));
    CKH(hipMemsetAsync(L.x.p, 0, (size_t)L.nu * 8, g_stream));
    CKH(hipMemsetAsync(L.b.p, 0, (size_t)L.nu * 8, g_stream));
    BicgState hs{};
    hs.status = kRunning;
    hs.rho = 1.0;
    hs.maxit = 1 << 30;
    CKH(hipMemcpyAsync(c.state.p, &hs, sizeof(hs), hipMemcpyHostToDevice, g_stream));
    BicgState *S = c.state.as<BicgState>();
    // algorithmic bytes per unknown of each sweep
    const double fp64_bytes[5] = {16, 24, 64, 72, 16};
    const double mixed_bytes[5] = {8, 24, 32, 44, 8};
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
                default: return copy_convert<double, double>(L.nu, r, c.q.as<double>(), g_stream);
            }
        }
        float *r = c.r.as<float>(), *rs = c.rs.as<float>();
        switch (which) {
            case 0: return stencil_apply<float>(L.g1, L.g1.ty, r, c.q.as<float>(), g_stream);
            case 1: return stencil_residual_cast(L.g1, L.g1.ty, L.b.as<double>(), L.x.as<double>(),
                                                 r, rs, c.part_a.as<Pair>(), g_stream);
            case 2: return stencil_pair_direction<float>(
                        L.g2, L.g2.ty, r, rs, c.p[0].as<float>(), c.ps[0].as<float>(), &S->beta,
                        0, c.p[1].as<float>(), c.ps[1].as<float>(), c.q.as<float>(),
                        c.qs.as<float>(), c.part_a.as<Pair>(), &S->status, g_stream);
            case 3: return bicg_update<double, float>(L.nu, S, L.x.as<double>(), c.p[1].as<float>(),
                                                      r, c.q.as<float>(), rs, c.qs.as<float>(),
                                                      c.part_b.as<Pair>(), g_stream);
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

int excmg_set_timing(int on) {
    g_timing = (on != 0);
    memset(g_time_ms, 0, sizeof(g_time_ms));
    memset(g_time_n, 0, sizeof(g_time_n));
    return EXCMG_OK;
}

int excmg_get_timing(int level, int sweep, double *ms_total, long long *launches) {
    if (level < 0 || level >= EXCMG_MAX_LEVELS || (sweep != 0 && sweep != 1))
        return fail(EXCMG_EINVAL, "bad level or sweep");
    if (ms_total) *ms_total = g_time_ms[level][sweep];
    if (launches) *launches = g_time_n[level][sweep];
    return EXCMG_OK;
}

int excmg_set_shape(int n, int kind, int ty, int zc) {
    g_err[0] = 0;
    if (n < 2) return fail(EXCMG_EINVAL, "n must be >= 2");
    if (kind != 0 && kind != 1) return fail(EXCMG_EINVAL, "kind must be 0 or 1");
    if (ty != 0 && ty != 4 && ty != 8 && ty != 16) return fail(EXCMG_EINVAL, "ty must be 4, 8 or 16");
    if (kind == 1 && ty == 16) return fail(EXCMG_EINVAL, "sweep A supports ty 4 or 8");
    if (ty != 0 && zc < 1) return fail(EXCMG_EINVAL, "zc must be >= 1");
    for (size_t i = 0; i < g_shapes.size(); i++)
        if (g_shapes[i].N == n && g_shapes[i].kind == kind) {
            g_shapes.erase(g_shapes.begin() + i);
            break;
        }
    if (ty != 0) g_shapes.push_back(ShapeOverride{n, kind, ty, zc});
    for (Level &L : g_ctx.lv) {
        if (L.N != n) continue;
        choose_shapes(L, g_ctx.bc);
        const size_t need = (size_t)std::max(stencil_blocks(L.g1), stencil_blocks(L.g2)) * sizeof(Pair);
        if (need > g_ctx.part_a.bytes) CKR(g_ctx.part_a.ensure(need));
    }
    return EXCMG_OK;
}

int excmg_get_shape(int n, int kind, int *ty, int *zc) {
    if (n < 2 || (kind != 0 && kind != 1)) return fail(EXCMG_EINVAL, "bad n or kind");
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
