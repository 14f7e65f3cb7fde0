// Launchers of the z-marched stencil kernels (device code in zmarch.hpp and zwide.hpp).
#include "plane2d.hpp"
#include "zmarch.hpp"
#include "zwide.hpp"

namespace excmg {

// ------------------------------------------------------------------ launchers

Geom make_geom(int n, int bc, int ty, int zc) {
    Geom g;
    g.n = n;
    g.ty = ty;
    g.tiles_x = (n + kWave - 1) / kWave;
    g.tiles_y = (n + ty - 1) / ty;
    g.zc = zc;
    g.tiles_z = (n + zc - 1) / zc;
    g.ntiles = g.tiles_x * g.tiles_y * g.tiles_z;
    g.sgn = (bc == 1) ? 1.0 : -1.0;
    g.ld = n;
    g.ps = (i64)n * n;
    return g;
}

Geom make_geom_wide(int n, int bc, int ty, int zc, int ld) {
    Geom g = with_rows(make_geom(n, bc, ty, zc), ld);
    g.tw = 2 * kWave;
    g.tiles_x = (n + g.tw - 1) / g.tw;
    g.ntiles = g.tiles_x * g.tiles_y * g.tiles_z;
    // a tile's descriptors start at its first plane; every byte offset of its accesses
    // (plane offset up to chunk + 3 planes on, plus an in-plane offset below one plane) must
    // stay below 2^32 for FP64 (the iterate of the update sweep)
    if (ld % 2 != 0 || (i64)((zc < n ? zc : n) + 4) * g.ps * 8 >= (1LL << 32)) g.tw = 0;
    return g;
}

Geom make_geom_2d(int n, int bc, int ty) {
    Geom g = make_geom(n, bc, ty, 1);
    g.zc = 1;
    g.tiles_z = 1;
    g.ntiles = g.tiles_x * g.tiles_y;
    g.dim = 2;
    return g;
}

template <int TY, typename T, class In, class Out, int NA>
static hipError_t launch(const Geom &g, const In &in, const Out &out, hipStream_t st) {
    dim3 block(kWave, TY);
    if (g.dim == 2)
        hipLaunchKernelGGL((plane2d<NA, TY, T, In, Out>), dim3(xcd_grid(g.ntiles)), block, 0, st,
                           g, in, out);
    else
        hipLaunchKernelGGL((zmarch<NA, TY, T, In, Out>), dim3(xcd_grid(g.ntiles)), block, 0, st,
                           g, in, out);
    return hipGetLastError();
}

// Launcher of epilogues that exist for 3D grids only (D: planes in flight).
template <int TY, typename T, class In, class Out, int NA, int D = 2>
static hipError_t launch3d(const Geom &g, const In &in, const Out &out, hipStream_t st) {
    hipLaunchKernelGGL((zmarch<NA, TY, T, In, Out, D>), dim3(xcd_grid(g.ntiles)), dim3(kWave, TY),
                       0, st, g, in, out);
    return hipGetLastError();
}
// The same launch marching every chunk from its top plane down (zmarch_down).
template <int TY, typename T, class In, class Out, int NA, int D>
static hipError_t launch3d_down(const Geom &g, const In &in, const Out &out, hipStream_t st) {
    hipLaunchKernelGGL((zmarch_down<NA, TY, T, In, Out, D>), dim3(xcd_grid(g.ntiles)),
                       dim3(kWave, TY), 0, st, g, in, out);
    return hipGetLastError();
}

// Planes in flight of the recomputing form's sweep A (one marched array, registers to spare):
// three (measured, FP32 at 512^3: 752 us with two, 733 us with three, four spill; FP64 at
// 256^3: 166 and 157 us, although three take 161 registers and lower the occupancy).
template <typename T>
constexpr int kSigmaDepth = 3;
// Planes in flight of its update sweep (two marched arrays plus the iterate and both
// residuals per output): three on tiles of up to 8 rows (512-thread workgroups, registers to
// spare), two on 16-row tiles (1024 threads, at most 128 registers).
constexpr int update_depth(int ty) { return ty >= 16 ? 2 : 3; }

#define EXCMG_DISPATCH_TY(TYV, ...)                                                          \
    switch (TYV) {                                                                           \
        case 4: { constexpr int TY = 4; __VA_ARGS__; } break;                              \
        case 8: { constexpr int TY = 8; __VA_ARGS__; } break;                              \
        case 16: { constexpr int TY = 16; __VA_ARGS__; } break;                            \
        default: return hipErrorInvalidValue;                                                \
    }

template <typename T>
hipError_t stencil_apply(const Geom &g, int ty, const T *x, T *y, hipStream_t st) {
    InPlain<T> in;
    in.x[0] = x;
    in.x[1] = x;
    OutApply<T> out;
    out.y = y;
    EXCMG_DISPATCH_TY(ty, return (launch<TY, T, InPlain<T>, OutApply<T>, 1>(g, in, out, st)));
    return hipSuccess;
}

template <typename T>
hipError_t stencil_residual(const Geom &g, int ty, const double *b, const T *x, T *r,
                            Pair *partials, hipStream_t st) {
    InPlain<T> in;
    in.x[0] = x;
    in.x[1] = x;
    OutResidual<T> out;
    out.b = b;
    out.r = r;
    out.partials = partials;
    out.acc = Pair{0.0, 0.0};
    EXCMG_DISPATCH_TY(ty, return (launch<TY, T, InPlain<T>, OutResidual<T>, 1>(g, in, out, st)));
    return hipSuccess;
}

hipError_t stencil_residual_cast(const Geom &g, int ty, const double *b, const double *u,
                                 float *r32, float *rs32, Pair *partials, hipStream_t st) {
    InPlain<double> in;
    in.x[0] = u;
    in.x[1] = u;
    OutResidualCast out;
    out.b = b;
    out.r32 = r32;
    out.rs32 = rs32;
    out.partials = partials;
    out.acc = Pair{0.0, 0.0};
    EXCMG_DISPATCH_TY(ty,
                      return (launch<TY, double, InPlain<double>, OutResidualCast, 1>(g, in, out, st)));
    return hipSuccess;
}

template <typename T>
hipError_t stencil_pair_direction(const Geom &g, int ty, const T *r, const T *rs,
                                  const T *p_old, const T *ps_old, const double *beta_dev,
                                  int first, T *p_new, T *ps_new, T *q, T *qs, Pair *partials,
                                  const int *status, hipStream_t st, StepLink link) {
    InDirection<T> in;
    in.link = link;
    in.r[0] = r;
    in.r[1] = rs;
    in.p[0] = p_old;
    in.p[1] = ps_old;
    in.beta_dev = beta_dev;
    in.first = first;
    in.beta = 0.0;
    OutPairApply<T> out;
    out.p_new[0] = p_new;
    out.p_new[1] = ps_new;
    out.q[0] = q;
    out.q[1] = qs;
    out.partials = partials;
    out.status = status;
    out.acc = Pair{0.0, 0.0};
    EXCMG_DISPATCH_TY(ty,
                      return (launch<TY, T, InDirection<T>, OutPairApply<T>, 2>(g, in, out, st)));
    return hipSuccess;
}

// Sweep A applying the previous iteration's update of the FP64 iterate (3D grids; see
// OutPairApplyX).
hipError_t stencil_pair_direction_x(const Geom &g, int ty, const float *r, const float *rs,
                                   const float *p_old, const float *ps_old, const double *beta_dev,
                                   float *p_new, float *ps_new, float *q, float *qs,
                                   Pair *partials, const int *status, double *x,
                                   const double *alpha_dev, hipStream_t st, StepLink link) {
    if (g.dim != 3) return hipErrorInvalidValue;
    InDirection<float> in;
    in.link = link;
    in.r[0] = r;
    in.r[1] = rs;
    in.p[0] = p_old;
    in.p[1] = ps_old;
    in.beta_dev = beta_dev;
    in.first = 0;
    in.beta = 0.0;
    OutPairApplyX<float> out;
    out.p_new[0] = p_new;
    out.p_new[1] = ps_new;
    out.q[0] = q;
    out.q[1] = qs;
    out.partials = partials;
    out.status = status;
    out.acc = Pair{0.0, 0.0};
    out.x = x;
    out.pold = p_old;
    out.alpha_dev = alpha_dev;
    out.alpha = 0.0;
    dim3 block(kWave, 1);
    switch (ty) {
        case 4:
            block.y = 4;
            hipLaunchKernelGGL((zmarch<2, 4, float, InDirection<float>, OutPairApplyX<float>>),
                               dim3(xcd_grid(g.ntiles)), block, 0, st, g, in, out);
            break;
        case 8:
            block.y = 8;
            hipLaunchKernelGGL((zmarch<2, 8, float, InDirection<float>, OutPairApplyX<float>>),
                               dim3(xcd_grid(g.ntiles)), block, 0, st, g, in, out);
            break;
        case 16:
            block.y = 16;
            hipLaunchKernelGGL((zmarch<2, 16, float, InDirection<float>, OutPairApplyX<float>>),
                               dim3(xcd_grid(g.ntiles)), block, 0, st, g, in, out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The recomputing form's two sweeps (3D grids; see OutDirSigma and OutPairUpdate).
// Planes in flight of the two-point sweeps (measured at 255^3: two 93 us, three 97 us).
constexpr int kWideDepth = 2;

#define EXCMG_DISPATCH_WIDE_TY(TYV, ...)                                                     \
    switch (TYV) {                                                                           \
        case 4: { constexpr int TY = 4; __VA_ARGS__; } break;                              \
        case 8: { constexpr int TY = 8; __VA_ARGS__; } break;                              \
        default: return hipErrorInvalidValue;                                                \
    }

template <typename T>
hipError_t stencil_dir_sigma(const Geom &g, int ty, const T *r, const T *rs, const T *p_old,
                             const T *ps_old, const double *beta_dev, int first, T *p_new,
                             T *ps_new, Pair *partials, const int *status, hipStream_t st,
                             StepLink link, double *owe_x, const double *alpha_owed, bool down) {
    if (g.dim != 3) return hipErrorInvalidValue;
    if (g.tw != kWave) {
        // paired updates and downward marches: single-point sweeps only
        if (owe_x || down) return hipErrorInvalidValue;
        if constexpr (sizeof(T) == 4) {
            if (g.tw != 2 * kWave) return hipErrorInvalidValue;
            WideDirection in;
            in.r = r;
            in.p = p_old;
            in.beta_dev = beta_dev;
            in.first = first;
            in.beta = 0.0;
            in.link = link;
            WideDirSigma out;
            out.p_new = p_new;
            out.ps_new = ps_new;
            out.rs = rs;
            out.ps_old = ps_old;
            out.partials = partials;
            out.status = status;
            out.beta = 0.0;
            out.first = first;
            out.acc = Pair{0.0, 0.0};
            EXCMG_DISPATCH_WIDE_TY(ty, hipLaunchKernelGGL(
                (zwide<1, TY, WideDirection, WideDirSigma, kWideDepth>),
                dim3(xcd_grid(g.ntiles)), dim3(kWave, TY), 0, st, g, in, out));
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    InDirection<T> in;
    in.link = link;
    in.r[0] = r;
    in.r[1] = r;
    in.p[0] = p_old;
    in.p[1] = p_old;
    in.beta_dev = beta_dev;
    in.first = first;
    in.beta = 0.0;
    OutDirSigma<T> out;
    out.p_new = p_new;
    out.ps_new = ps_new;
    out.rs = rs;
    out.ps_old = ps_old;
    out.partials = partials;
    out.status = status;
    out.beta = 0.0;
    out.first = first;
    out.acc = Pair{0.0, 0.0};
    if (owe_x) {
        if (!alpha_owed || first) return hipErrorInvalidValue;
        OutDirSigmaX<T> ox;
        static_cast<OutDirSigma<T> &>(ox) = out;
        ox.x = owe_x;
        ox.pold = p_old;
        ox.alpha_dev = alpha_owed;
        ox.alpha_owed = 0.0;
        if (down)
            EXCMG_DISPATCH_TY(ty, return (launch3d_down<TY, T, InDirection<T>, OutDirSigmaX<T>, 1,
                                                        kSigmaDepth<T>>(g, in, ox, st)));
        EXCMG_DISPATCH_TY(ty, return (launch3d<TY, T, InDirection<T>, OutDirSigmaX<T>, 1,
                                               kSigmaDepth<T>>(g, in, ox, st)));
        return hipSuccess;
    }
    if (down)
        EXCMG_DISPATCH_TY(ty, return (launch3d_down<TY, T, InDirection<T>, OutDirSigma<T>, 1,
                                                    kSigmaDepth<T>>(g, in, out, st)));
    EXCMG_DISPATCH_TY(ty, return (launch3d<TY, T, InDirection<T>, OutDirSigma<T>, 1, kSigmaDepth<T>>(
                              g, in, out, st)));
    return hipSuccess;
}

template <typename T>
hipError_t stencil_pair_update(const Geom &g, int ty, const T *p, const T *ps, double *x, T *r,
                               T *rs, Pair *partials, const int *status, const double *alpha_dev,
                               hipStream_t st, StepLink link, int xmode, const T *p_prev,
                               const double *alpha_prev, bool down) {
    if (g.dim != 3 || xmode < 0 || xmode > 2) return hipErrorInvalidValue;
    if (down && g.tw != kWave) return hipErrorInvalidValue;
    // paired updates: single-point tiles; with folded finalisations, mode 2 owes the update
    // (alpha_j in its slot, the breakdown rule of link_alpha)
    if (xmode != 0 && g.tw != kWave) return hipErrorInvalidValue;
    if (xmode == 2 && (!p_prev || !alpha_prev || (link.state && !link.defer)))
        return hipErrorInvalidValue;
    if (g.tw != kWave) {
        if constexpr (sizeof(T) == 4) {
            if (g.tw != 2 * kWave) return hipErrorInvalidValue;
            WidePlainAlpha in;
            in.x[0] = p;
            in.x[1] = ps;
            in.alpha_dev = alpha_dev;
            in.link = link;
            in.alpha = 0.0;
            WidePairUpdate out;
            out.x = x;
            out.r = r;
            out.rs = rs;
            out.partials = partials;
            out.status = status;
            out.alpha = 0.0;
            out.acc[0] = Pair{0.0, 0.0};
            out.acc[1] = Pair{0.0, 0.0};
            EXCMG_DISPATCH_WIDE_TY(ty, hipLaunchKernelGGL(
                (zwide<2, TY, WidePlainAlpha, WidePairUpdate, kWideDepth>),
                dim3(xcd_grid(g.ntiles)), dim3(kWave, TY), 0, st, g, in, out));
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    InPlainAlpha<T> in;
    in.x[0] = p;
    in.x[1] = ps;
    in.alpha_dev = alpha_dev;
    in.link = link;
    in.alpha = 0.0;
    auto fill = [&](auto &out) {
        out.x = x;
        out.r = r;
        out.rs = rs;
        out.partials = partials;
        out.status = status;
        out.alpha = 0.0;
        out.acc[0] = Pair{0.0, 0.0};
        out.acc[1] = Pair{0.0, 0.0};
        out.p_prev = p_prev;
        out.alpha_prev = 0.0;
    };
    if (xmode == 1) {
        OutPairUpdate<T, 1> out;
        fill(out);
        if (down)
            EXCMG_DISPATCH_TY(ty, return (launch3d_down<TY, T, InPlainAlpha<T>, OutPairUpdate<T, 1>,
                                                        2, update_depth(TY)>(g, in, out, st)));
        EXCMG_DISPATCH_TY(ty, return (launch3d<TY, T, InPlainAlpha<T>, OutPairUpdate<T, 1>, 2,
                                               update_depth(TY)>(g, in, out, st)));
        return hipSuccess;
    }
    if (xmode == 2) {
        OutPairUpdate2<T> out;
        fill(out);
        out.state = link.state;
        out.alpha_prev_dev = alpha_prev;
        if (down)
            EXCMG_DISPATCH_TY(ty, return (launch3d_down<TY, T, InPlainAlpha<T>, OutPairUpdate2<T>,
                                                        2, update_depth(TY)>(g, in, out, st)));
        EXCMG_DISPATCH_TY(ty, return (launch3d<TY, T, InPlainAlpha<T>, OutPairUpdate2<T>, 2,
                                               update_depth(TY)>(g, in, out, st)));
        return hipSuccess;
    }
    OutPairUpdate<T> out;
    fill(out);
    if (down)
        EXCMG_DISPATCH_TY(ty, return (launch3d_down<TY, T, InPlainAlpha<T>, OutPairUpdate<T>, 2,
                                                    update_depth(TY)>(g, in, out, st)));
    EXCMG_DISPATCH_TY(ty, return (launch3d<TY, T, InPlainAlpha<T>, OutPairUpdate<T>, 2,
                                           update_depth(TY)>(g, in, out, st)));
    return hipSuccess;
}
template hipError_t stencil_dir_sigma<float>(const Geom &, int, const float *, const float *,
                                             const float *, const float *, const double *, int,
                                             float *, float *, Pair *, const int *, hipStream_t,
                                             StepLink, double *, const double *, bool);
template hipError_t stencil_dir_sigma<double>(const Geom &, int, const double *, const double *,
                                              const double *, const double *, const double *,
                                              int, double *, double *, Pair *, const int *,
                                              hipStream_t, StepLink, double *, const double *, bool);
template hipError_t stencil_pair_update<float>(const Geom &, int, const float *, const float *,
                                               double *, float *, float *, Pair *, const int *,
                                               const double *, hipStream_t, StepLink, int,
                                               const float *, const double *, bool);
template hipError_t stencil_pair_update<double>(const Geom &, int, const double *,
                                                const double *, double *, double *, double *,
                                                Pair *, const int *, const double *, hipStream_t,
                                                StepLink, int, const double *, const double *, bool);

hipError_t stencil_pair_direction_m(const Geom &g, int ty, const double *r, const double *rs,
                                   const double *p_old, const double *ps_old, const double *d,
                                   const double *beta_dev, int first, double *p_new,
                                   double *ps_new, double *q, double *qs, Pair *partials,
                                   const int *status, hipStream_t st, StepLink link) {
    InDirectionM<double> in;
    in.link = link;
    in.r[0] = r;
    in.r[1] = rs;
    in.p[0] = p_old;
    in.p[1] = ps_old;
    in.d = d;
    in.beta_dev = beta_dev;
    in.first = first;
    in.beta = 0.0;
    OutPairApply<double> out;
    out.p_new[0] = p_new;
    out.p_new[1] = ps_new;
    out.q[0] = q;
    out.q[1] = qs;
    out.partials = partials;
    out.status = status;
    out.acc = Pair{0.0, 0.0};
    EXCMG_DISPATCH_TY(ty, return (launch<TY, double, InDirectionM<double>, OutPairApply<double>, 2>(
                              g, in, out, st)));
    return hipSuccess;
}

template hipError_t stencil_apply<double>(const Geom &, int, const double *, double *,
                                          hipStream_t);
template hipError_t stencil_apply<float>(const Geom &, int, const float *, float *, hipStream_t);
template hipError_t stencil_residual<double>(const Geom &, int, const double *, const double *,
                                             double *, Pair *, hipStream_t);
template hipError_t stencil_residual<float>(const Geom &, int, const double *, const float *,
                                            float *, Pair *, hipStream_t);
template <typename T>
hipError_t stencil_direction(const Geom &g, int ty, const T *r, const T *p_old,
                             const double *beta_dev, int first, T *p_new, T *q, Pair *partials,
                             const int *status, hipStream_t st, StepLink link) {
    InDirection<T> in;
    in.link = link;
    in.r[0] = r;
    in.r[1] = r;
    in.p[0] = p_old;
    in.p[1] = p_old;
    in.beta_dev = beta_dev;
    in.first = first;
    in.beta = 0.0;
    OutDirApply<T> out;
    out.p_new = p_new;
    out.q = q;
    out.partials = partials;
    out.status = status;
    out.acc = Pair{0.0, 0.0};
    EXCMG_DISPATCH_TY(ty, return (launch<TY, T, InDirection<T>, OutDirApply<T>, 1>(g, in, out, st)));
    return hipSuccess;
}
template hipError_t stencil_direction<double>(const Geom &, int, const double *, const double *,
                                              const double *, int, double *, double *, Pair *,
                                              const int *, hipStream_t, StepLink);
template hipError_t stencil_direction<float>(const Geom &, int, const float *, const float *,
                                             const double *, int, float *, float *, Pair *,
                                             const int *, hipStream_t, StepLink);

template hipError_t stencil_pair_direction<double>(const Geom &, int, const double *,
                                                   const double *, const double *,
                                                   const double *, const double *, int,
                                                   double *, double *, double *, double *,
                                                   Pair *, const int *, hipStream_t, StepLink);
template hipError_t stencil_pair_direction<float>(const Geom &, int, const float *,
                                                  const float *, const float *, const float *,
                                                  const double *, int, float *, float *,
                                                  float *, float *, Pair *, const int *,
                                                  hipStream_t, StepLink);

}  // namespace excmg
