// Internal interfaces between the kernels and the host driver of the EXCMG library.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace excmg {

// Geometry of a z-marched stencil launch on an interior grid of n^3 unknowns.
struct Geom {
    int n;                          // unknowns per axis (N - 1)
    int ty;                         // tile height (4, 8 or 16); tiles are 64 x ty columns
    int tiles_x, tiles_y, tiles_z;  // 64-wide x tiles, TY-high y tiles, ZC-deep z chunks
    int zc;
    int ntiles;
    double sgn;                     // fictitious-point sign: +1 first kind, -1 second kind
    int dim = 3;                    // 3: n^3 unknowns (z-marched); 2: n^2 unknowns (one plane)
    int ld = 0;                     // elements from one row of a vector to the next (>= n)
    i64 ps = 0;                     // elements from one plane to the next (n * ld)
    int tw = 64;                    // tile width: 64, or 128 for the two-point sweeps
};

// The same launch on vectors whose rows are ld elements apart (ld >= n).
inline Geom with_rows(Geom g, int ld) {
    g.ld = ld;
    g.ps = (i64)g.n * ld;
    return g;
}

// Row layout of a vector: rows of len elements, ld apart (positions whose column is len or
// more are padding).  The vector kernels walk the unknowns in contiguous order and address
// them through the layout, so they read and write no padding.  {1, 1}: contiguous.
struct Rows {
    int len = 1, ld = 1;
};

Geom make_geom(int n, int bc, int ty, int zc);
// Tiles of 128 x ty columns for the recomputing form's two-point FP32 sweeps, on rows ld
// apart (ld even); the ld stride is part of the geometry.  Returns tw = 0 when those sweeps
// cannot address the grid (the 32-bit byte offsets of a chunk of FP64 planes overflow).
Geom make_geom_wide(int n, int bc, int ty, int zc, int ld);
Geom make_geom_2d(int n, int bc, int ty);   // the 13-point scheme on an n x n plane

// Device-resident state of one Bi-CG run (Algorithm 2); all scalars FP64.
struct BicgState {
    double rho;      // r* . r of the current iterate
    double sigma;    // p* . A p
    double alpha;
    double beta;
    double rr;       // r . r (recurrence residual)
    double bb;       // b . b
    double thr;      // (eps * eps) * bb
    int iter;        // iterations done in this run
    int maxit;
    int status;      // 0 running, 1 converged, -3 iteration cap, -4 breakdown
    int poll_status; // the status as the host polls it: a window's closing check writes only
                     // this one when the run's last update is still pending (see step.hpp)
    double rho_slot[2];  // rho_j in slot j & 1 (steps with folded finalisations)
    double alpha_slot[2];  // alpha_j in slot j & 1 (update sweeps that apply the updates of
                           // two iterations to the iterate read alpha_{j-1} from it)
};

// A sweep that folds in the finalisation of the preceding sweep (see step.hpp).  state ==
// nullptr: not folded; the scalars come from the one-workgroup finalisation kernels.
struct StepLink {
    BicgState *state = nullptr;
    const Pair *part = nullptr;  // partials of the preceding sweep
    int count = 0;               // pairs per value
    int nv = 1;                  // values: 2 = (r*.r, r.r), 1 = r.r (CG) or sigma
    int par = 0;                 // parity of the iteration
    int poll_only = 0;           // end-of-window check: publish the decision for the host only
    int defer = 0;               // the sweep owes the iterate's update of the previous
                                 // iteration: a sweep A that stops the run publishes kStopping;
                                 // a sweep B that breaks down publishes its breakdown in
                                 // poll_status only, so that its workgroups that start later
                                 // still apply the update (the next check takes it from there)
};

// kStopping: the sweep A that stops a run while owing the iterate's update publishes this
// transient status, so its workgroups that start after the decision still apply their part
// of the update; the sweep B that follows replaces it by the final status (poll_status).
constexpr int kRunning = 0, kConverged = 1, kStopping = 2, kNoConv = -3, kBreakdown = -4;

// ---------------------------------------------------------------- stencil kernels

template <typename T>
hipError_t stencil_apply(const Geom &g, int ty, const T *x, T *y, hipStream_t st);

// r = b - A x and per-tile Dot2 partials of r.r (one per launched block)
template <typename T>
hipError_t stencil_residual(const Geom &g, int ty, const double *b, const T *x, T *r,
                            Pair *partials, hipStream_t st);

// Iterative-refinement residual: r64 = b - A u (FP64), r32 = rs32 = (float) r64, partials of
// r64.r64
hipError_t stencil_residual_cast(const Geom &g, int ty, const double *b, const double *u,
                                 float *r32, float *rs32, Pair *partials, hipStream_t st);

// Sweep A of a Bi-CG iteration: p_new = r + beta p_old, ps_new = rs + beta ps_old (or
// p_new = r, ps_new = rs when first), q = A p_new, qs = A ps_new, partials of ps_new . q.
template <typename T>
hipError_t stencil_pair_direction(const Geom &g, int ty, const T *r, const T *rs,
                                  const T *p_old, const T *ps_old, const double *beta_dev,
                                  int first, T *p_new, T *ps_new, T *q, T *qs, Pair *partials,
                                  const int *status, hipStream_t st, StepLink link = StepLink{});

// Sweep A with a diagonal preconditioner (entries d): p_new = r / d + beta p_old, likewise
// for the shadow direction (FP64)
hipError_t stencil_pair_direction_x(const Geom &g, int ty, const float *r, const float *rs,
                                   const float *p_old, const float *ps_old, const double *beta_dev,
                                   float *p_new, float *ps_new, float *q, float *qs,
                                   Pair *partials, const int *status, double *x,
                                   const double *alpha_dev, hipStream_t st, StepLink link);
// The recomputing form of a Bi-CG iteration (3D): sweep A marches p only
// (p_new, p*_new, partial of sigma = p*_new . A p_new); sweep B marches the stored p_new,
// p*_new again for q, q* and applies x += alpha p, r -= alpha q, r* -= alpha q* with the
// partials of r*.r and r.r (two values per workgroup, the layout of bicg_update's).
// Paired updates of the iterate (single-point sweeps): sweep B of an odd iteration leaves
// x untouched (xmode 1), sweep B of the next, even one applies both updates, x += alpha' p'
// then x += alpha p (xmode 2: p' = p_prev, alpha' from alpha_prev), and a sweep A that stops
// the run while x owes an update applies it on its own (owe_x: x += alpha p_old, alpha from
// alpha_owed).  xmode 0: x += alpha p in every sweep B.  down: the sweep marches each chunk
// from its top plane down (zmarch_down; single-point tiles).
template <typename T>
hipError_t stencil_dir_sigma(const Geom &g, int ty, const T *r, const T *rs, const T *p_old,
                             const T *ps_old, const double *beta_dev, int first, T *p_new,
                             T *ps_new, Pair *partials, const int *status, hipStream_t st,
                             StepLink link, double *owe_x = nullptr,
                             const double *alpha_owed = nullptr, bool down = false);
template <typename T>
hipError_t stencil_pair_update(const Geom &g, int ty, const T *p, const T *ps, double *x, T *r,
                               T *rs, Pair *partials, const int *status, const double *alpha_dev,
                               hipStream_t st, StepLink link, int xmode = 0,
                               const T *p_prev = nullptr, const double *alpha_prev = nullptr,
                               bool down = false);
// One sweep of each recomputing-form iteration marches downwards (same values), so that it
// starts on the planes the other sweep touched last, which the last-level cache still holds
// in part: sweep A with FP32 vectors, sweep B with FP64 vectors below this many unknowns.
constexpr long long kDownMaxUnknowns = 1LL << 26;
hipError_t stencil_pair_direction_m(const Geom &g, int ty, const double *r, const double *rs,
                                   const double *p_old, const double *ps_old, const double *d,
                                   const double *beta_dev, int first, double *p_new,
                                   double *ps_new, double *q, double *qs, Pair *partials,
                                   const int *status, hipStream_t st, StepLink link = StepLink{});

// CG sweep A: p_new = r + beta p_old (p_new = r when first), q = A p_new, partials of p_new . q
template <typename T>
hipError_t stencil_direction(const Geom &g, int ty, const T *r, const T *p_old,
                             const double *beta_dev, int first, T *p_new, T *q, Pair *partials,
                             const int *status, hipStream_t st, StepLink link = StepLink{});

inline int stencil_blocks(const Geom &g) { return xcd_grid(g.ntiles); }

// ---------------------------------------------------------------- vector kernels

int vec_blocks(long long n);
int update_blocks(long long n);   // workgroups (= partial pairs per value) of the Bi-CG updates

// x += (scale*alpha) p; r -= alpha q; rs -= alpha qs; partials of rs.r and r.r.  x may be
// held in higher precision than the other vectors (FP64 iterate, FP32 Bi-CG vectors).
template <typename TX, typename T>
hipError_t bicg_update(long long n, const BicgState *s, TX *x, const T *p, T *r, const T *q,
                       T *rs, const T *qs, Pair *partials, hipStream_t st,
                       StepLink link = StepLink{}, Rows rows = Rows{});

// CG sweep B: x += alpha p; r -= alpha q; partials of r.r
template <typename TX, typename T>
hipError_t cg_update(long long n, const BicgState *s, TX *x, const T *p, T *r, const T *q,
                     Pair *partials, hipStream_t st, StepLink link = StepLink{},
                     Rows rows = Rows{});
// the end-of-iteration checks of a folded step as a kernel of its own (one workgroup), run
// before the host reads the state
hipError_t step_check(StepLink link, hipStream_t st);
// partials of rs.r and r.r in the layout of bicg_update's (after a residual replacement);
// with d, of rs.(r / d) and r.r
template <typename T>
hipError_t rho_partials(long long n, const T *r, const T *rs, Pair *partials, hipStream_t st,
                        const T *d = nullptr, Rows rows = Rows{}, int nblocks = 0);
// Algorithm 2's sweep B with its options (FP64): d != NULL divides by the diagonal
// preconditioner in rho' = r*.(M^-1 r); xs != NULL also updates the dual iterate
// x* += alpha p* (ps)
hipError_t bicg_update_ex(long long n, const BicgState *s, double *x, const double *p,
                          double *r, const double *q, double *rs, const double *qs,
                          const double *d, double *xs, const double *ps, Pair *partials,
                          hipStream_t st, StepLink link = StepLink{});
// a run started from 2-valued partials: rho = first value (r*.M^-1 r), r.r = second
hipError_t bicg_start2(BicgState *s, const Pair *part, int count, double eps, int maxit,
                       hipStream_t st);
// diag(A_h): 42 + sgn * (faces the unknown is next to) on an n^3 grid, or 20 + sgn * (edges)
// on an n^2 plane (dim 2)
hipError_t operator_diagonal(int n, double sgn, double *d, hipStream_t st, int dim = 3);
// status = running (or iteration cap), thr = new recurrence threshold
hipError_t state_resume(BicgState *s, double thr, hipStream_t st);

// partials of x.y
template <typename T>
hipError_t dot_partials(long long n, const T *x, const T *y, Pair *partials, int nblocks,
                        hipStream_t st, Rows rows = Rows{});

// Row padding of an n^3 FP64 vector: dst (rows ld apart, padding set to 0) from src
// (contiguous), and back.
hipError_t pad_rows(int n, int ld, const double *src, double *dst, hipStream_t st);
hipError_t unpad_rows(int n, int ld, const double *src, double *dst, hipStream_t st);

template <typename TD, typename TS>
hipError_t copy_convert(long long n, const TS *src, TD *dst, hipStream_t st);

// finalisation kernels (one workgroup): merge `count` partials
hipError_t bicg_start(BicgState *s, const Pair *rr_part, int count, double eps, int maxit,
                      hipStream_t st);   // rr = rho = r.r (r* = r), bb precomputed
hipError_t reduce_to(double *out, const Pair *part, int count, int slot, hipStream_t st);

// ---------------------------------------------------------------- level kernels

// b = h^4 f - known terms, from finest-grid node arrays sampled at `stride`
hipError_t rhs_assemble(int N, int bc, int stride, int Nf, const double *f, const double *g1,
                        const double *g2, double *b, hipStream_t st);

// node array of N cells: interior from x (interior vector), boundary from g1 (finest
// node array sampled at stride)
template <typename T>
hipError_t to_nodes(int N, int stride, int Nf, const T *x, const double *g1, double *u,
                    hipStream_t st);

// interior vector from a node array
hipError_t from_nodes(int N, const double *u, double *x, hipStream_t st);

hipError_t exp_finite(int N, const double *u1, const double *u0, double *v_scratch, double *w,
                      hipStream_t st);
hipError_t exp_true(int N, const double *uh, const double *u2h, double *ut, hipStream_t st);

// DSOLVE of the two coarsest levels: Cholesky factor in lower-band storage (column c of
// the matrix at C[c (w+1) + d], d = 0..w, holding entry (c+d, c)), w = band_width(N, dim)
int band_width(int N, int dim);
hipError_t band_assemble(int N, int bc, int dim, int w, double *C, int *bad, hipStream_t st);
hipError_t band_cholesky(int n, int w, double *C, int *info, hipStream_t st);
hipError_t band_solve(int n, int w, const double *C, const double *b, double *x, hipStream_t st);

// the same level operations for the 2D equation (node arrays (N+1)^2, interior (N-1)^2)
hipError_t rhs_assemble_2d(int N, int bc, int stride, int Nf, const double *f, const double *g1,
                           const double *g2, double *b, hipStream_t st);
template <typename T>
hipError_t to_nodes_2d(int N, int stride, int Nf, const T *x, const double *g1, double *u,
                       hipStream_t st);
hipError_t from_nodes_2d(int N, const double *u, double *x, hipStream_t st);
hipError_t exp_finite_2d(int N, const double *u1, const double *u0, double *v_scratch, double *w,
                         hipStream_t st);
hipError_t exp_true_2d(int N, const double *uh, const double *u2h, double *ut, hipStream_t st);

// ---------------------------------------------------------------- batched Bi-CG

constexpr int kBatchTY = 8;            // default tile height of the batched sweep A (4 or 8)
constexpr int kMaxRuns = 256;          // systems per batch
constexpr long long kChunkGraph = 16384;      // unknowns per sweep-B item (phase kernels)
constexpr long long kChunkPersistent = 32768; // unknowns per sweep-B item (persistent kernel)

// One running Bi-CG system of a batch (device-resident table).
struct BatchRun {
    Geom g;                 // sweep-A geometry (ty: the batch's tile height)
    long long nu;           // unknowns
    int a_count, b_count;   // sweep-A tiles, sweep-B chunks
    long long chunk;        // unknowns per sweep-B chunk
    void *r, *rs, *p[2], *ps[2], *q, *qs;   // Bi-CG vectors (FP64 or FP32)
    double *x;              // iterate (FP64)
    BicgState *state;
    Pair *part_a;           // a_count partials of sigma
    Pair *part_b;           // 2 * b_count partials of rho and r.r
};

// Control block of the persistent step kernel (device).
struct BatchCtl {
    int queue;              // next item to claim
    int exit_count;         // workgroups that left the queue loop
    int epoch;              // launch number (advanced by the last workgroup out)
    int error;              // set if a bounded wait expired
    int n_a;                // items [0, n_a) are sweep-A items
    int n_items;
    int n_runs;
    int n_active;           // running systems (phase kernels)
    int active[kMaxRuns];   // their indices
    int a_done[kMaxRuns];
    int b_done[kMaxRuns];
    int alpha_epoch[kMaxRuns];
};

// One Bi-CG iteration of every running system as ONE launch of the persistent work-queue
// kernel (grid = resident workgroups).
template <typename T>
hipError_t batch_step(int ty, int grid, const BatchRun *runs, const int2 *items, BatchCtl *ctl,
                      hipStream_t st);
template <typename T>
hipError_t batch_step_grid(int ty, int *grid);
// Residual replacement of a stopped batched FP32 run (r, r* already replaced): rho from the
// `count` partials of r.r, beta = rho / rho of the previous iteration, threshold thr, and
// the run resumes with its search directions.
hipError_t batch_resume(BicgState *s, const Pair *part, int count, double thr, hipStream_t st);

// The same iteration as four phase launches (sweep A, alpha, sweep B, beta) over the work
// list in ctl; grid-stride, no inter-workgroup communication inside a launch.
template <typename T>
hipError_t batch_step_phases(int ty, const BatchRun *runs, const int2 *items, const BatchCtl *ctl,
                             hipStream_t st);

}  // namespace excmg
