"""ctypes binding of the C ABI in ``include/excmg.h`` (argument marshalling only).

Array arguments may be torch tensors (device or host) or numpy arrays; they must be
float64 and contiguous with the size the C function expects.  Device tensors are passed as
device pointers; host arrays are staged by the library.  Every function raises
``ExcmgError`` on a negative return code (``bicg``, ``level_solve`` and ``solve_ex`` return
the code together with their results instead, for the codes that still produce output)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "ExcmgError", "OK", "EINVAL", "ENOMEM", "ENOCONV", "EBREAKDOWN", "EHIP", "ENOCTX", "FP64",
    "MIXED", "EXIT_TOL", "EXIT_CAP", "EXIT_FLOOR", "EXIT_BREAKDOWN",
    "BICG", "CG", "RELIABLE", "RESTART", "PRECOND_NONE", "PRECOND_JACOBI", "bicg_ex", "diagonal",
    "lib_path", "load", "set_stream", "setup", "apply_stencil", "apply_operator", "rhs", "dsolve", "bicg",
    "level_solve", "exp_finite", "exp_finite_noalloc", "exp_true", "solve", "solve_ex", "profile_sweep",
    "set_shape", "get_shape", "set_timing", "get_timing", "autotune", "solve_batch",
    "autotune_batch", "get_batch_shape",
    "get_level_solution", "setup_2d", "solve_ex_2d", "exp_finite_2d", "exp_true_2d",
    "Problem",
    "last_error", "finalize",
    "LevelStats", "Stats",
]

OK, EINVAL, ENOMEM, ENOCONV, EBREAKDOWN, EHIP, ENOCTX = 0, -1, -2, -3, -4, -5, -6
EXIT_TOL, EXIT_CAP, EXIT_FLOOR, EXIT_BREAKDOWN = 0, 1, 2, 3
FP64, MIXED = 0, 1
BICG, CG = 0, 1
RELIABLE, RESTART = 0, 1
PRECOND_NONE, PRECOND_JACOBI = 0, 1
MAX_LEVELS = 16

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libexcmg.so")


class ExcmgError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} returned {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("n_finest", ctypes.c_int), ("n_levels", ctypes.c_int),
                ("bc_kind", ctypes.c_int), ("precision", ctypes.c_int),
                ("tol", ctypes.c_double), ("max_iters", ctypes.c_int),
                ("max_runs", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("batch_mode", ctypes.c_int),
                ("method", ctypes.c_int), ("refine", ctypes.c_int), ("precond", ctypes.c_int),
                ("fp32_min_unknowns", ctypes.c_int), ("row_pad", ctypes.c_int),
                ("recompute_min_unknowns", ctypes.c_int)]


class LevelStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("iterations", ctypes.c_int), ("runs", ctypes.c_int),
                ("status", ctypes.c_int), ("eps", ctypes.c_double),
                ("rel_residual", ctypes.c_double), ("ms", ctypes.c_double),
                ("floor", ctypes.c_double), ("exit", ctypes.c_int)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("level", LevelStats * MAX_LEVELS),
                ("total_ms", ctypes.c_double)]

    def levels(self):
        return [self.level[i].asdict() for i in range(self.n_levels)]


class Problem(ctypes.Structure):
    _fields_ = [("n_finest", ctypes.c_int), ("n_levels", ctypes.c_int), ("bc_kind", ctypes.c_int),
                ("f", ctypes.c_void_p), ("g1", ctypes.c_void_p), ("g2", ctypes.c_void_p),
                ("u_out", ctypes.c_void_p), ("ut_out", ctypes.c_void_p)]


_lib = None


def load():
    """Load the HIP library.  It must have been built (``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(lib_path):
        raise ImportError(f"{lib_path} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(lib_path)
    vp, dp, ip = ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)
    c_int, c_dbl = ctypes.c_int, ctypes.c_double
    sig = {
        "excmg_set_stream": (c_int, [vp]),
        "excmg_setup": (c_int, [c_int, c_int, c_int]),
        "excmg_apply_stencil": (c_int, [c_int, c_int, dp, dp]),
        "excmg_apply_operator": (c_int, [c_int, c_int, c_int, dp, dp]),
        "excmg_rhs": (c_int, [c_int, dp, dp, dp, dp]),
        "excmg_dsolve": (c_int, [c_int, dp, dp]),
        "excmg_bicg": (c_int, [c_int, dp, dp, c_dbl, c_int, ip, ctypes.POINTER(c_dbl)]),
        "excmg_level_solve": (c_int, [c_int, dp, dp, c_dbl, c_int, c_int,
                                      ctypes.POINTER(LevelStats)]),
        "excmg_exp_finite": (c_int, [c_int, dp, dp, dp]),
        "excmg_get_level_solution": (c_int, [c_int, dp]),
        "excmg_bicg_ex": (c_int, [c_int, dp, dp, dp, dp, dp, dp, c_dbl, c_int, ip,
                                  ctypes.POINTER(c_dbl)]),
        "excmg_diagonal": (c_int, [c_int, dp]),
        "excmg2d_setup": (c_int, [c_int, c_int, c_int]),
        "excmg2d_solve_ex": (c_int, [ctypes.POINTER(Opts), dp, dp, dp, dp, dp,
                                     ctypes.POINTER(Stats)]),
        "excmg2d_exp_finite": (c_int, [c_int, dp, dp, dp]),
        "excmg2d_exp_true": (c_int, [c_int, dp, dp, dp]),
        "excmg_exp_true": (c_int, [c_int, dp, dp, dp]),
        "excmg_solve": (c_int, [c_int, c_int, c_int, dp, dp, dp, c_dbl, dp]),
        "excmg_solve_ex": (c_int, [ctypes.POINTER(Opts), dp, dp, dp, dp, dp,
                                   ctypes.POINTER(Stats)]),
        "excmg_profile_sweep": (c_int, [c_int, c_int, c_int, ctypes.POINTER(c_dbl),
                                        ctypes.POINTER(c_dbl)]),
        "excmg_solve_batch": (c_int, [c_int, ctypes.POINTER(Problem), ctypes.POINTER(Opts),
                                      ctypes.POINTER(Stats)]),
        "excmg_autotune": (c_int, [c_int, c_int, c_int, c_int, ip, ip, ctypes.POINTER(c_dbl)]),
        "excmg_set_timing": (c_int, [c_int]),
        "excmg_get_timing": (c_int, [c_int, c_int, ctypes.POINTER(c_dbl),
                                     ctypes.POINTER(ctypes.c_longlong)]),
        "excmg_set_shape": (c_int, [c_int, c_int, c_int, c_int]),
        "excmg_get_shape": (c_int, [c_int, c_int, ip, ip]),
        "excmg_last_error": (ctypes.c_char_p, []),
        "excmg_finalize": (None, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return load().excmg_last_error().decode()


def _check(fn, rc):
    if rc != OK:
        raise ExcmgError(fn, rc, last_error())
    return rc


def _ptr(a, count=None, name="array"):
    """Address of a float64 contiguous torch tensor or numpy array (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise TypeError(f"{name}: need a contiguous float64 array")
        n = a.size
        p = a.ctypes.data
    else:
        import torch
        if not isinstance(a, torch.Tensor):
            raise TypeError(f"{name}: expected a torch tensor or numpy array")
        if a.dtype != torch.float64 or not a.is_contiguous():
            raise TypeError(f"{name}: need a contiguous float64 tensor")
        n = a.numel()
        p = a.data_ptr()
    if count is not None and n != count:
        raise ValueError(f"{name}: expected {count} values, got {n}")
    return ctypes.c_void_p(p)


def set_stream(stream=None):
    """Issue later work on ``stream`` (a torch.cuda.Stream, a raw hipStream_t, or None)."""
    h = None
    if stream is not None:
        h = getattr(stream, "cuda_stream", stream)
    _check("excmg_set_stream", load().excmg_set_stream(ctypes.c_void_p(h) if h else None))


def setup(n_finest: int, n_levels: int, bc_kind: int):
    _check("excmg_setup", load().excmg_setup(n_finest, n_levels, bc_kind))


def apply_stencil(level: int, transpose: int, x, y):
    _check("excmg_apply_stencil", load().excmg_apply_stencil(level, int(transpose), _ptr(x, name="x"),
                                                             _ptr(y, name="y")))


def apply_operator(n: int, bc_kind: int, transpose: int, x, y):
    _check("excmg_apply_operator", load().excmg_apply_operator(n, bc_kind, int(transpose),
                                                               _ptr(x, name="x"), _ptr(y, name="y")))


def rhs(level: int, f, g1, g2, b):
    _check("excmg_rhs", load().excmg_rhs(level, _ptr(f, name="f"), _ptr(g1, name="g1"),
                                         _ptr(g2, name="g2"), _ptr(b, name="b")))


def dsolve(level: int, b, x):
    _check("excmg_dsolve", load().excmg_dsolve(level, _ptr(b, name="b"), _ptr(x, name="x")))


def bicg(level: int, b, x, eps: float, max_iters: int = 100000):
    """One Bi-CG run from x (in place).  Returns (code, iterations, recurrence r.r)."""
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    rc = load().excmg_bicg(level, _ptr(b, name="b"), _ptr(x, name="x"), eps, max_iters,
                           ctypes.byref(it), ctypes.byref(rr))
    if rc not in (OK, ENOCONV, EBREAKDOWN):
        _check("excmg_bicg", rc)
    return rc, it.value, rr.value


def level_solve(level: int, b, x, eps: float, max_iters: int = 100000, max_runs: int = 5):
    """Algorithm 1's loop on one level.  Returns (code, stats dict)."""
    st = LevelStats()
    rc = load().excmg_level_solve(level, _ptr(b, name="b"), _ptr(x, name="x"), eps, max_iters,
                                  max_runs, ctypes.byref(st))
    if rc not in (OK, ENOCONV, EBREAKDOWN):
        _check("excmg_level_solve", rc)
    return rc, st.asdict()


def bicg_ex(level: int, b, x, eps: float, max_iters: int = 100000, shadow=None, bstar=None,
            xstar=None, mdiag=None):
    """One run of Algorithm 2 with its options (see excmg_bicg_ex).  x (and xstar) are
    updated in place.  Returns (code, iterations, recurrence r.r)."""
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    rc = load().excmg_bicg_ex(level, _ptr(b, name="b"), _ptr(x, name="x"),
                              _ptr(shadow, name="shadow"), _ptr(bstar, name="bstar"),
                              _ptr(xstar, name="xstar"), _ptr(mdiag, name="mdiag"), eps, max_iters,
                              ctypes.byref(it), ctypes.byref(rr))
    if rc not in (OK, ENOCONV, EBREAKDOWN):
        _check("excmg_bicg_ex", rc)
    return rc, it.value, rr.value


def diagonal(level: int, d):
    """diag(A_h) of a level of the current context into d."""
    _check("excmg_diagonal", load().excmg_diagonal(level, _ptr(d, name="d")))


def get_level_solution(level: int, u):
    """Node array of level `level` from the last solve on the current context."""
    _check("excmg_get_level_solution", load().excmg_get_level_solution(level, _ptr(u, name="u")))


def exp_finite(n: int, u1, u0, w):
    _check("excmg_exp_finite", load().excmg_exp_finite(n, _ptr(u1, name="u1"), _ptr(u0, name="u0"),
                                                       _ptr(w, name="w")))


def exp_finite_noalloc(n: int, u1, u0, w):
    """excmg_exp_finite_noalloc: EXP_finite with the library's fixed scratch array (device
    arrays only, n <= 256); queued on the library stream, not waited for."""
    _check("excmg_exp_finite_noalloc",
           load().excmg_exp_finite_noalloc(n, _ptr(u1, name="u1"), _ptr(u0, name="u0"),
                                           _ptr(w, name="w")))


def exp_true(n: int, uh, u2h, ut):
    _check("excmg_exp_true", load().excmg_exp_true(n, _ptr(uh, name="uh"), _ptr(u2h, name="u2h"),
                                                   _ptr(ut, name="ut")))


def solve(n_finest: int, n_levels: int, bc_kind: int, f, g1, g2, tol: float, u_out):
    _check("excmg_solve", load().excmg_solve(n_finest, n_levels, bc_kind, _ptr(f, name="f"),
                                             _ptr(g1, name="g1"), _ptr(g2, name="g2"), tol,
                                             _ptr(u_out, name="u_out")))


def solve_ex(n_finest: int, n_levels: int, bc_kind: int, f, g1, g2, tol: float, u_out,
             ut_out=None, precision: int = FP64, max_iters: int = 0, max_runs: int = 0,
             inner_tol: float = 0.0, max_outer: int = 0, method: int = BICG,
             refine: int = RELIABLE, precond: int = PRECOND_NONE, fp32_min_unknowns: int = 0,
             row_pad: int = 0, recompute_min_unknowns: int = 0):
    """Algorithm 1 with options.  Returns (code, Stats)."""
    o = Opts(n_finest, n_levels, bc_kind, precision, tol, max_iters, max_runs, inner_tol,
             max_outer, 0, method, refine, precond, fp32_min_unknowns, row_pad,
             recompute_min_unknowns)
    st = Stats()
    rc = load().excmg_solve_ex(ctypes.byref(o), _ptr(f, name="f"), _ptr(g1, name="g1"),
                               _ptr(g2, name="g2"), _ptr(u_out, name="u_out"),
                               _ptr(ut_out, name="ut_out"), ctypes.byref(st))
    if rc not in (OK, ENOCONV, EBREAKDOWN):
        _check("excmg_solve_ex", rc)
    return rc, st


def setup_2d(n_finest: int, n_levels: int, bc_kind: int):
    """Make the current context the 2D problem (eq. bvp2d) of n_finest^2 cells."""
    _check("excmg2d_setup", load().excmg2d_setup(n_finest, n_levels, bc_kind))


def solve_ex_2d(n_finest: int, n_levels: int, bc_kind: int, f, g1, g2, tol: float, u_out,
                ut_out=None, precision: int = FP64, max_iters: int = 0, max_runs: int = 0,
                inner_tol: float = 0.0, max_outer: int = 0, method: int = BICG,
                refine: int = RELIABLE, precond: int = PRECOND_NONE,
                fp32_min_unknowns: int = 0):
    """Algorithm 1 for the 2D equation.  Returns (code, Stats)."""
    o = Opts(n_finest, n_levels, bc_kind, precision, tol, max_iters, max_runs, inner_tol,
             max_outer, 0, method, refine, precond, fp32_min_unknowns, 0, 0)
    st = Stats()
    rc = load().excmg2d_solve_ex(ctypes.byref(o), _ptr(f, name="f"), _ptr(g1, name="g1"),
                                 _ptr(g2, name="g2"), _ptr(u_out, name="u_out"),
                                 _ptr(ut_out, name="ut_out"), ctypes.byref(st))
    if rc not in (OK, ENOCONV, EBREAKDOWN):
        _check("excmg2d_solve_ex", rc)
    return rc, st


def exp_finite_2d(n: int, u1, u0, w):
    _check("excmg2d_exp_finite", load().excmg2d_exp_finite(n, _ptr(u1, name="u1"),
                                                           _ptr(u0, name="u0"), _ptr(w, name="w")))


def exp_true_2d(n: int, uh, u2h, ut):
    _check("excmg2d_exp_true", load().excmg2d_exp_true(n, _ptr(uh, name="uh"),
                                                       _ptr(u2h, name="u2h"), _ptr(ut, name="ut")))


def profile_sweep(which: int, precision: int = FP64, reps: int = 20):
    """Mean ms per launch and algorithmic bytes per launch of a solver sweep on the finest
    level of the current context (see excmg.h)."""
    ms = ctypes.c_double(0.0)
    nb = ctypes.c_double(0.0)
    _check("excmg_profile_sweep", load().excmg_profile_sweep(which, precision, reps,
                                                             ctypes.byref(ms), ctypes.byref(nb)))
    return ms.value, nb.value


def solve_batch(problems, tol: float, precision: int = FP64, max_iters: int = 0,
                max_runs: int = 0, inner_tol: float = 0.0, max_outer: int = 0,
                persistent: bool = False, fp32_min_unknowns: int = 0, refine: int = RELIABLE):
    """Solve independent problems together.  ``problems`` is a list of dicts with keys
    n_finest, n_levels, bc_kind, f, g1, g2, u_out and optionally ut_out.  Returns
    (code, list of Stats)."""
    n = len(problems)
    arr = (Problem * n)()
    for i, p in enumerate(problems):
        arr[i] = Problem(p["n_finest"], p["n_levels"], p["bc_kind"],
                         _ptr(p["f"], name="f"), _ptr(p["g1"], name="g1"), _ptr(p["g2"], name="g2"),
                         _ptr(p["u_out"], name="u_out"), _ptr(p.get("ut_out"), name="ut_out"))
    o = Opts(0, 0, 0, precision, tol, max_iters, max_runs, inner_tol, max_outer,
             1 if persistent else 0, BICG, refine, PRECOND_NONE, fp32_min_unknowns)
    st = (Stats * n)()
    rc = load().excmg_solve_batch(n, arr, ctypes.byref(o), st)
    if rc not in (OK, ENOCONV, EBREAKDOWN):
        _check("excmg_solve_batch", rc)
    return rc, list(st)


def autotune(n: int, kind: int, precision: int = FP64, reps: int = 5):
    """Time every tile shape of a stencil kernel on a grid of n cells and keep the fastest.
    Returns (ty, zc, ms per launch)."""
    ty, zc = ctypes.c_int(0), ctypes.c_int(0)
    ms = ctypes.c_double(0.0)
    _check("excmg_autotune", load().excmg_autotune(n, kind, precision, reps, ctypes.byref(ty),
                                                   ctypes.byref(zc), ctypes.byref(ms)))
    return ty.value, zc.value, ms.value


def autotune_batch(problems, precision: int = FP64, reps: int = 3, fp32_min_unknowns: int = 0):
    """Tune the batched sweep A's tile height and per-size z-chunks on this batch (see
    excmg_autotune_batch).  ``problems`` as for solve_batch.  Returns (ty, sum over the grid
    sizes of the best step time of that size's systems, in ms)."""
    n = len(problems)
    arr = (Problem * n)()
    for i, p in enumerate(problems):
        arr[i] = Problem(p["n_finest"], p["n_levels"], p["bc_kind"],
                         _ptr(p["f"], name="f"), _ptr(p["g1"], name="g1"), _ptr(p["g2"], name="g2"),
                         _ptr(p["u_out"], name="u_out"), _ptr(p.get("ut_out"), name="ut_out"))
    o = Opts(0, 0, 0, precision, 1e-8, 0, 0, 0.0, 0, 0, BICG, RESTART, PRECOND_NONE,
             fp32_min_unknowns)
    ty = ctypes.c_int(0)
    ms = ctypes.c_double(0.0)
    _check("excmg_autotune_batch", load().excmg_autotune_batch(n, arr, ctypes.byref(o), reps,
                                                               ctypes.byref(ty),
                                                               ctypes.byref(ms)))
    return ty.value, ms.value


def get_batch_shape(n: int, precision: int = FP64):
    """(tile height, z-chunk) of the batched sweep A on grids of n cells."""
    ty, zc = ctypes.c_int(0), ctypes.c_int(0)
    _check("excmg_get_batch_shape", load().excmg_get_batch_shape(n, precision, ctypes.byref(ty),
                                                                 ctypes.byref(zc)))
    return ty.value, zc.value


def set_timing(on: bool):
    """Bracket every later Bi-CG sweep with device events (and reset the totals)."""
    _check("excmg_set_timing", load().excmg_set_timing(int(bool(on))))


def get_timing(level: int, sweep: int):
    """(total ms, launches) of sweep 0 (A), 1 (B), 2 (A with the deferred x update), 3 (B
    leaving x to the next iteration) or 4 (B applying two iterations' x updates) on a level
    since set_timing(True)."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_longlong(0)
    _check("excmg_get_timing", load().excmg_get_timing(level, sweep, ctypes.byref(ms),
                                                       ctypes.byref(n)))
    return ms.value, n.value


def set_shape(n: int, kind: int, ty: int, zc: int):
    """Tile shape (64 x ty columns, zc planes per chunk) for grids of n cells; kind 0 = the
    one-array stencil kernels, 1 / 2 = Bi-CG sweep A in FP64 / FP32; ty=0 restores the
    default."""
    _check("excmg_set_shape", load().excmg_set_shape(n, kind, ty, zc))


def get_shape(n: int, kind: int):
    ty, zc = ctypes.c_int(0), ctypes.c_int(0)
    _check("excmg_get_shape", load().excmg_get_shape(n, kind, ctypes.byref(ty),
                                                     ctypes.byref(zc)))
    return ty.value, zc.value


def finalize():
    if _lib is not None:
        _lib.excmg_finalize()
