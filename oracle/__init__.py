"""Plain FP64 CPU oracle of EXCMG for the 3D biharmonic equation (arXiv:1901.05118).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of the
benchmark are the only users.  The library under ``paper_1901_05118_amd`` never imports
this package and this package never imports the library.

The heavy primitives are plain C (``excmg_oracle.c``, compiled with gcc by ``build.py``);
the cascade driver of Algorithm 1 is written here in Python so that it reads like the
algorithm.  All arrays are numpy float64.  Node arrays have shape (N+1, N+1, N+1) indexed
[k, j, i] (x fastest in memory); interior vectors have (N-1)^3 entries in the same order.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_lib = None

OK, EINVAL, ENOMEM, ENOCONV, EBREAKDOWN = 0, -1, -2, -3, -4


class OracleError(RuntimeError):
    def __init__(self, name, code):
        super().__init__(f"oracle {name} failed with code {code}")
        self.code = code


def lib():
    """Load ``liboracle.so``; compile it first only if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        c_int, c_dbl, c_ll = ctypes.c_int, ctypes.c_double, ctypes.c_longlong
        sig = {
            "oracle_dot": (c_dbl, [c_ll, dp, dp]),
            "oracle_stencil_padded": (c_int, [c_int, dp, dp]),
            "oracle_apply": (c_int, [c_int, c_int, dp, dp]),
            "oracle_apply_transpose": (c_int, [c_int, c_int, dp, dp]),
            "oracle_residual": (c_int, [c_int, c_int, dp, dp, dp]),
            "oracle_rhs": (c_int, [c_int, c_int, dp, dp, dp, dp]),
            "oracle_dsolve": (c_int, [c_int, c_int, dp, dp]),
            "oracle_assemble": (c_int, [c_int, c_int, dp]),
            "oracle_bicg": (c_int, [c_int, c_int, dp, dp, dp, c_dbl, c_int, c_int, ip, dp]),
            "oracle_bicg_ex": (c_int, [c_int, c_int, dp, dp, dp, dp, dp, dp, c_dbl, c_int, c_int,
                                       ip, dp]),
            "oracle_diagonal": (c_int, [c_int, c_int, dp]),
            "oracle_level_solve": (c_int, [c_int, c_int, dp, dp, c_dbl, c_int, c_int, c_int,
                                           ip, ip, dp, dp]),
            "oracle_level_solve_ex": (c_int, [c_int, c_int, dp, dp, dp, c_dbl, c_int, c_int,
                                              c_int, ip, ip, dp, dp]),
            "oracle_exp_finite": (c_int, [c_int, dp, dp, dp]),
            "oracle2d_apply": (c_int, [c_int, c_int, dp, dp]),
            "oracle2d_residual": (c_int, [c_int, c_int, dp, dp, dp]),
            "oracle2d_rhs": (c_int, [c_int, c_int, dp, dp, dp, dp]),
            "oracle2d_assemble": (c_int, [c_int, c_int, dp]),
            "oracle2d_dsolve": (c_int, [c_int, c_int, dp, dp]),
            "oracle2d_bicg": (c_int, [c_int, c_int, dp, dp, c_dbl, c_int, ip, dp]),
            "oracle2d_level_solve": (c_int, [c_int, c_int, dp, dp, c_dbl, c_int, c_int, ip, ip,
                                             dp, dp]),
            "oracle2d_exp_finite": (c_int, [c_int, dp, dp, dp]),
            "oracle2d_exp_true": (c_int, [c_int, dp, dp, dp]),
            "oracle_exp_true": (c_int, [c_int, dp, dp, dp]),
            "oracle_threads": (c_int, []),
            "oracle_set_threads": (None, [c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(name, rc):
    if rc != OK:
        raise OracleError(name, rc)


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().oracle_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP threads of the oracle's loops (timing runs; results do not depend on
    the thread count)."""
    lib().oracle_set_threads(int(n))


def n_interior(N: int) -> int:
    return (N - 1) ** 3


# ----------------------------------------------------------------- primitives (C)

def dot(x, y) -> float:
    """Compensated (Dot2) inner product."""
    x, y = _f64(x).ravel(), _f64(y).ravel()
    return lib().oracle_dot(x.size, _p(x), _p(y))


def stencil_padded(N: int, P) -> np.ndarray:
    """Eq. (method1) at every interior node of a padded (N+3)^3 array (nodes -1..N+1)."""
    P = _f64(P)
    assert P.size == (N + 3) ** 3
    out = np.empty(n_interior(N))
    _check("stencil_padded", lib().oracle_stencil_padded(N, _p(P), _p(out)))
    return out


def apply(N: int, bc: int, x) -> np.ndarray:
    """y = A_h x (homogeneous boundary data), interior vectors."""
    x = _f64(x).ravel()
    y = np.empty(n_interior(N))
    _check("apply", lib().oracle_apply(N, bc, _p(x), _p(y)))
    return y


def apply_transpose(N: int, bc: int, x) -> np.ndarray:
    """y = A_h^T x by scattering each row of A_h (no symmetry assumed)."""
    x = _f64(x).ravel()
    y = np.empty(n_interior(N))
    _check("apply_transpose", lib().oracle_apply_transpose(N, bc, _p(x), _p(y)))
    return y


def residual(N: int, bc: int, b, x) -> np.ndarray:
    b, x = _f64(b).ravel(), _f64(x).ravel()
    r = np.empty(n_interior(N))
    _check("residual", lib().oracle_residual(N, bc, _p(b), _p(x), _p(r)))
    return r


def rhs(N: int, bc: int, f, g1, g2) -> np.ndarray:
    """f_h of eq. (sec) from level node arrays f, g1, g2."""
    f, g1, g2 = _f64(f), _f64(g1), _f64(g2)
    for a in (f, g1, g2):
        assert a.size == (N + 1) ** 3
    b = np.empty(n_interior(N))
    _check("rhs", lib().oracle_rhs(N, bc, _p(f), _p(g1), _p(g2), _p(b)))
    return b


def dsolve(N: int, bc: int, b) -> np.ndarray:
    """DSOLVE of Algorithm 1: dense Cholesky solve of A_h x = b."""
    b = _f64(b).ravel()
    x = np.empty(n_interior(N))
    _check("dsolve", lib().oracle_dsolve(N, bc, _p(b), _p(x)))
    return x


def assemble(N: int, bc: int) -> np.ndarray:
    """Dense A_h assembled from unit vectors (small N only)."""
    n = n_interior(N)
    A = np.empty((n, n))
    _check("assemble", lib().oracle_assemble(N, bc, _p(A)))
    return A


def bicg_ex(N: int, bc: int, b, x0, eps: float, maxit: int = 100000, shadow=None,
            bstar=None, xstar0=None, mdiag=None, literal_transpose: bool = False):
    """One run of Algorithm 2 with a diagonal preconditioner M = diag(mdiag) (None: M = I)
    and a chosen shadow system: r*_0 = shadow, or r*_0 = b* - A^T x*_0 with the dual iterate
    x* updated alongside (bstar, xstar0).  Returns (x, x* or None, iterations, recurrence
    r.r, code)."""
    b = _f64(b).ravel()
    x = _f64(x0).ravel().copy()
    sh = None if shadow is None else _f64(shadow).ravel()
    bs = None if bstar is None else _f64(bstar).ravel()
    xs = None if xstar0 is None else _f64(xstar0).ravel().copy()
    md = None if mdiag is None else _f64(mdiag).ravel()
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    rc = lib().oracle_bicg_ex(N, bc, _p(b), _p(x), _p(sh), _p(bs), _p(xs), _p(md), eps, maxit,
                              int(literal_transpose), ctypes.byref(it), ctypes.byref(rr))
    if rc not in (OK, ENOCONV):
        raise OracleError("bicg_ex", rc)
    return x, xs, it.value, rr.value, rc


def diagonal(N: int, bc: int) -> np.ndarray:
    """The diagonal of A_h, read off the operator (the Jacobi preconditioner)."""
    d = np.empty(n_interior(N))
    _check("diagonal", lib().oracle_diagonal(N, bc, _p(d)))
    return d


def bicg(N: int, bc: int, b, x0, eps: float, maxit: int = 100000, shadow=None,
         literal_transpose: bool = False):
    """One run of Algorithm 2 (M = I).  Returns (x, iterations, recurrence r.r, code).
    ``literal_transpose`` forms the shadow product by scattering the rows of A_h; otherwise
    it is formed as A_h p* (A_h is exactly symmetric)."""
    b = _f64(b).ravel()
    x = _f64(x0).ravel().copy()
    sh = None if shadow is None else _f64(shadow).ravel()
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    rc = lib().oracle_bicg(N, bc, _p(b), _p(x), _p(sh), eps, maxit, int(literal_transpose),
                           ctypes.byref(it), ctypes.byref(rr))
    if rc not in (OK, ENOCONV):
        raise OracleError("bicg", rc)
    return x, it.value, rr.value, rc


@dataclass
class LevelResult:
    N: int
    iters: int
    runs: int
    rr_true: float
    bb: float
    eps: float
    code: int


def level_solve(N: int, bc: int, b, x0, eps: float, maxit: int = 100000, max_runs: int = 5,
                literal_transpose: bool = False, mdiag=None):
    """The while loop of Algorithm 1 on one level (Bi-CG preconditioned by diag(mdiag) if
    given).  Returns (x, LevelResult)."""
    b = _f64(b).ravel()
    x = _f64(x0).ravel().copy()
    md = None if mdiag is None else _f64(mdiag).ravel()
    it, runs = ctypes.c_int(0), ctypes.c_int(0)
    rr, bb = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().oracle_level_solve_ex(N, bc, _p(b), _p(x), _p(md), eps, maxit, max_runs,
                                     int(literal_transpose), ctypes.byref(it), ctypes.byref(runs),
                                     ctypes.byref(rr), ctypes.byref(bb))
    if rc not in (OK, ENOCONV):
        raise OracleError("level_solve", rc)
    return x, LevelResult(N, it.value, runs.value, rr.value, bb.value, eps, rc)


def exp_finite(N: int, u1, u0) -> np.ndarray:
    """EXP_finite (Steps 1-5): node array on N cells from node arrays on N/2 and N/4."""
    u1, u0 = _f64(u1), _f64(u0)
    assert u1.size == (N // 2 + 1) ** 3 and u0.size == (N // 4 + 1) ** 3
    w = np.empty((N + 1, N + 1, N + 1))
    _check("exp_finite", lib().oracle_exp_finite(N, _p(u1), _p(u0), _p(w)))
    return w


def exp_true(N: int, uh, u2h) -> np.ndarray:
    """EXP_true: node array on N cells from node arrays on N and N/2 cells."""
    uh, u2h = _f64(uh), _f64(u2h)
    assert uh.size == (N + 1) ** 3 and u2h.size == (N // 2 + 1) ** 3
    ut = np.empty((N + 1, N + 1, N + 1))
    _check("exp_true", lib().oracle_exp_true(N, _p(uh), _p(u2h), _p(ut)))
    return ut


# ----------------------------------------------------------------- helpers (numpy)

def interior(u) -> np.ndarray:
    """Interior vector of a node array."""
    return np.ascontiguousarray(np.asarray(u)[1:-1, 1:-1, 1:-1]).ravel()


def to_nodes(N: int, x, g1) -> np.ndarray:
    """Node array with interior = x and boundary = g1 (a level node array)."""
    u = np.array(np.asarray(g1).reshape(N + 1, N + 1, N + 1), dtype=np.float64, copy=True)
    u[1:-1, 1:-1, 1:-1] = np.asarray(x).reshape(N - 1, N - 1, N - 1)
    return u


def inject(a, stride: int) -> np.ndarray:
    """Coarse-level node array sampled at every stride-th node of a finer one."""
    return np.ascontiguousarray(np.asarray(a)[::stride, ::stride, ::stride])


def norm2(e) -> float:
    """The tables' discrete L2 norm: root mean square over all (N+1)^3 nodes."""
    e = np.asarray(e, dtype=np.float64)
    return float(np.sqrt(np.mean(e * e)))


def norminf(e) -> float:
    return float(np.max(np.abs(e)))


def level_tolerance(tol: float, i: int, L: int) -> float:
    """eps_i = eps * 10^(i-L) (Algorithm 1), as tol divided by the exact power 10^(L-i)."""
    p = 1.0
    for _ in range(L - i):
        p *= 10.0
    return tol / p


def work_units(iters_coarse_to_fine) -> float:
    """Cost in work units: iterations on a level weighted by 8^-(levels below the finest)."""
    its = list(iters_coarse_to_fine)
    nl = len(its)
    return float(sum(it * 8.0 ** (-(nl - 1 - l)) for l, it in enumerate(its)))


# ------------------------------------------------------------ Algorithm 1 (driver)

@dataclass
class ExcmgResult:
    u: np.ndarray                       # finest FD solution, node array
    ut: np.ndarray                      # EXP_true extrapolated solution, node array
    levels: list = field(default_factory=list)   # LevelResult per Bi-CG level
    u_levels: list = field(default_factory=list)  # node arrays of every level (if kept)
    w_levels: list = field(default_factory=list)  # EXP_finite guesses (if kept; None on DSOLVE levels)


def level_sizes(n_finest: int, n_levels: int):
    if n_levels < 3:
        raise ValueError("n_levels must be >= 3 (two direct levels and one Bi-CG level)")
    N0 = n_finest >> (n_levels - 1)
    if N0 < 2 or (N0 << (n_levels - 1)) != n_finest:
        raise ValueError("n_finest must be N0 * 2^(n_levels-1) with N0 >= 2")
    return [N0 << l for l in range(n_levels)]


def excmg(n_finest: int, n_levels: int, bc: int, f, g1, g2, tol: float, *,
          maxit: int = 100000, max_runs: int = 5, keep_levels: bool = False,
          literal_transpose: bool = False, jacobi: bool = False) -> ExcmgResult:
    """Algorithm 1.  f, g1, g2 are node arrays on the finest grid; coarser levels take
    every 2^m-th node (injection).  Levels 0 and 1 use DSOLVE; level l >= 2 is the paper's
    i = l-1 with L = n_levels-2, starts from EXP_finite of the two previous levels and runs
    Bi-CG (preconditioned by diag(A_h) with ``jacobi``) until the true relative residual
    is at most eps_i."""
    sizes = level_sizes(n_finest, n_levels)
    M = n_finest + 1
    f = np.asarray(f, dtype=np.float64).reshape(M, M, M)
    g1 = np.asarray(g1, dtype=np.float64).reshape(M, M, M)
    g2 = np.asarray(g2, dtype=np.float64).reshape(M, M, M)
    L = n_levels - 2
    res = ExcmgResult(u=None, ut=None)
    u_prev2 = u_prev = None
    for l, N in enumerate(sizes):
        s = 1 << (n_levels - 1 - l)
        fl, g1l, g2l = inject(f, s), inject(g1, s), inject(g2, s)
        b = rhs(N, bc, fl, g1l, g2l)
        w = None
        if l <= 1:
            x = dsolve(N, bc, b)
        else:
            w = exp_finite(N, u_prev, u_prev2)
            eps = level_tolerance(tol, l - 1, L)
            x, st = level_solve(N, bc, b, interior(w), eps, maxit=maxit, max_runs=max_runs,
                                literal_transpose=literal_transpose,
                                mdiag=diagonal(N, bc) if jacobi else None)
            res.levels.append(st)
        u = to_nodes(N, x, g1l)
        if keep_levels:
            res.u_levels.append(u)
            res.w_levels.append(w)
        u_prev2, u_prev = u_prev, u
    res.u = u_prev
    res.ut = exp_true(n_finest, u_prev, u_prev2)
    return res


# ------------------------------------------------------------------ 2D (eq. bvp2d)

def n_interior_2d(N: int) -> int:
    return (N - 1) ** 2


def apply_2d(N: int, bc: int, x) -> np.ndarray:
    """y = A_h x for the 13-point scheme (homogeneous boundary data)."""
    x = _f64(x).ravel()
    y = np.empty(n_interior_2d(N))
    _check("apply_2d", lib().oracle2d_apply(N, bc, _p(x), _p(y)))
    return y


def residual_2d(N: int, bc: int, b, x) -> np.ndarray:
    b, x = _f64(b).ravel(), _f64(x).ravel()
    r = np.empty(n_interior_2d(N))
    _check("residual_2d", lib().oracle2d_residual(N, bc, _p(b), _p(x), _p(r)))
    return r


def rhs_2d(N: int, bc: int, f, g1, g2) -> np.ndarray:
    f, g1, g2 = _f64(f), _f64(g1), _f64(g2)
    for a in (f, g1, g2):
        assert a.size == (N + 1) ** 2
    b = np.empty(n_interior_2d(N))
    _check("rhs_2d", lib().oracle2d_rhs(N, bc, _p(f), _p(g1), _p(g2), _p(b)))
    return b


def assemble_2d(N: int, bc: int) -> np.ndarray:
    n = n_interior_2d(N)
    A = np.empty((n, n))
    _check("assemble_2d", lib().oracle2d_assemble(N, bc, _p(A)))
    return A


def dsolve_2d(N: int, bc: int, b) -> np.ndarray:
    b = _f64(b).ravel()
    x = np.empty(n_interior_2d(N))
    _check("dsolve_2d", lib().oracle2d_dsolve(N, bc, _p(b), _p(x)))
    return x


def bicg_2d(N: int, bc: int, b, x0, eps: float, maxit: int = 100000):
    b = _f64(b).ravel()
    x = _f64(x0).ravel().copy()
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    rc = lib().oracle2d_bicg(N, bc, _p(b), _p(x), eps, maxit, ctypes.byref(it), ctypes.byref(rr))
    if rc not in (OK, ENOCONV):
        raise OracleError("bicg_2d", rc)
    return x, it.value, rr.value, rc


def level_solve_2d(N: int, bc: int, b, x0, eps: float, maxit: int = 100000, max_runs: int = 5):
    b = _f64(b).ravel()
    x = _f64(x0).ravel().copy()
    it, runs = ctypes.c_int(0), ctypes.c_int(0)
    rr, bb = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().oracle2d_level_solve(N, bc, _p(b), _p(x), eps, maxit, max_runs, ctypes.byref(it),
                                    ctypes.byref(runs), ctypes.byref(rr), ctypes.byref(bb))
    if rc not in (OK, ENOCONV):
        raise OracleError("level_solve_2d", rc)
    return x, LevelResult(N, it.value, runs.value, rr.value, bb.value, eps, rc)


def exp_finite_2d(N: int, u1, u0) -> np.ndarray:
    u1, u0 = _f64(u1).ravel(), _f64(u0).ravel()
    w = np.empty((N + 1) ** 2)
    _check("exp_finite_2d", lib().oracle2d_exp_finite(N, _p(u1), _p(u0), _p(w)))
    return w.reshape(N + 1, N + 1)


def exp_true_2d(N: int, uh, u2h) -> np.ndarray:
    uh, u2h = _f64(uh).ravel(), _f64(u2h).ravel()
    ut = np.empty((N + 1) ** 2)
    _check("exp_true_2d", lib().oracle2d_exp_true(N, _p(uh), _p(u2h), _p(ut)))
    return ut.reshape(N + 1, N + 1)


def interior_2d(u) -> np.ndarray:
    u = np.asarray(u, dtype=np.float64)
    return np.ascontiguousarray(u[1:-1, 1:-1]).ravel()


def to_nodes_2d(N: int, x, g1) -> np.ndarray:
    u = np.array(np.asarray(g1, dtype=np.float64).reshape(N + 1, N + 1), copy=True)
    u[1:-1, 1:-1] = np.asarray(x).reshape(N - 1, N - 1)
    return u


def excmg_2d(n_finest: int, n_levels: int, bc: int, f, g1, g2, tol: float, *,
             maxit: int = 100000, max_runs: int = 5, keep_levels: bool = False) -> ExcmgResult:
    """Algorithm 1 for the 2D equation: DSOLVE on levels 0 and 1, EXP_finite guesses,
    Bi-CG level solves to eps_i, EXP_true on the finest grid."""
    sizes = level_sizes(n_finest, n_levels)
    M = n_finest + 1
    f = np.asarray(f, dtype=np.float64).reshape(M, M)
    g1 = np.asarray(g1, dtype=np.float64).reshape(M, M)
    g2 = np.asarray(g2, dtype=np.float64).reshape(M, M)
    L = n_levels - 2
    res = ExcmgResult(u=None, ut=None)
    u_prev2 = u_prev = None
    for l, N in enumerate(sizes):
        s = 1 << (n_levels - 1 - l)
        fl, g1l, g2l = f[::s, ::s], g1[::s, ::s], g2[::s, ::s]
        b = rhs_2d(N, bc, fl, g1l, g2l)
        w = None
        if l <= 1:
            x = dsolve_2d(N, bc, b)
        else:
            w = exp_finite_2d(N, u_prev, u_prev2)
            eps = level_tolerance(tol, l - 1, L)
            x, st = level_solve_2d(N, bc, b, interior_2d(w), eps, maxit=maxit, max_runs=max_runs)
            res.levels.append(st)
        u = to_nodes_2d(N, x, g1l)
        if keep_levels:
            res.u_levels.append(u)
            res.w_levels.append(w)
        u_prev2, u_prev = u_prev, u
    res.u = u_prev
    res.ut = exp_true_2d(n_finest, u_prev, u_prev2)
    return res
