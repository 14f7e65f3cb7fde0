"""Closed-form test problems: the paper's Problems 1-5 (Sec. 6) and the seeded families
used by the benchmark configurations.

Every problem provides u, f = Delta^2 u and the boundary derivatives on a tensor grid.
Hand-written closed forms are used where they are cheap to evaluate on large grids; a
SymPy-backed problem class derives everything symbolically for the rest (and the tests use
it to check the hand-written forms).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

PI = np.pi


class Problem:
    """Interface: evaluate u and f on the full node grid and boundary data on faces.

    ``x`` is the 1D coordinate array (i/N, i = 0..N).  Grids are indexed [k, j, i]."""

    name = "problem"

    def u_grid(self, x):
        raise NotImplementedError

    def f_grid(self, x):
        raise NotImplementedError

    def deriv_face(self, x, axis, side, order):
        """d^order u / d(coordinate of ``axis``)^order on the face where that coordinate is
        x[side]; returns a 2D array over the other two axes (in [k, j, i] order)."""
        raise NotImplementedError

    def u_face(self, x, axis, side):
        return self.deriv_face(x, axis, side, 0)

    def normal_data(self, x, axis, side, bc):
        if bc == 1:
            d = self.deriv_face(x, axis, side, 1)
            return -d if side == 0 else d  # outward normal derivative
        return self.deriv_face(x, axis, side, 2)


def _face_zyx(x, axis, side):
    c = x[side]
    a = x[:, None]   # slower of the two remaining axes
    b = x[None, :]   # faster of the two remaining axes
    if axis == 0:    # z = c, array over (y, x)
        return c, a, b
    if axis == 1:    # y = c, array over (z, x)
        return a, c, b
    return a, b, c   # x = c, array over (z, y)


class SeparableFamily(Problem):
    """u = exp(a x + b y + c z) + sum_m A_m sin(k1 pi x) sin(k2 pi y) sin(k3 pi z).

    Delta^2 exp(ax+by+cz) = (a^2+b^2+c^2)^2 exp(...); Delta^2 of a sine mode is
    pi^4 (k1^2+k2^2+k3^2)^2 times the mode.  ``exp_coef`` = None drops the exponential."""

    def __init__(self, exp_coef, modes, name="family"):
        self.exp_coef = None if exp_coef is None else tuple(float(v) for v in exp_coef)
        self.modes = [(float(A), int(k1), int(k2), int(k3)) for (A, k1, k2, k3) in modes]
        self.name = name

    # each term is a product of 1D factors; evaluate them by outer products
    def _terms(self):
        out = []
        if self.exp_coef is not None:
            a, b, c = self.exp_coef
            out.append(("exp", 1.0, (a, b, c)))
        for (A, k1, k2, k3) in self.modes:
            out.append(("sin", A, (k1 * PI, k2 * PI, k3 * PI)))
        return out

    @staticmethod
    def _fac(kind, w, t, order):
        if kind == "exp":
            return (w ** order) * np.exp(w * t)
        # derivatives of sin(w t)
        if order == 0:
            return np.sin(w * t)
        if order == 1:
            return w * np.cos(w * t)
        if order == 2:
            return -(w * w) * np.sin(w * t)
        raise ValueError(order)

    def _grid(self, x, scale_fn):
        M = x.size
        out = np.zeros((M, M, M))
        for kind, A, (wx, wy, wz) in self._terms():
            s = A * scale_fn(kind, wx, wy, wz)
            fx = self._fac(kind, wx, x, 0)
            fy = self._fac(kind, wy, x, 0)
            fz = self._fac(kind, wz, x, 0)
            out += s * (fz[:, None, None] * fy[None, :, None] * fx[None, None, :])
        return out

    def u_grid(self, x):
        return self._grid(x, lambda kind, wx, wy, wz: 1.0)

    def f_grid(self, x):
        def sc(kind, wx, wy, wz):
            s2 = wx * wx + wy * wy + wz * wz
            return s2 * s2  # the same for exp (w real) and sine modes (w = k pi)
        return self._grid(x, sc)

    def deriv_face(self, x, axis, side, order):
        z, y, xx = _face_zyx(x, axis, side)
        out = 0.0
        for kind, A, (wx, wy, wz) in self._terms():
            oz = order if axis == 0 else 0
            oy = order if axis == 1 else 0
            ox = order if axis == 2 else 0
            out = out + A * (self._fac(kind, wz, np.asarray(z), oz) *
                             self._fac(kind, wy, np.asarray(y), oy) *
                             self._fac(kind, wx, np.asarray(xx), ox))
        M = x.size
        return np.broadcast_to(out, (M, M)).copy()


class GridFunctions(Problem):
    """A problem given by numpy callables u(x,y,z), f(x,y,z) and partial derivatives."""

    def __init__(self, name, u, f, d1, d2):
        self.name = name
        self._u, self._f, self._d1, self._d2 = u, f, d1, d2

    def _mesh(self, x):
        return x[None, None, :], x[None, :, None], x[:, None, None]

    def u_grid(self, x):
        X, Y, Z = self._mesh(x)
        M = x.size
        return np.broadcast_to(self._u(X, Y, Z), (M, M, M)).astype(np.float64).copy()

    def f_grid(self, x):
        X, Y, Z = self._mesh(x)
        M = x.size
        return np.broadcast_to(self._f(X, Y, Z), (M, M, M)).astype(np.float64).copy()

    def deriv_face(self, x, axis, side, order):
        z, y, xx = _face_zyx(x, axis, side)
        X, Y, Z = np.asarray(xx, dtype=np.float64), np.asarray(y, dtype=np.float64), \
            np.asarray(z, dtype=np.float64)
        if order == 0:
            v = self._u(X, Y, Z)
        elif order == 1:
            v = self._d1[axis](X, Y, Z)
        else:
            v = self._d2[axis](X, Y, Z)
        M = x.size
        return np.broadcast_to(v, (M, M)).astype(np.float64).copy()


class SympyProblem(GridFunctions):
    """u given as a SymPy expression in x, y, z; f = Delta^2 u and the boundary
    derivatives are derived symbolically and lambdified."""

    def __init__(self, name, expr_fn, simplify=True):
        import sympy as sp
        x, y, z = sp.symbols("x y z", real=True)
        u = expr_fn(sp, x, y, z)
        lap = lambda e: sp.diff(e, x, 2) + sp.diff(e, y, 2) + sp.diff(e, z, 2)  # noqa: E731
        f = lap(lap(u))
        if simplify:
            f = sp.simplify(f)
        lam = lambda e: sp.lambdify((x, y, z), e, "numpy")  # noqa: E731
        # axis 0 is z, 1 is y, 2 is x (array order)
        d1 = [lam(sp.diff(u, z)), lam(sp.diff(u, y)), lam(sp.diff(u, x))]
        d2 = [lam(sp.diff(u, z, 2)), lam(sp.diff(u, y, 2)), lam(sp.diff(u, x, 2))]
        self.expr = u
        self.f_expr = f
        super().__init__(name, lam(u), lam(f), d1, d2)


# ----------------------------------------------------------------- the paper's problems

def _p1():
    c = lambda t: np.cos(2 * PI * t)  # noqa: E731
    s = lambda t: np.sin(2 * PI * t)  # noqa: E731
    u = lambda X, Y, Z: (1 - c(X)) * (1 - c(Y)) * (1 - c(Z))  # noqa: E731
    # Delta^2 u as printed in eq. (force1)
    f = lambda X, Y, Z: -16 * PI ** 4 * (c(X) - 4 * c(X) * c(Z) - 4 * c(X) * c(Y)  # noqa: E731
                                          + 9 * c(X) * c(Y) * c(Z) + c(Y) - 4 * c(Y) * c(Z)
                                          + c(Z))
    dx = lambda X, Y, Z: 2 * PI * s(X) * (1 - c(Y)) * (1 - c(Z))  # noqa: E731
    dy = lambda X, Y, Z: 2 * PI * s(Y) * (1 - c(X)) * (1 - c(Z))  # noqa: E731
    dz = lambda X, Y, Z: 2 * PI * s(Z) * (1 - c(X)) * (1 - c(Y))  # noqa: E731
    dxx = lambda X, Y, Z: 4 * PI ** 2 * c(X) * (1 - c(Y)) * (1 - c(Z))  # noqa: E731
    dyy = lambda X, Y, Z: 4 * PI ** 2 * c(Y) * (1 - c(X)) * (1 - c(Z))  # noqa: E731
    dzz = lambda X, Y, Z: 4 * PI ** 2 * c(Z) * (1 - c(X)) * (1 - c(Y))  # noqa: E731
    return GridFunctions("P1", u, f, [dz, dy, dx], [dzz, dyy, dxx])


def _p2():
    e = lambda X, Y, Z: np.exp(X * Y * Z)  # noqa: E731
    # eq. (force2)
    f = lambda x, y, z: np.exp(x * y * z) * (  # noqa: E731
        x**4 * y**4 + 2 * x**4 * y**2 * z**2 + x**4 * z**4 + 8 * x**3 * y * z
        + 2 * x**2 * y**4 * z**2 + 2 * x**2 * y**2 * z**4 + 4 * x**2 + 8 * x * y**3 * z
        + 8 * x * y * z**3 + y**4 * z**4 + 4 * y**2 + 4 * z**2)
    dx = lambda X, Y, Z: Y * Z * e(X, Y, Z)  # noqa: E731
    dy = lambda X, Y, Z: X * Z * e(X, Y, Z)  # noqa: E731
    dz = lambda X, Y, Z: X * Y * e(X, Y, Z)  # noqa: E731
    dxx = lambda X, Y, Z: (Y * Z) ** 2 * e(X, Y, Z)  # noqa: E731
    dyy = lambda X, Y, Z: (X * Z) ** 2 * e(X, Y, Z)  # noqa: E731
    dzz = lambda X, Y, Z: (X * Y) ** 2 * e(X, Y, Z)  # noqa: E731
    return GridFunctions("P2", e, f, [dz, dy, dx], [dzz, dyy, dxx])


def _p3():
    sh, ch = np.sinh, np.cosh
    u = lambda X, Y, Z: sh(X) * sh(Y) * sh(Z)  # noqa: E731
    # eq. (force3) prints f = u; Delta u = 3u, so Delta^2 u = 9u (the printed form is a typo)
    f = lambda X, Y, Z: 9.0 * sh(X) * sh(Y) * sh(Z)  # noqa: E731
    dx = lambda X, Y, Z: ch(X) * sh(Y) * sh(Z)  # noqa: E731
    dy = lambda X, Y, Z: sh(X) * ch(Y) * sh(Z)  # noqa: E731
    dz = lambda X, Y, Z: sh(X) * sh(Y) * ch(Z)  # noqa: E731
    return GridFunctions("P3", u, f, [dz, dy, dx], [u, u, u])


def _p4():
    u = lambda x, y, z: x * y * z * np.log(1 + x + y + z)  # noqa: E731
    # eq. (force4)
    f = lambda x, y, z: -(2 * (4 * x**3 + 8 * x**2 + 15 * x * y * z + 4 * x * y + 4 * x * z  # noqa: E731
                               + 4 * x + 4 * y**3 + 8 * y**2 + 4 * y * z + 4 * y + 4 * z**3
                               + 8 * z**2 + 4 * z)) / (x + y + z + 1) ** 4
    s = lambda x, y, z: 1 + x + y + z  # noqa: E731
    dx = lambda x, y, z: y * z * np.log(s(x, y, z)) + x * y * z / s(x, y, z)  # noqa: E731
    dy = lambda x, y, z: x * z * np.log(s(x, y, z)) + x * y * z / s(x, y, z)  # noqa: E731
    dz = lambda x, y, z: x * y * np.log(s(x, y, z)) + x * y * z / s(x, y, z)  # noqa: E731
    dxx = lambda x, y, z: 2 * y * z / s(x, y, z) - x * y * z / s(x, y, z) ** 2  # noqa: E731
    dyy = lambda x, y, z: 2 * x * z / s(x, y, z) - x * y * z / s(x, y, z) ** 2  # noqa: E731
    dzz = lambda x, y, z: 2 * x * y / s(x, y, z) - x * y * z / s(x, y, z) ** 2  # noqa: E731
    return GridFunctions("P4", u, f, [dz, dy, dx], [dzz, dyy, dxx])


def _p5():
    # the exponent's sign is kept as printed in eq. (test5); f is not printed and is
    # derived symbolically
    return SympyProblem("P5", lambda sp, x, y, z: -sp.exp(
        10 * (x - sp.Rational(1, 2)) ** 2 + 10 * (y - sp.Rational(1, 2)) ** 2
        + 10 * (z - sp.Rational(1, 5)) ** 2) * (x - x**2) * (y - y**2) * (z - z**2))


def paper_problem(k: int) -> Problem:
    """Test Problem k (1..5) of Sec. 6."""
    return {1: _p1, 2: _p2, 3: _p3, 4: _p4, 5: _p5}[k]()


def polynomial_problem(expr_fn, name="poly") -> SympyProblem:
    return SympyProblem(name, expr_fn)


# ------------------------------------------------------------ benchmark configurations

def family(rng, n_modes: int, kmax: int, name="family") -> SeparableFamily:
    """exp(a x + b y + c z) + sum of n_modes sine modes: a, b, c ~ U(-1, 1); integer
    wave numbers k1, k2, k3 uniform on 1..kmax; amplitudes ~ N(0, 1).  Draw order: a, b, c;
    then the (n_modes, 3) wave numbers; then the amplitudes."""
    abc = rng.uniform(-1.0, 1.0, size=3)
    ks = rng.integers(1, kmax + 1, size=(n_modes, 3))
    amps = rng.standard_normal(n_modes)
    modes = [(amps[m], ks[m, 0], ks[m, 1], ks[m, 2]) for m in range(n_modes)]
    return SeparableFamily(tuple(abc), modes, name=name)


def config_problem(c: int) -> Problem:
    """Manufactured solution of benchmark configuration c (1..4); config c is seeded
    with numpy.random.default_rng(1000 + c)."""
    if c == 1:
        # u = sin(pi x) sin(pi y) sin(pi z), f = Delta^2 u = 9 pi^4 u
        return SeparableFamily(None, [(1.0, 1, 1, 1)], name="config1")
    rng = np.random.default_rng(1000 + c)
    if c in (2, 3):
        return family(rng, 4, 4, name=f"config{c}")
    if c == 4:
        return family(rng, 8, 8, name="config4")
    raise ValueError(c)


@dataclass
class BatchItem:
    j: int
    N: int
    n_levels: int
    bc: int
    problem: Problem


def batch_problems(count: int = 64):
    """Configuration 5: problem j is seeded with default_rng(5000 + j); its finest grid is
    drawn uniformly from {32, 48, 64, 96, 128} cells; the coarsest grid has 4 cells (32, 64,
    128) or 3 cells (48, 96); first-kind data for even j, second kind for odd j; the
    solution family is that of configuration 2."""
    sizes = [32, 48, 64, 96, 128]
    out = []
    for j in range(count):
        rng = np.random.default_rng(5000 + j)
        N = int(sizes[int(rng.integers(0, len(sizes)))])
        N0 = 4 if N in (32, 64, 128) else 3
        n_levels = int(round(np.log2(N // N0))) + 1
        bc = 1 if j % 2 == 0 else 2
        out.append(BatchItem(j=j, N=N, n_levels=n_levels, bc=bc,
                             problem=family(rng, 4, 4, name=f"batch{j}")))
    return out
