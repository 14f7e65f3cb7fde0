"""Pins of the oracle's discrete operator, right-hand side and direct solver (Sec. 2).

Each check is against something other than the oracle itself: exact polynomial identities,
an independently assembled Kronecker-product matrix, the discrete sine eigenpairs, numpy's
dense solver, and manufactured solutions that the scheme must reproduce exactly."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sps

import oracle as O
from manufactured import make_arrays, polynomial_problem


def _padded_poly(N, coef_fn):
    """Values of a polynomial on nodes -1..N+1 (padded layout, x fastest)."""
    t = np.arange(-1, N + 2) / N
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    return coef_fn(X, Y, Z)


def _random_poly(rng, degree):
    """Random polynomial of total degree <= degree with its bilaplacian (both numpy)."""
    import sympy as sp
    x, y, z = sp.symbols("x y z")
    expr = 0
    for a, b, c in itertools.product(range(degree + 1), repeat=3):
        if a + b + c <= degree:
            expr += int(rng.integers(-3, 4)) * x**a * y**b * z**c
    lap = lambda e: sp.diff(e, x, 2) + sp.diff(e, y, 2) + sp.diff(e, z, 2)  # noqa: E731
    f = lap(lap(expr))
    fu = sp.lambdify((x, y, z), expr, "numpy")
    ff = sp.lambdify((x, y, z), f, "numpy")
    return (lambda X, Y, Z: fu(X, Y, Z) + 0 * X), (lambda X, Y, Z: ff(X, Y, Z) + 0 * X)


@pytest.mark.parametrize("seed", range(4))
def test_interior_stencil_exact_on_degree5(seed):
    """Eq. (method1) equals h^4 Delta^2 u exactly for polynomials of total degree <= 5."""
    rng = np.random.default_rng(seed)
    u, f = _random_poly(rng, 5)
    N = 8
    P = _padded_poly(N, u)
    got = O.stencil_padded(N, P.ravel())
    t = np.arange(1, N) / N
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    ref = f(X, Y, Z).ravel() / N**4
    scale = np.abs(P).max() + np.abs(ref).max()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)


def test_interior_stencil_not_exact_on_degree6():
    """The exactness above is not vacuous: x^6 leaves an O(h^2) truncation term."""
    N = 8
    P = _padded_poly(N, lambda X, Y, Z: X**6 + 0 * Y)
    got = O.stencil_padded(N, P.ravel())
    t = np.arange(1, N) / N
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    ref = (360 * X**2).ravel() / N**4
    assert np.abs(got - ref).max() > 1e-3 * np.abs(ref).max()


def _lap_dirichlet(N):
    n = N - 1
    L1 = sps.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1])
    I = sps.identity(n)
    return (sps.kron(sps.kron(I, I), L1) + sps.kron(sps.kron(I, L1), I) +
            sps.kron(sps.kron(L1, I), I)).tocsr()


def _closed_form(N, bc):
    """A_h = (L_D)^2 + 2 diag(m) (first kind) or (L_D)^2 (second kind), where L_D is the
    7-point Dirichlet Laplacian and m counts the faces a node is next to (on a grid with
    N = 2 the single unknown is next to all six)."""
    L = _lap_dirichlet(N)
    A = (L @ L).toarray()
    if bc == 1:
        n = N - 1
        e = np.zeros(n)
        e[0] += 1
        e[-1] += 1
        m = (e[None, None, :] + e[None, :, None] + e[:, None, None]).ravel()
        A = A + 2 * np.diag(m)
    return A


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 8])
@pytest.mark.parametrize("bc", [1, 2])
def test_operator_closed_form_and_symmetry(N, bc):
    A = O.assemble(N, bc)
    np.testing.assert_array_equal(A, _closed_form(N, bc))
    np.testing.assert_array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0  # symmetric positive definite


@pytest.mark.parametrize("N", [3, 6, 9])
@pytest.mark.parametrize("bc", [1, 2])
def test_literal_transpose_matches_assembled(N, bc):
    A = O.assemble(N, bc)
    rng = np.random.default_rng(N)
    x = rng.standard_normal(A.shape[0])
    np.testing.assert_allclose(O.apply_transpose(N, bc, x), A.T @ x, rtol=0,
                               atol=1e-12 * np.abs(x).max())
    np.testing.assert_allclose(O.apply(N, bc, x), A @ x, rtol=0, atol=1e-12 * np.abs(x).max())


@pytest.mark.parametrize("N", [16, 24])
def test_second_kind_sine_eigenpairs(N):
    """Second kind: A_h v = lambda v for v = sin(p pi i/N) sin(q pi j/N) sin(r pi k/N),
    lambda = (sum over p, q, r of 4 sin^2(a pi / 2N))^2."""
    t = np.arange(1, N)
    for (p, q, r) in [(1, 1, 1), (2, 5, 3), (N - 1, 1, N // 2)]:
        v = (np.sin(r * np.pi * t / N)[:, None, None] * np.sin(q * np.pi * t / N)[None, :, None]
             * np.sin(p * np.pi * t / N)[None, None, :]).ravel()
        lam = sum(4 * np.sin(a * np.pi / (2 * N)) ** 2 for a in (p, q, r)) ** 2
        np.testing.assert_allclose(O.apply(N, 2, v), lam * v, rtol=0, atol=1e-11 * lam)


@pytest.mark.parametrize("N", [2, 4, 6])
@pytest.mark.parametrize("bc", [1, 2])
def test_dsolve_matches_numpy(N, bc):
    rng = np.random.default_rng(100 + N)
    b = rng.standard_normal((N - 1) ** 3)
    x = O.dsolve(N, bc, b)
    ref = np.linalg.solve(_closed_form(N, bc), b)
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


POLY_FIRST = lambda sp, x, y, z: x**2 * y**2 * z + x * y * z**2 + 3 * y**2  # noqa: E731
POLY_SECOND = lambda sp, x, y, z: x**3 * y**2 + x * z**3 + y**3 * z  # noqa: E731


@pytest.mark.parametrize("N", [4, 6, 8])
@pytest.mark.parametrize("bc,expr", [(1, POLY_FIRST), (2, POLY_SECOND)])
def test_rhs_and_reflection_reproduce_polynomials(N, bc, expr):
    """The reflection formulas are exact for quadratics (first kind) or cubics (second
    kind) in the normal variable, and eq. (method1) is exact to total degree 5, so the
    discrete solution equals u at every node."""
    arr = make_arrays(polynomial_problem(expr), N, bc, poison=True)
    b = O.rhs(N, bc, arr.f, arr.g1, arr.g2)
    x = O.dsolve(N, bc, b)
    ref = O.interior(arr.u)
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-11 * np.abs(arr.u).max())


@pytest.mark.parametrize("bc", [1, 2])
def test_polynomial_pin_is_sensitive(bc):
    """Plausible mistakes in the boundary treatment break the polynomial pin: a flipped
    sign of g2, or a polynomial of too high a degree in the normal variable."""
    N = 6
    expr = POLY_FIRST if bc == 1 else POLY_SECOND
    arr = make_arrays(polynomial_problem(expr), N, bc)
    b = O.rhs(N, bc, arr.f, arr.g1, -arr.g2)
    x = O.dsolve(N, bc, b)
    assert np.abs(x - O.interior(arr.u)).max() > 1e-4
    high = (lambda sp, x, y, z: x**3 * y) if bc == 1 else (lambda sp, x, y, z: x**4 * y)
    arr = make_arrays(polynomial_problem(high), N, bc)
    x = O.dsolve(N, bc, O.rhs(N, bc, arr.f, arr.g1, arr.g2))
    assert np.abs(x - O.interior(arr.u)).max() > 1e-6


def test_rhs_reads_only_documented_entries():
    """f on interior nodes, g1 on boundary nodes, g2 on face-interior nodes: with NaN
    everywhere else the right-hand side stays finite."""
    N = 6
    arr = make_arrays(polynomial_problem(POLY_FIRST), N, 1, poison=True)
    f = arr.f.copy()
    f[0, :, :] = f[-1, :, :] = np.nan
    f[:, 0, :] = f[:, -1, :] = np.nan
    f[:, :, 0] = f[:, :, -1] = np.nan
    g2 = arr.g2.copy()
    for sl in [(slice(None), 0, 0), (slice(None), 0, -1), (slice(None), -1, 0),
               (slice(None), -1, -1), (0, slice(None), 0), (0, slice(None), -1),
               (-1, slice(None), 0), (-1, slice(None), -1), (0, 0, slice(None)),
               (0, -1, slice(None)), (-1, 0, slice(None)), (-1, -1, slice(None))]:
        g2[sl] = np.nan
    for bc in (1, 2):
        assert np.isfinite(O.rhs(N, bc, f, arr.g1, g2)).all()


def test_dot2_is_correctly_rounded():
    """Dot2 returns the exactly rounded dot product (checked with math.fsum on the exact
    error-free split of every product) on ill-conditioned sums."""
    import math
    rng = np.random.default_rng(7)
    bad = 0
    for trial in range(200):
        n = int(rng.integers(1, 3000))
        x = rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))
        y = rng.standard_normal(n)
        # force cancellation
        x = np.concatenate([x, -x[: n // 2]])
        y = np.concatenate([y, y[: n // 2] * (1 + 1e-12)])
        p = x * y
        e = np.array([math.fma(a, b, -c) for a, b, c in zip(x, y, p)]) if hasattr(math, "fma") \
            else _two_prod_err(x, y, p)
        exact = math.fsum(np.concatenate([p, e]))
        bad += O.dot(x, y) != exact
    assert bad <= 2


def _two_prod_err(a, b, p):
    """Exact error of a*b via Dekker's split (no FMA needed)."""
    def split(v):
        c = 134217729.0 * v
        hi = c - (c - v)
        return hi, v - hi
    ah, al = split(a)
    bh, bl = split(b)
    return ((ah * bh - p) + ah * bl + al * bh) + al * bl
