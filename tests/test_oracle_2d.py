"""Pins of the 2D oracle (eq. bvp2d through the same pipeline): the 13-point scheme against
the square of the 5-point Laplacian and against polynomials it must reproduce, the
reflections through discrete solutions that are exact, DSOLVE and Bi-CG against dense
solves, EXP_finite and EXP_true through the polynomials they reproduce, and the whole
cascade through its convergence orders."""
import numpy as np
import pytest
import scipy.sparse as sps

import oracle as O
from manufactured.twod import Family2D, family_2d, make_arrays_2d, sine_2d


def _lap_2d(N):
    n = N - 1
    T = sps.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    I = sps.identity(n)
    return (sps.kron(I, T) + sps.kron(T, I)).tocsr()


def _closed_form_2d(N, bc):
    """(L_D)^2 + 2 diag(m) (first kind) or (L_D)^2 (second kind); m counts the edges a node
    is next to."""
    L = _lap_2d(N)
    A = (L @ L).toarray()
    if bc == 1:
        e = np.zeros(N - 1)
        e[0] += 1
        e[-1] += 1
        A = A + 2 * np.diag((e[None, :] + e[:, None]).ravel())
    return A


@pytest.mark.parametrize("N", [2, 3, 4, 6, 9])
@pytest.mark.parametrize("bc", [1, 2])
def test_operator_closed_form(N, bc):
    A = O.assemble_2d(N, bc)
    np.testing.assert_array_equal(A, _closed_form_2d(N, bc))
    np.testing.assert_array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0


def _poly_grid(coef, N):
    x = np.arange(N + 1) / N
    X, Y = np.meshgrid(x, x)
    return sum(c * X**a * Y**b for (a, b), c in coef.items())


def _bih_poly(coef, N):
    """Delta^2 of sum c x^a y^b, exactly."""
    x = np.arange(N + 1) / N
    X, Y = np.meshgrid(x, x)

    def d(a, k):  # k-th derivative coefficient of x^a
        out = 1.0
        for t in range(k):
            out *= (a - t)
        return out
    f = np.zeros_like(X)
    for (a, b), c in coef.items():
        for ka, kb, w in ((4, 0, 1.0), (0, 4, 1.0), (2, 2, 2.0)):
            if a >= ka and b >= kb:
                f += w * c * d(a, ka) * d(b, kb) * X ** (a - ka) * Y ** (b - kb)
    return f


def test_interior_scheme_is_exact_to_degree_five():
    """Rows of b - A u away from the edges (no fictitious point involved) vanish for every
    polynomial of total degree <= 5 and not for x^6."""
    N = 16
    rng = np.random.default_rng(4)
    coef = {(a, b): rng.standard_normal() for a in range(6) for b in range(6) if a + b <= 5}
    for c, exact in ((coef, True), ({(6, 0): 1.0}, False)):
        u = _poly_grid(c, N)
        f = _bih_poly(c, N)
        zero = np.zeros_like(u)
        b = O.rhs_2d(N, 1, f, np.where(_boundary(N), u, 0.0), zero)
        r = (b - O.apply_2d(N, 1, O.interior_2d(u))).reshape(N - 1, N - 1)
        deep = np.abs(r[2:-2, 2:-2]).max()
        scale = (1.0 / N) ** 4 * np.abs(f).max() + 1e-300
        if exact:
            assert deep <= 1e-9 * max(scale, np.abs(u).max() * 1e-6)
        else:
            assert deep > 1e-6 * (1.0 / N) ** 4


def _boundary(N):
    m = np.zeros((N + 1, N + 1), dtype=bool)
    m[0, :] = m[-1, :] = m[:, 0] = m[:, -1] = True
    return m


@pytest.mark.parametrize("bc,coef", [
    (1, {(2, 2): 1.0, (1, 1): 3.0, (0, 2): 1.0, (1, 0): 1.0}),   # quadratic in each normal
    (2, {(3, 2): 1.0, (0, 3): 1.0, (2, 1): 1.0}),               # cubic in each normal
])
def test_discrete_solution_is_exact_when_the_reflection_is(bc, coef):
    """The reflections are exact for u quadratic (first kind) or cubic (second kind) along
    each edge normal, and the scheme for total degree <= 5: the discrete solution is u."""
    N = 8
    u = _poly_grid(coef, N)
    f = _bih_poly(coef, N)
    x = np.arange(N + 1) / N
    X, Y = np.meshgrid(x, x)
    # boundary data from the exact polynomial
    ux = sum(c * a * X ** max(a - 1, 0) * Y**b for (a, b), c in coef.items() if a >= 1)
    uy = sum(c * b * X**a * Y ** max(b - 1, 0) for (a, b), c in coef.items() if b >= 1)
    uxx = sum(c * a * (a - 1) * X ** max(a - 2, 0) * Y**b for (a, b), c in coef.items() if a >= 2)
    uyy = sum(c * b * (b - 1) * X**a * Y ** max(b - 2, 0) for (a, b), c in coef.items() if b >= 2)
    ux, uy, uxx, uyy = (np.broadcast_to(v, u.shape) if np.ndim(v) else np.full(u.shape, v)
                        for v in (ux, uy, uxx, uyy))
    g1 = np.where(_boundary(N), u, 0.0)
    g2 = np.zeros_like(u)
    for sl, dn, dnn in ((np.s_[:, 0], -ux, uxx), (np.s_[:, N], ux, uxx),
                        (np.s_[0, :], -uy, uyy), (np.s_[N, :], uy, uyy)):
        g2[sl] = (dn if bc == 1 else dnn)[sl]
    b = O.rhs_2d(N, bc, f, g1, g2)
    x_ = O.dsolve_2d(N, bc, b)
    np.testing.assert_allclose(x_, O.interior_2d(u), rtol=0, atol=1e-11 * np.abs(u).max())


@pytest.mark.parametrize("bc", [1, 2])
def test_dsolve_and_bicg_reach_the_dense_solution(bc):
    N = 10
    rng = np.random.default_rng(bc)
    b = rng.standard_normal((N - 1) ** 2)
    ref = np.linalg.solve(_closed_form_2d(N, bc), b)
    np.testing.assert_allclose(O.dsolve_2d(N, bc, b), ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    x, it, rr, rc = O.bicg_2d(N, bc, b, np.zeros_like(b), 1e-13)
    assert rc == O.OK
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_exp_finite_reproduces_biquadratics_and_formulas():
    N = 16
    rng = np.random.default_rng(9)
    coef = {(a, b): rng.standard_normal() for a in range(3) for b in range(3)}
    p2, p1, p0 = _poly_grid(coef, N), _poly_grid(coef, N // 2), _poly_grid(coef, N // 4)
    np.testing.assert_allclose(O.exp_finite_2d(N, p1, p0), p2, rtol=0, atol=1e-13)
    # coarse nodes take eq. (secfff) of the two coarse solutions
    u1 = rng.standard_normal((N // 2 + 1,) * 2)
    u0 = rng.standard_normal((N // 4 + 1,) * 2)
    w = O.exp_finite_2d(N, u1, u0)
    np.testing.assert_allclose(w[::4, ::4], (5 * u1[::2, ::2] - u0) / 4, rtol=0, atol=1e-14)
    assert not np.allclose(O.exp_finite_2d(N, p1, p0 + 1e-3), p2)


def test_exp_true_identity_and_coarse_formula():
    N = 12
    rng = np.random.default_rng(1)
    uh = rng.standard_normal((N + 1,) * 2)
    same = uh[::2, ::2].copy()
    np.testing.assert_allclose(O.exp_true_2d(N, uh, same), uh, rtol=0, atol=1e-14)
    u2h = rng.standard_normal((N // 2 + 1,) * 2)
    ut = O.exp_true_2d(N, uh, u2h)
    np.testing.assert_allclose(ut[::2, ::2], (4 * uh[::2, ::2] - u2h) / 3, rtol=0, atol=1e-14)


@pytest.mark.parametrize("bc", [1, 2])
def test_cascade_orders(bc):
    """u_h converges with order 2, w_h - u_h with order 3 and EXP_true with order 4."""
    prob = family_2d(7)
    errs, werrs, terrs = [], [], []
    for N, nl in ((32, 4), (64, 5), (128, 6)):
        arr = make_arrays_2d(prob, N, bc)
        res = O.excmg_2d(N, nl, bc, arr.f, arr.g1, arr.g2, 1e-11, keep_levels=True)
        assert res.levels[-1].code == O.OK
        errs.append(O.norm2(res.u - arr.u))
        werrs.append(O.norm2(res.w_levels[-1] - res.u))
        terrs.append(O.norm2(res.ut - arr.u))
    for e in (errs, werrs, terrs):
        print(e)
    for a, b in zip(errs, errs[1:]):
        assert 1.9 < np.log2(a / b) < 2.1
    assert 2.7 < np.log2(werrs[1] / werrs[2]) < 3.3
    for a, b in zip(terrs, terrs[1:]):
        assert 3.5 < np.log2(a / b) < 4.5


def _separable_exp_finite_2d(N, u1, u0):
    """Independent tensor-product form: w = Q(u1 + 1/4 T(u1|Z0 - u0)), T bilinear Z0 -> Z1,
    Q piecewise quadratic Z1 -> Z2 on each Z0 cell, applied axis by axis."""
    def lin_up(a, axis):
        a = np.moveaxis(a, axis, 0)
        out = np.empty((2 * a.shape[0] - 1,) + a.shape[1:])
        out[::2] = a
        out[1::2] = 0.5 * (a[:-1] + a[1:])
        return np.moveaxis(out, 0, axis)

    def quad_up(a, axis):
        a = np.moveaxis(a, axis, 0)
        m = a.shape[0]
        out = np.empty((2 * m - 1,) + a.shape[1:])
        out[::2] = a
        for c in range((m - 1) // 2):      # quadratic through Z1 nodes 2c, 2c+1, 2c+2
            y0, y1, y2 = a[2 * c], a[2 * c + 1], a[2 * c + 2]
            out[4 * c + 1] = (3 * y0 + 6 * y1 - y2) / 8
            out[4 * c + 3] = (-y0 + 6 * y1 + 3 * y2) / 8
        return np.moveaxis(out, 0, axis)

    t = u1[::2, ::2] - u0
    for ax in range(2):
        t = lin_up(t, ax)
    v = u1 + 0.25 * t
    for ax in range(2):
        v = quad_up(v, ax)
    return v


@pytest.mark.parametrize("N", [4, 8, 16])
def test_exp_finite_equals_separable_form(N):
    rng = np.random.default_rng(N + 5)
    u1 = rng.standard_normal((N // 2 + 1,) * 2)
    u0 = rng.standard_normal((N // 4 + 1,) * 2)
    np.testing.assert_allclose(O.exp_finite_2d(N, u1, u0), _separable_exp_finite_2d(N, u1, u0),
                               rtol=0, atol=1e-13)


def test_exp_true_bilinear_correction():
    """ut = uh + (1/3) bilinear interpolation of (uh - u2h) over the coarse grid."""
    N = 8
    rng = np.random.default_rng(3)
    uh = rng.standard_normal((N + 1,) * 2)
    x = np.arange(N + 1) / N
    X, Y = np.meshgrid(x, x)
    lin = 1 + 2 * X - Y + 3 * X * Y
    ut = O.exp_true_2d(N, uh, uh[::2, ::2] - lin[::2, ::2])
    np.testing.assert_allclose(ut, uh + lin / 3, rtol=0, atol=1e-14)
