"""The input generator: hand-written closed forms agree with SymPy's derivatives.

The paper's forcing terms (Sec. 6, eqs. force1-force4) are checked against Delta^2 u
computed symbolically; Problem 3's printed f = u is the one that fails (Delta^2 u = 9u)."""
import numpy as np
import pytest
import sympy as sp

from manufactured import make_arrays, paper_problem, config_problem, SympyProblem
from manufactured.problems import SeparableFamily


def _sym_u(k):
    x, y, z = sp.symbols("x y z", real=True)
    return {
        1: (1 - sp.cos(2 * sp.pi * x)) * (1 - sp.cos(2 * sp.pi * y)) * (1 - sp.cos(2 * sp.pi * z)),
        2: sp.exp(x * y * z),
        3: sp.sinh(x) * sp.sinh(y) * sp.sinh(z),
        4: x * y * z * sp.log(1 + x + y + z),
    }[k], (x, y, z)


def _bih(u, v):
    x, y, z = v
    lap = lambda e: sp.diff(e, x, 2) + sp.diff(e, y, 2) + sp.diff(e, z, 2)  # noqa: E731
    return lap(lap(u))


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_paper_forcing_matches_bilaplacian(k):
    u, v = _sym_u(k)
    f = sp.lambdify(v, _bih(u, v), "numpy")
    P = paper_problem(k)
    rng = np.random.default_rng(k)
    pts = rng.uniform(0, 1, size=(20, 3))
    for (x, y, z) in pts:
        ref = float(f(x, y, z))
        got = float(np.asarray(P._f(np.float64(x), np.float64(y), np.float64(z))))
        assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref))


def test_problem3_printed_forcing_is_a_typo():
    u, v = _sym_u(3)
    assert sp.simplify(_bih(u, v) - 9 * u) == 0
    assert sp.simplify(_bih(u, v) - u) != 0


@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", [1, 2])
def test_boundary_data_matches_symbolic(k, bc):
    u, (x, y, z) = _sym_u(k)
    N = 6
    arr = make_arrays(paper_problem(k), N, bc)
    ux = sp.lambdify((x, y, z), u, "numpy")
    d1 = [sp.lambdify((x, y, z), sp.diff(u, s), "numpy") for s in (x, y, z)]
    d2 = [sp.lambdify((x, y, z), sp.diff(u, s, 2), "numpy") for s in (x, y, z)]
    h = 1.0 / N
    for kk in range(N + 1):
        for jj in range(N + 1):
            for ii in range(N + 1):
                X, Y, Z = ii * h, jj * h, kk * h
                on = [ii in (0, N), jj in (0, N), kk in (0, N)]
                if not any(on):
                    continue
                assert np.isclose(arr.g1[kk, jj, ii], float(ux(X, Y, Z)), rtol=1e-12, atol=1e-13)
                if sum(on) != 1:
                    continue  # g2 is read on face-interior nodes only
                a = on.index(True)
                idx = (ii, jj, kk)[a]
                if bc == 1:
                    ref = float(d1[a](X, Y, Z)) * (-1.0 if idx == 0 else 1.0)
                else:
                    ref = float(d2[a](X, Y, Z))
                assert np.isclose(arr.g2[kk, jj, ii], ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("c", [1, 2, 3, 4])
def test_config_family_closed_form(c):
    P = config_problem(c)
    assert isinstance(P, SeparableFamily)
    x, y, z = sp.symbols("x y z", real=True)
    u = 0
    if P.exp_coef is not None:
        a, b, cc = P.exp_coef
        u += sp.exp(a * x + b * y + cc * z)
    for (A, k1, k2, k3) in P.modes:
        u += A * sp.sin(k1 * sp.pi * x) * sp.sin(k2 * sp.pi * y) * sp.sin(k3 * sp.pi * z)
    N = 8
    for bc in (1, 2):
        arr = make_arrays(P, N, bc)
        S = SympyProblem("check", lambda _sp, X, Y, Z: u.subs({x: X, y: Y, z: Z}),
                         simplify=False)
        ref = make_arrays(S, N, bc)
        np.testing.assert_allclose(arr.f, ref.f, rtol=1e-10, atol=1e-8)
        np.testing.assert_allclose(arr.u, ref.u, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(arr.g1, ref.g1, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(arr.g2, ref.g2, rtol=1e-10, atol=1e-10)


def test_config1_forcing_is_nine_pi4_u():
    P = config_problem(1)
    x = np.arange(9) / 8.0
    np.testing.assert_allclose(P.f_grid(x), 9 * np.pi ** 4 * P.u_grid(x), rtol=1e-13, atol=1e-10)


def test_config_seeds_are_fixed():
    a = config_problem(2)
    b = config_problem(2)
    assert a.exp_coef == b.exp_coef and a.modes == b.modes
    assert len(config_problem(4).modes) == 8
    assert max(max(k1, k2, k3) for (_, k1, k2, k3) in config_problem(4).modes) <= 8
