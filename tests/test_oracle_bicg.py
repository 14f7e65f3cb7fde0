"""Pins of the oracle's Bi-CG (Algorithm 2, Sec. 5) and of the level loop of Algorithm 1.

References: numpy's dense solver on the independently assembled Kronecker matrix, and the
textbook property that Bi-CG in exact arithmetic terminates within n steps."""
import numpy as np
import pytest
import scipy.sparse as sps

import oracle as O
from test_oracle_operator import _closed_form


@pytest.mark.parametrize("N", [4, 8])
@pytest.mark.parametrize("bc", [1, 2])
@pytest.mark.parametrize("literal", [False, True])
def test_bicg_reaches_direct_solution(N, bc, literal):
    rng = np.random.default_rng(N * 10 + bc)
    n = (N - 1) ** 3
    b = rng.standard_normal(n)
    ref = np.linalg.solve(_closed_form(N, bc), b)
    x, it, rr, rc = O.bicg(N, bc, b, np.zeros(n), 1e-14, literal_transpose=literal)
    assert rc == O.OK
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    assert rr <= (1e-14 ** 2) * O.dot(b, b)


@pytest.mark.parametrize("bc", [1, 2])
def test_bicg_with_random_shadow(bc):
    """A shadow residual different from r_0 exercises the dual recurrence; the iteration
    still converges to the solution of A x = b."""
    N = 6
    n = (N - 1) ** 3
    rng = np.random.default_rng(3)
    b = rng.standard_normal(n)
    shadow = rng.standard_normal(n)
    ref = np.linalg.solve(_closed_form(N, bc), b)
    x, it, rr, rc = O.bicg(N, bc, b, np.zeros(n), 1e-12, shadow=shadow, literal_transpose=True)
    assert rc == O.OK
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-7 * np.abs(ref).max())


def test_bicg_terminates_within_n_steps_on_tiny_system():
    """n = 1 (N = 2): one step solves the system exactly."""
    b = np.array([3.0])
    for bc in (1, 2):
        x, it, rr, rc = O.bicg(2, bc, b, np.zeros(1), 1e-15)
        assert it == 1 and rc == O.OK
        np.testing.assert_allclose(x, b / _closed_form(2, bc)[0, 0], rtol=1e-15)


def test_bicg_literal_and_symmetric_transpose_agree():
    """Forming p*A by scattering the rows of A_h or as A_h p* gives the same converged
    solution up to the tolerance-limited difference."""
    N = 12
    rng = np.random.default_rng(5)
    n = (N - 1) ** 3
    b = rng.standard_normal(n)
    x1, *_ = O.bicg(N, 1, b, np.zeros(n), 1e-13, literal_transpose=True)
    x2, *_ = O.bicg(N, 1, b, np.zeros(n), 1e-13, literal_transpose=False)
    assert np.linalg.norm(x1 - x2) <= 1e-8 * np.linalg.norm(x1)


def test_bicg_maxit_reports_no_convergence():
    N = 10
    n = (N - 1) ** 3
    b = np.random.default_rng(1).standard_normal(n)
    x, it, rr, rc = O.bicg(N, 2, b, np.zeros(n), 1e-14, maxit=3)
    assert rc == O.ENOCONV and it == 3


def test_bicg_zero_rhs_needs_no_iteration():
    N = 6
    n = (N - 1) ** 3
    x, it, rr, rc = O.bicg(N, 1, np.zeros(n), np.zeros(n), 1e-10)
    assert it == 0 and rc == O.OK and rr == 0.0


def test_level_solve_restarts_until_true_residual():
    """The while loop of Algorithm 1 keeps calling Bi-CG while the true residual is above
    the tolerance; with a small iteration cap per call it needs several calls."""
    N = 10
    n = (N - 1) ** 3
    b = np.random.default_rng(2).standard_normal(n)
    x, st = O.level_solve(N, 1, b, np.zeros(n), 1e-10, maxit=40, max_runs=50)
    assert st.code == O.OK and st.runs > 1
    r = O.residual(N, 1, b, x)
    assert O.dot(r, r) <= 1e-20 * O.dot(b, b)
    assert st.rr_true == O.dot(r, r)


def test_level_solve_skips_converged_start():
    N = 6
    n = (N - 1) ** 3
    b = np.random.default_rng(4).standard_normal(n)
    xs = O.dsolve(N, 2, b)
    x, st = O.level_solve(N, 2, b, xs, 1e-8)
    assert st.iters == 0 and st.runs == 0
    np.testing.assert_array_equal(x, xs)


def test_level_tolerance_schedule():
    """eps_i = eps * 10^(i-L) (Algorithm 1): the coarser the level, the tighter."""
    L = 6
    for i in range(1, L + 1):
        assert np.isclose(O.level_tolerance(1e-8, i, L), 1e-8 * 10.0 ** (i - L), rtol=1e-15)
    assert O.level_tolerance(1e-8, L, L) == 1e-8


def test_work_units_match_paper_footnotes(golden_tables):
    """WU = sum over levels of iterations x 8^-(levels below the finest); Tables 1-5
    footnotes."""
    for k, t in golden_tables["problems"].items():
        assert round(O.work_units(t["iters"]), 2) == pytest.approx(t["wu"], abs=0.006), k
