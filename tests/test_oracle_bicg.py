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


def test_level_solve_stops_at_the_fp64_floor():
    """The while loop of Algorithm 1 cannot push the true residual below the FP64 floor:
    with zero boundary data (paper Problem 1) the floor at 16^3 is ~7e-13 relative.  A
    tolerance of 1e-15 (below 10x the estimate 22 u ||x|| / ||b||) ends the level as soon
    as a run no longer halves r.r, long before max_runs; the estimate is within two orders
    of the floor actually reached; a tolerance above the floor converges."""
    from manufactured import make_arrays, paper_problem
    N = 16
    arr = make_arrays(paper_problem(1), N, 1)
    b = O.rhs(N, 1, arr.f, arr.g1, arr.g2)
    x, st = O.level_solve(N, 1, b, np.zeros((N - 1) ** 3), 1e-15, max_runs=20)
    assert st.code == O.ENOCONV and st.runs < 5
    reached = np.sqrt(st.rr_true / st.bb)
    est = 22 * 2.0 ** -53 * np.sqrt(O.dot(x, x) / O.dot(b, b))
    assert 1e-15 < 10 * est and est < reached < 100 * est
    x, st = O.level_solve(N, 1, b, np.zeros((N - 1) ** 3), 1e-11, max_runs=20)
    assert st.code == O.OK and np.sqrt(st.rr_true / st.bb) <= 1e-11


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


# ------------------------------------------------------------------ Algorithm 2 variants

@pytest.mark.parametrize("N", [2, 3, 5, 8])
@pytest.mark.parametrize("bc", [1, 2])
def test_diagonal_matches_the_assembled_operator(N, bc):
    """diag(A_h) read off the operator equals that of the Kronecker construction."""
    np.testing.assert_array_equal(O.diagonal(N, bc), np.diag(_closed_form(N, bc)))


@pytest.mark.parametrize("bc", [1, 2])
@pytest.mark.parametrize("literal", [False, True])
def test_jacobi_preconditioned_bicg_reaches_direct_solution(bc, literal):
    N = 8
    n = (N - 1) ** 3
    rng = np.random.default_rng(11 + bc)
    b = rng.standard_normal(n)
    A = _closed_form(N, bc)
    x, xs, it, rr, rc = O.bicg_ex(N, bc, b, np.zeros(n), 1e-13, mdiag=O.diagonal(N, bc),
                                  literal_transpose=literal)
    assert rc == O.OK and xs is None
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-9 * np.abs(x).max())


def test_scalar_preconditioner_gives_the_unpreconditioned_iterates():
    """M = c I changes p by 1/c and alpha by c: the iterates x_k are those of M = I."""
    N, bc = 8, 1
    n = (N - 1) ** 3
    rng = np.random.default_rng(2)
    b = rng.standard_normal(n)
    for k in (1, 3, 7):
        x1, _, _, _, _ = O.bicg_ex(N, bc, b, np.zeros(n), 1e-30, maxit=k)
        x2, _, _, _, _ = O.bicg_ex(N, bc, b, np.zeros(n), 1e-30, maxit=k,
                                   mdiag=np.full(n, 4.0))
        np.testing.assert_allclose(x2, x1, rtol=1e-12, atol=1e-14 * np.abs(x1).max())


@pytest.mark.parametrize("bc", [1, 2])
def test_dual_iterate_solves_the_transposed_system(bc):
    """With b* and x*_0 the shadow recurrence is the Bi-CG iteration of A^T x* = b*."""
    N = 6
    n = (N - 1) ** 3
    rng = np.random.default_rng(21 + bc)
    b, bstar, xs0 = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
    A = _closed_form(N, bc)
    x, xs, it, rr, rc = O.bicg_ex(N, bc, b, np.zeros(n), 1e-13, bstar=bstar, xstar0=xs0,
                                  literal_transpose=True)
    assert rc == O.OK
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-8 * np.abs(x).max())
    ref = np.linalg.solve(A.T, bstar)
    np.testing.assert_allclose(xs, ref, rtol=0, atol=1e-6 * np.abs(ref).max())


def test_residuals_are_biorthogonal():
    """r_i . r*_j = 0 for i != j (the defining property of the two Bi-CG sequences), with
    r_k = b - A x_k and r*_k = b* - A^T x*_k from runs stopped after k steps."""
    N, bc = 6, 2
    n = (N - 1) ** 3
    rng = np.random.default_rng(7)
    b, bstar = rng.standard_normal(n), rng.standard_normal(n)
    A = _closed_form(N, bc)
    rs, rss = [], []
    for k in range(5):
        x, xs, *_ = O.bicg_ex(N, bc, b, np.zeros(n), 1e-30, maxit=k, bstar=bstar,
                              xstar0=np.zeros(n), literal_transpose=True)
        rs.append(b - A @ x)
        rss.append(bstar - A.T @ xs)
    for i in range(5):
        for j in range(5):
            c = abs(rs[i] @ rss[j]) / (np.linalg.norm(rs[i]) * np.linalg.norm(rss[j]))
            if i != j:
                assert c < 1e-9, (i, j, c)
            else:
                assert c > 1e-3


def test_preconditioned_residuals_are_biorthogonal_in_the_inverse_metric():
    """With a diagonal M the two residual sequences are biorthogonal in the M^-1 inner
    product: r_i . M^-1 r*_j = 0 for i != j.  A strongly varying M separates this from the
    M inner product, which would vanish instead if M were applied where M^-1 belongs."""
    N, bc = 6, 2
    n = (N - 1) ** 3
    rng = np.random.default_rng(17)
    b, bstar = rng.standard_normal(n), rng.standard_normal(n)
    m = rng.uniform(1.0, 10.0, n)
    A = _closed_form(N, bc)
    rs, rss = [], []
    for k in range(5):
        x, xs, *_ = O.bicg_ex(N, bc, b, np.zeros(n), 1e-30, maxit=k, bstar=bstar,
                              xstar0=np.zeros(n), mdiag=m, literal_transpose=True)
        rs.append(b - A @ x)
        rss.append(bstar - A.T @ xs)

    def cos(u, v, w):
        return abs(u @ (w * v)) / np.sqrt((u @ (w * u)) * (v @ (w * v)))

    worst_wrong = 0.0
    for i in range(5):
        for j in range(5):
            if i != j:
                assert cos(rs[i], rss[j], 1.0 / m) < 1e-9, (i, j)
                worst_wrong = max(worst_wrong, cos(rs[i], rss[j], m))
    assert worst_wrong > 1e-3
