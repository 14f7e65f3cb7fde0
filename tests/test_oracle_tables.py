"""The oracle reproduces the paper's printed accuracy (Sec. 6, Tables 1-5).

Reading of the experiments (the paper leaves these implicit): first-kind boundary data,
direct solves on the 8^3 and 16^3 grids, the tables' ||.||_2 is the root mean square over
all (N+1)^3 nodes and ||w_h - u_h||_2 keeps the raw interpolant on boundary nodes.  The
finite-difference solutions are converged far below their discretisation error (relative
residual 1e-12, or 1e-11 where FP64 cannot go lower), so the printed error columns can be compared digit for digit; the
iteration columns depend on the unprinted tolerance and are not compared."""
import numpy as np
import pytest

import oracle as O
from manufactured import make_arrays, paper_problem


def _sig3(v):
    return float(f"{v:.2e}")


def _run(k, N, n_levels, tol):
    arr = make_arrays(paper_problem(k), N, 1)
    res = O.excmg(N, n_levels, 1, arr.f, arr.g1, arr.g2, tol, keep_levels=True)
    return arr, res


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_tables_32cube_rows(k, golden_tables):
    t = golden_tables["problems"][str(k)]
    # Problem 1 has zero boundary data, so f_h is only the h^4 f term and the FP64
    # relative-residual floor sits near 4e-12 on this grid
    arr, res = _run(k, 32, 3, 1e-11 if k == 1 else 1e-12)
    assert res.levels[-1].code == O.OK
    e = res.u - arr.u
    werr = res.w_levels[-1] - res.u
    assert _sig3(O.norm2(e)) == t["err2"][0]
    assert _sig3(O.norminf(e)) == t["errinf"][0]
    assert _sig3(O.norm2(werr)) == t["w_err2"][0]


@pytest.mark.slow
def test_table3_64cube_row_and_orders(golden_tables):
    """Problem 3 on 64^3 cells: the printed errors, and the observed orders of u_h (2),
    of w_h - u_h (3) and of the extrapolated EXP_true solution (4)."""
    t = golden_tables["problems"]["3"]
    arr, res = _run(3, 64, 4, 1e-12)
    assert all(st.code == O.OK for st in res.levels)
    u32, u64 = res.u_levels[2], res.u_levels[3]
    e64 = res.u - arr.u
    assert _sig3(O.norm2(e64)) == t["err2"][1]
    assert _sig3(O.norminf(e64)) == t["errinf"][1]
    assert _sig3(O.norm2(res.w_levels[3] - u64)) == t["w_err2"][1]
    x32 = np.arange(33) / 32.0
    uex32 = paper_problem(3).u_grid(x32)
    order_u = np.log2(O.norm2(u32 - uex32) / O.norm2(e64))
    order_w = np.log2(O.norm2(res.w_levels[2] - u32) / O.norm2(res.w_levels[3] - u64))
    assert 1.9 < order_u < 2.1
    assert 2.8 < order_w < 3.3
    ut32 = O.exp_true(32, u32, res.u_levels[1])
    order_t = np.log2(O.norm2(ut32 - uex32) / O.norm2(res.ut - arr.u))
    assert 3.5 < order_t < 4.6
    # the extrapolated solution is far more accurate than u_h
    assert O.norm2(res.ut - arr.u) < 0.05 * O.norm2(e64)


def test_jacobi_cascade_reaches_the_same_finite_difference_solution(golden_tables):
    """Preconditioning changes the path, not the limit: the Jacobi-preconditioned cascade
    reproduces Table 2's 32^3 row as the plain one does."""
    arr = make_arrays(paper_problem(2), 32, 1)
    res = O.excmg(32, 3, 1, arr.f, arr.g1, arr.g2, 1e-12, jacobi=True)
    assert res.levels[-1].code == O.OK
    t = golden_tables["problems"]["2"]
    assert _sig3(O.norm2(res.u - arr.u)) == t["err2"][0]
    assert _sig3(O.norminf(res.u - arr.u)) == t["errinf"][0]
