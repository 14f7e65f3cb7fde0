"""The GPU cascade reproduces the accuracy columns of the paper's Tables 1-4 (Sec. 6).

One cascade to the finest grid gives every row of a table: the level-l solution u_h of
Algorithm 1 (``get_level_solution``) against the exact solution, and EXP_finite of the two
coarser solutions against u_h.  Reading of the experiments as in the oracle's table test:
first-kind data, direct solves on 8^3 and 16^3, RMS over all nodes.

The solves are converged to (or, for the coarse levels of a tight cascade, down to the
FP64 floor of) the relative residual, so the 32^3 and 64^3 rows agree digit for digit.  On
finer grids the printed values come from the paper's own, unprinted, tolerance: with one to
eight iterations on the finest grids its iterate still carries part of the EXP_finite guess,
which sits closer to the continuous solution than u_h does.  Those rows are held to a
relative bound (0.5% at 128^3, 2% at 256^3 and 512^3); the convergence orders are checked as
well (2 for u_h, 3 for w_h - u_h)."""
import numpy as np
import pytest

import oracle as O
from manufactured import make_arrays, paper_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ex():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_05118_amd as ex
    ex.load()
    yield ex
    ex.finalize()


def _cascade_rows(ex, k, N, n_levels, tol):
    """(n, err2, errinf, w_err2) for every Bi-CG level of one cascade."""
    arr = make_arrays(paper_problem(k), N, 1)
    f, g1, g2 = (torch.from_numpy(a).cuda() for a in (arr.f, arr.g1, arr.g2))
    u = torch.empty_like(f)
    rc, st = ex.solve_ex(N, n_levels, 1, f, g1, g2, tol, u, max_iters=30000, max_runs=3)
    # coarse levels of a tight cascade stop at the FP64 floor (ENOCONV); none may break down
    assert rc in (ex.OK, ex.ENOCONV)
    lv = st.levels()
    assert all(l["status"] in (ex.OK, ex.ENOCONV) and l["rel_residual"] < 1e-6 for l in lv)
    del f, g1, g2
    us = []
    for l in range(n_levels):
        n = N >> (n_levels - 1 - l)
        t = torch.empty((n + 1,) * 3, dtype=torch.float64, device="cuda")
        ex.get_level_solution(l, t)
        us.append(t)
    np.testing.assert_array_equal(us[-1].cpu().numpy(), u.cpu().numpy())
    rows = []
    for l in range(2, n_levels):
        n = N >> (n_levels - 1 - l)
        s = N // n
        ul = us[l].cpu().numpy()
        w = torch.empty_like(us[l])
        ex.exp_finite(n, us[l - 1], us[l - 2], w)
        e = ul - arr.u[::s, ::s, ::s]
        rows.append((n, O.norm2(e), O.norminf(e), O.norm2(w.cpu().numpy() - ul)))
    torch.cuda.empty_cache()
    return rows


def _check(rows, table, meshes):
    for n, err2, errinf, werr in rows:
        i = meshes.index(n)
        got = (err2, errinf, werr)
        want = (table["err2"][i], table["errinf"][i], table["w_err2"][i])
        if n <= 64:
            assert tuple(float(f"{v:.2e}") for v in got) == want, (n, got, want)
        else:
            bound = 0.005 if n == 128 else 0.02
            for g, w in zip(got, want):
                assert abs(g / w - 1.0) <= bound, (n, got, want)
    for (n0, e0, _, w0), (n1, e1, _, w1) in zip(rows, rows[1:]):
        assert 1.9 < np.log2(e0 / e1) < 2.1
        assert 2.9 < np.log2(w0 / w1) < 3.2


def test_table1_to_128cube(ex, golden_tables):
    """Problem 1 (zero boundary data): its FP64 floor rises quickly with N (about 5e-10
    relative residual at 64^3, 2e-8 at 128^3), so the rows are taken from a 1e-9 cascade."""
    rows = _cascade_rows(ex, 1, 128, 5, 1e-9)
    _check(rows, golden_tables["problems"]["1"], golden_tables["meshes"])


@pytest.mark.slow
@pytest.mark.parametrize("k", [2, 3, 4])
def test_tables_2_to_4_to_512cube(ex, k, golden_tables):
    rows = _cascade_rows(ex, k, 512, 7, 1e-12)
    assert [r[0] for r in rows] == [32, 64, 128, 256, 512]
    _check(rows, golden_tables["problems"][str(k)], golden_tables["meshes"])
