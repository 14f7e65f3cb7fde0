"""Parity of the HIP library with the CPU oracle, element by element, through the C ABI.

The library and the oracle evaluate every formula in the same arithmetic order (no FMA
contraction, the paper's term order, compensated dot products), so most outputs are
compared for exact equality; solver outputs are held to the 1e-10 relative L2 bar and are
expected to agree far more closely."""
import numpy as np
import pytest

import oracle as O
from manufactured import config_problem, make_arrays, paper_problem

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    a, b = np.ravel(a), np.ravel(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


# ------------------------------------------------------------------ operator

@pytest.mark.parametrize("N", [2, 3, 4, 5, 8, 16, 33, 64, 127, 128])
@pytest.mark.parametrize("bc", [1, 2])
def test_apply_operator_bit_exact(ex, N, bc):
    print(f"apply N={N} bc={bc}", flush=True)
    rng = np.random.default_rng(1000 * N + bc)
    x = rng.standard_normal((N - 1) ** 3)
    y = torch.empty((N - 1) ** 3, dtype=torch.float64, device="cuda")
    ex.apply_operator(N, bc, 0, dev(x), y)
    np.testing.assert_array_equal(host(y), O.apply(N, bc, x))


@pytest.mark.parametrize("N", [3, 16, 65])
@pytest.mark.parametrize("bc", [1, 2])
def test_apply_transpose_matches_literal_transpose(ex, N, bc):
    rng = np.random.default_rng(N + 7 * bc)
    x = rng.standard_normal((N - 1) ** 3)
    y = torch.empty((N - 1) ** 3, dtype=torch.float64, device="cuda")
    ex.apply_operator(N, bc, 1, dev(x), y)
    ref = O.apply_transpose(N, bc, x)
    np.testing.assert_allclose(host(y), ref, rtol=0, atol=1e-13 * np.abs(x).max())


@pytest.mark.parametrize("bc", [1, 2])
def test_apply_stencil_on_context_levels(ex, bc):
    ex.setup(96, 5, bc)   # levels of 6, 12, 24, 48, 96 cells
    for level, N in enumerate([6, 12, 24, 48, 96]):
        x = np.random.default_rng(level).standard_normal((N - 1) ** 3)
        y = torch.empty_like(dev(x))
        ex.apply_stencil(level, level % 2, dev(x), y)
        np.testing.assert_array_equal(host(y), O.apply(N, bc, x))


def test_host_arrays_are_staged(ex):
    N, bc = 20, 2
    x = np.random.default_rng(3).standard_normal((N - 1) ** 3)
    y = np.empty_like(x)
    ex.apply_operator(N, bc, 0, x, y)
    np.testing.assert_array_equal(y, O.apply(N, bc, x))


# ------------------------------------------------------------------ right-hand side

@pytest.mark.parametrize("bc", [1, 2])
def test_rhs_bit_exact_every_level(ex, bc):
    Nf, nl = 64, 5
    arr = make_arrays(config_problem(2), Nf, bc, poison=True)
    ex.setup(Nf, nl, bc)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    for level in range(nl):
        N = (Nf >> (nl - 1)) << level
        s = Nf // N
        b = torch.empty((N - 1) ** 3, dtype=torch.float64, device="cuda")
        ex.rhs(level, f, g1, g2, b)
        ref = O.rhs(N, bc, O.inject(arr.f, s), O.inject(arr.g1, s), O.inject(arr.g2, s))
        np.testing.assert_array_equal(host(b), ref)


# ------------------------------------------------------------------ transfers

@pytest.mark.parametrize("N", [4, 8, 16, 44, 128])
def test_exp_finite_bit_exact(ex, N):
    rng = np.random.default_rng(N)
    u1 = rng.standard_normal((N // 2 + 1,) * 3)
    u0 = rng.standard_normal((N // 4 + 1,) * 3)
    w = torch.empty((N + 1) ** 3, dtype=torch.float64, device="cuda")
    ex.exp_finite(N, dev(u1), dev(u0), w)
    np.testing.assert_array_equal(host(w).reshape((N + 1,) * 3), O.exp_finite(N, u1, u0))


@pytest.mark.parametrize("N", [2, 6, 32, 128])
def test_exp_true_bit_exact(ex, N):
    rng = np.random.default_rng(N + 1)
    uh = rng.standard_normal((N + 1,) * 3)
    u2h = rng.standard_normal((N // 2 + 1,) * 3)
    ut = torch.empty((N + 1) ** 3, dtype=torch.float64, device="cuda")
    ex.exp_true(N, dev(uh), dev(u2h), ut)
    np.testing.assert_array_equal(host(ut).reshape((N + 1,) * 3), O.exp_true(N, uh, u2h))


# ------------------------------------------------------------------ DSOLVE and Bi-CG

@pytest.mark.parametrize("N0", [2, 3, 4, 8])
@pytest.mark.parametrize("bc", [1, 2])
def test_dsolve_matches_oracle(ex, N0, bc):
    ex.setup(N0 * 4, 3, bc)
    for level in (0, 1):
        N = N0 << level
        b = np.random.default_rng(N).standard_normal((N - 1) ** 3)
        x = torch.empty_like(dev(b))
        ex.dsolve(level, dev(b), x)
        ref = O.dsolve(N, bc, b)
        # the banded factor skips only exact zeros of the dense elimination: same bits
        np.testing.assert_array_equal(host(x), ref)


@pytest.mark.parametrize("bc", [1, 2])
def test_bicg_run_matches_oracle(ex, bc):
    Nf, nl = 32, 4
    ex.setup(Nf, nl, bc)
    N = 32
    arr = make_arrays(config_problem(2), N, bc)
    b = O.rhs(N, bc, arr.f, arr.g1, arr.g2)
    x0 = O.interior(arr.u) * (1 + 1e-3 * np.sin(np.arange((N - 1) ** 3)))
    xg = dev(x0)
    rc, it, rr = ex.bicg(3, dev(b), xg, 1e-9, 5000)
    xr, itr, rrr, rcr = O.bicg(N, bc, b, x0, 1e-9, maxit=5000)
    assert rc == ex.OK and rcr == O.OK
    assert it == itr
    assert rr == rrr
    np.testing.assert_array_equal(host(xg), xr)


def test_bicg_iteration_cap(ex):
    ex.setup(32, 4, 1)
    N = 32
    b = np.random.default_rng(2).standard_normal((N - 1) ** 3)
    x = torch.zeros_like(dev(b))
    rc, it, rr = ex.bicg(3, dev(b), x, 1e-14, 7)
    assert rc == ex.ENOCONV and it == 7
    xr, itr, rrr, rcr = O.bicg(N, 1, b, np.zeros_like(b), 1e-14, maxit=7)
    np.testing.assert_array_equal(host(x), xr)


@pytest.mark.parametrize("bc", [1, 2])
def test_level_solve_matches_oracle(ex, bc):
    ex.setup(64, 5, bc)
    N = 32
    b = np.random.default_rng(5).standard_normal((N - 1) ** 3)
    x = torch.zeros_like(dev(b))
    # restarted every 150 iterations: first kind converges in 25 runs, second kind does not
    # within 30 (both sides must agree on that too)
    rc, st = ex.level_solve(3, dev(b), x, 1e-8, 150, 30)
    xr, str_ = O.level_solve(N, bc, b, np.zeros_like(b), 1e-8, maxit=150, max_runs=30)
    assert rc == str_.code == (O.OK if bc == 1 else O.ENOCONV)
    assert (st["iterations"], st["runs"]) == (str_.iters, str_.runs)
    np.testing.assert_array_equal(host(x), xr)


# ------------------------------------------------------------------ whole cascade

def _solve_both(ex, prob, N, nl, bc, tol):
    arr = make_arrays(prob, N, bc)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    u = torch.empty_like(f)
    ut = torch.empty_like(f)
    rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, tol, u, ut)
    assert rc == ex.OK, ex.last_error()
    ref = O.excmg(N, nl, bc, arr.f, arr.g1, arr.g2, tol)
    return arr, host(u), host(ut), st, ref


def test_config1_solve(ex):
    """32^3 cells, first kind, sin(pi x) sin(pi y) sin(pi z), tol 1e-10."""
    arr, u, ut, st, ref = _solve_both(ex, config_problem(1), 32, 4, 1, 1e-10)
    print("levels", st.levels(), flush=True)
    assert rel_l2(u, ref.u.ravel()) <= 1e-10
    assert rel_l2(ut, ref.ut.ravel()) <= 1e-10
    assert [l["iterations"] for l in st.levels()[2:]] == [lv.iters for lv in ref.levels]


@pytest.mark.parametrize("bc", [1, 2])
def test_recomputing_form_fp64_matches_oracle(ex, bc):
    """FP64 Bi-CG in the recomputing form on every level (recompute_min_unknowns = 1): q and
    q* formed again in the update sweep, rho and r.r summed per tile, x updated once per two
    iterations, the update sweeps marching downwards.  The cascade equals the stored form's
    bit for bit and the oracle's counts and solution (1e-10), with graph windows and launch
    by launch."""
    N, nl = 48, 5
    arr = make_arrays(config_problem(2), N, bc)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    outs = []
    for m in (1 << 30, 1):
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u, recompute_min_unknowns=m)
        assert rc == ex.OK, ex.last_error()
        outs.append((host(u), [l["iterations"] for l in st.levels()]))
    assert outs[0][1] == outs[1][1]
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    ref = O.excmg(N, nl, bc, arr.f, arr.g1, arr.g2, 1e-9)
    assert outs[1][1][2:] == [lv.iters for lv in ref.levels]
    assert rel_l2(outs[1][0], ref.u.ravel()) <= 1e-10
    # launch by launch (event timing, no graphs): the same iterates; per level one sweep A
    # and one sweep B per iteration, the sweeps B of odd and even iterations apart
    ex.set_timing(True)
    try:
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u, recompute_min_unknowns=1)
        counts = [[ex.get_timing(li, k)[1] for k in range(5)] for li in range(nl)]
    finally:
        ex.set_timing(False)
    assert rc == ex.OK
    np.testing.assert_array_equal(host(u), outs[1][0])
    for li, lv in enumerate(st.levels()):
        n_a, n_b, n_x, n_keep, n_pair = counts[li]
        assert n_x == 0 and n_a == n_b + n_keep + n_pair == lv["iterations"]
        if lv["iterations"] >= 4:
            assert n_keep > 0 and n_pair > 0 and n_b <= lv["runs"]


@pytest.mark.parametrize("k", [2, 3])
def test_paper_problem_32cube(ex, k, golden_tables):
    """The cascade reproduces Table 2/3's 32^3 error columns (8^3 and 16^3 direct)."""
    arr, u, ut, st, ref = _solve_both(ex, paper_problem(k), 32, 3, 1, 1e-12)
    assert rel_l2(u, ref.u.ravel()) <= 1e-10
    e = u.ravel() - arr.u.ravel()
    assert float(f"{O.norm2(e):.2e}") == golden_tables["problems"][str(k)]["err2"][0]


@pytest.mark.timeout(600)
def test_config2_solve(ex):
    """128^3 cells, second kind, seeded family, tol 1e-10 (the oracle runs the whole
    cascade on the host)."""
    arr, u, ut, st, ref = _solve_both(ex, config_problem(2), 128, 6, 2, 1e-10)
    print("levels", st.levels(), flush=True)
    assert rel_l2(u, ref.u.ravel()) <= 1e-10
    assert rel_l2(ut, ref.ut.ravel()) <= 1e-10


# ------------------------------------------------------------------ batched solves

def _batch_inputs(items):
    out = []
    for (N, nl, bc, prob) in items:
        arr = make_arrays(prob, N, bc)
        out.append((N, nl, bc, arr, dev(arr.f), dev(arr.g1), dev(arr.g2)))
    return out


BATCH_ITEMS = [(16, 3, 1, 2), (24, 4, 2, 2), (32, 4, 1, 3), (48, 5, 2, 2), (32, 4, 2, 4),
               (12, 3, 1, 3)]


def _batch_problems():
    return _batch_inputs([(N, nl, bc, config_problem(c)) for (N, nl, bc, c) in BATCH_ITEMS])


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_fp64_matches_single_solves_and_oracle(ex, persistent):
    data = _batch_problems()
    probs = []
    for (N, nl, bc, arr, f, g1, g2) in data:
        probs.append(dict(n_finest=N, n_levels=nl, bc_kind=bc, f=f, g1=g1, g2=g2,
                          u_out=torch.empty_like(f), ut_out=torch.empty_like(f)))
    rc, stats = ex.solve_batch(probs, 1e-9, persistent=persistent)
    assert rc == ex.OK, ex.last_error()
    for (N, nl, bc, arr, f, g1, g2), p, st in zip(data, probs, stats):
        print(f"batch N={N} bc={bc}", [l["iterations"] for l in st.levels()], flush=True)
        u1 = torch.empty_like(f)
        rc1, st1 = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u1)
        assert rc1 == ex.OK
        assert [l["iterations"] for l in st.levels()] == [l["iterations"] for l in st1.levels()]
        np.testing.assert_array_equal(host(p["u_out"]), host(u1))
        ref = O.excmg(N, nl, bc, arr.f, arr.g1, arr.g2, 1e-9)
        assert rel_l2(host(p["u_out"]), ref.u) <= 1e-10
        assert rel_l2(host(p["ut_out"]), ref.ut) <= 1e-10


# Problem sizes of the 64-problem batch workload (32^3 ... 128^3 cells): coarsest grids of
# 4 and 3 cells, both boundary kinds; from 96^3 on the grids split into several 64-wide
# x tiles.
BATCH_LARGE = [(64, 5, 2, 2), (96, 6, 1, 3), (128, 6, 2, 4)]
_LARGE_REF = {}


def _large_ref(N, nl, bc, c, arr):
    key = (N, nl, bc, c)
    if key not in _LARGE_REF:
        print(f"oracle {N}^3 bc={bc}", flush=True)
        _LARGE_REF[key] = O.excmg(N, nl, bc, arr.f, arr.g1, arr.g2, 1e-9)
    return _LARGE_REF[key]


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_fp64_large_grids_match_single_solves_and_oracle(ex, persistent):
    data = _batch_inputs([(N, nl, bc, config_problem(c)) for (N, nl, bc, c) in BATCH_LARGE])
    probs = [dict(n_finest=N, n_levels=nl, bc_kind=bc, f=f, g1=g1, g2=g2,
                  u_out=torch.empty_like(f), ut_out=torch.empty_like(f))
             for (N, nl, bc, arr, f, g1, g2) in data]
    rc, stats = ex.solve_batch(probs, 1e-9, persistent=persistent)
    assert rc == ex.OK, ex.last_error()
    for (N, nl, bc, arr, f, g1, g2), item, p, st in zip(data, BATCH_LARGE, probs, stats):
        print(f"batch N={N} bc={bc}", [l["iterations"] for l in st.levels()], flush=True)
        u1 = torch.empty_like(f)
        rc1, st1 = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u1)
        assert rc1 == ex.OK
        assert [l["iterations"] for l in st.levels()] == [l["iterations"] for l in st1.levels()]
        np.testing.assert_array_equal(host(p["u_out"]), host(u1))
        ref = _large_ref(N, nl, bc, item[3], arr)
        assert [l["iterations"] for l in st.levels()[2:]] == [l.iters for l in ref.levels]
        assert rel_l2(host(p["u_out"]), ref.u) <= 1e-10
        assert rel_l2(host(p["ut_out"]), ref.ut) <= 1e-10


@pytest.mark.parametrize("refine", ["reliable", "restart"])
@pytest.mark.parametrize("persistent", [False, True])
def test_batch_mixed_large_grids_meet_tolerance_and_accuracy(ex, persistent, refine):
    """Levels under 2^18 unknowns run FP64 Bi-CG, the larger ones (95^3, 127^3) FP32 Bi-CG in
    FP64 refinement.  Both refinement forms meet the tolerance in the oracle's FP64 residual
    with the FP64 discretisation error; restarted refinement equals the single solve with the
    same split bit for bit, and residual replacement leaves the all-FP64 problem (64^3) equal
    to the FP64 solve."""
    mode = ex.RELIABLE if refine == "reliable" else ex.RESTART
    data = _batch_inputs([(N, nl, bc, config_problem(c)) for (N, nl, bc, c) in BATCH_LARGE])
    probs = [dict(n_finest=N, n_levels=nl, bc_kind=bc, f=f, g1=g1, g2=g2,
                  u_out=torch.empty_like(f)) for (N, nl, bc, arr, f, g1, g2) in data]
    rc, stats = ex.solve_batch(probs, 1e-9, precision=ex.MIXED, persistent=persistent,
                               refine=mode)
    assert rc == ex.OK, ex.last_error()
    for (N, nl, bc, arr, f, g1, g2), item, p, st in zip(data, BATCH_LARGE, probs, stats):
        u = host(p["u_out"]).reshape((N + 1,) * 3)
        b = O.rhs(N, bc, arr.f, arr.g1, arr.g2)
        r = O.residual(N, bc, b, O.interior(u))
        assert np.sqrt(O.dot(r, r) / O.dot(b, b)) <= 1e-9
        ref = _large_ref(N, nl, bc, item[3], arr)
        e_fp64 = O.norm2(ref.u - arr.u)
        assert abs(O.norm2(u - arr.u) - e_fp64) <= 0.01 * e_fp64
        print(f"batch mixed ({refine}) N={N}: iterations {[l['iterations'] for l in st.levels()]}, "
              f"max |u - u_oracle| = {np.abs(u - ref.u).max():.3e}", flush=True)
        if mode == ex.RELIABLE:
            if (N - 1) ** 3 < (1 << 18):
                single = torch.empty_like(f)
                assert ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, single)[0] == ex.OK
                np.testing.assert_array_equal(u.ravel(), host(single).ravel())
            continue
        single = torch.empty_like(f)
        rc1, st1 = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, single, precision=ex.MIXED,
                               refine=ex.RESTART, fp32_min_unknowns=1 << 18, inner_tol=1e-5)
        assert rc1 == ex.OK
        assert [l["iterations"] for l in st.levels()] == [l["iterations"] for l in st1.levels()]
        assert [l["runs"] for l in st.levels()] == [l["runs"] for l in st1.levels()]
        np.testing.assert_array_equal(u.ravel(), host(single).ravel())


def test_batch_autotuned_shapes_keep_results(ex):
    """The batch shape tuner times whole batch steps on the batch's own work list; the
    shapes it records leave every batched solution equal to the single solves."""
    items = [(32, 4, 1, 2), (48, 5, 2, 3), (64, 5, 1, 4), (96, 6, 2, 2)]
    data = _batch_inputs([(N, nl, bc, config_problem(c)) for (N, nl, bc, c) in items])
    probs = [dict(n_finest=N, n_levels=nl, bc_kind=bc, f=f, g1=g1, g2=g2,
                  u_out=torch.empty_like(f)) for (N, nl, bc, arr, f, g1, g2) in data]
    ty, ms = ex.autotune_batch(probs, precision=ex.FP64, reps=2)
    assert ty in (4, 8) and ms > 0
    shapes = {N: ex.get_batch_shape(N) for (N, *_rest) in items}
    print("batch shapes", shapes, f"{ms:.3f} ms per step (sizes alone, summed)", flush=True)
    assert all(t == ty and 1 <= zc <= N - 1 for N, (t, zc) in shapes.items())
    for persistent in (False, True):
        rc, stats = ex.solve_batch(probs, 1e-9, persistent=persistent)
        assert rc == ex.OK, ex.last_error()
        for (N, nl, bc, arr, f, g1, g2), p in zip(data, probs):
            u1 = torch.empty_like(f)
            assert ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u1)[0] == ex.OK
            np.testing.assert_array_equal(host(p["u_out"]), host(u1))
    # mixed: the 96^3 problem's finest level runs FP32 (its own tuned chunk)
    ty, ms = ex.autotune_batch(probs, precision=ex.MIXED, reps=2)
    print("mixed batch: ty", ty, "96^3 FP32 shape", ex.get_batch_shape(96, ex.MIXED),
          f"{ms:.3f} ms per step (sizes alone, summed)", flush=True)
    rc, stats = ex.solve_batch(probs, 1e-9, precision=ex.MIXED, refine=ex.RESTART)
    assert rc == ex.OK, ex.last_error()
    for (N, nl, bc, arr, f, g1, g2), p in zip(data, probs):
        u1 = torch.empty_like(f)
        assert ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u1, precision=ex.MIXED, refine=ex.RESTART,
                           fp32_min_unknowns=1 << 18, inner_tol=1e-5)[0] == ex.OK
        np.testing.assert_array_equal(host(p["u_out"]), host(u1))


@pytest.mark.parametrize("fp32_min", [0, 1])
def test_batch_mixed_meets_tolerance_and_accuracy(ex, fp32_min):
    """fp32_min 0: every level of these grids (up to 47^3 unknowns) is under 2^18 unknowns
    and runs FP64 Bi-CG, so the mixed batch equals the FP64 solves; 1: every level runs
    FP32 Bi-CG in restarted refinement, as the single restarted solve does."""
    data = _batch_problems()
    probs = [dict(n_finest=N, n_levels=nl, bc_kind=bc, f=f, g1=g1, g2=g2,
                  u_out=torch.empty_like(f)) for (N, nl, bc, arr, f, g1, g2) in data]
    rc, stats = ex.solve_batch(probs, 1e-8, precision=ex.MIXED, fp32_min_unknowns=fp32_min,
                               refine=ex.RESTART)
    assert rc == ex.OK, ex.last_error()
    for (N, nl, bc, arr, f, g1, g2), p, st in zip(data, probs, stats):
        u = host(p["u_out"]).reshape((N + 1,) * 3)
        # the oracle checks the final residual of the GPU's mixed-precision solution
        b = O.rhs(N, bc, arr.f, arr.g1, arr.g2)
        r = O.residual(N, bc, b, O.interior(u))
        assert np.sqrt(O.dot(r, r) / O.dot(b, b)) <= 1e-8
        ref = O.excmg(N, nl, bc, arr.f, arr.g1, arr.g2, 1e-8)
        e_mixed = O.norm2(u - arr.u)
        e_fp64 = O.norm2(ref.u - arr.u)
        assert abs(e_mixed - e_fp64) <= 0.01 * e_fp64
        single = torch.empty_like(f)
        if fp32_min == 0:
            rc1, st1 = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-8, single)
        else:
            # the batch path refines by restarted FP32 solves
            rc1, st1 = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-8, single, precision=ex.MIXED,
                                   refine=ex.RESTART, inner_tol=1e-5)
        assert rc1 == ex.OK
        assert [l["iterations"] for l in st.levels()] == [l["iterations"] for l in st1.levels()]
        np.testing.assert_array_equal(u.ravel(), host(single).ravel())


@pytest.mark.parametrize("refine", ["reliable", "restart"])
@pytest.mark.parametrize("case", [(32, 4, 1, 1, 1e-10), (64, 5, 2, 2, 1e-9)])
def test_mixed_solve_meets_tolerance(ex, refine, case):
    """Both refinement forms: the oracle's FP64 residual of the returned solution meets the
    tolerance, and its error against the exact solution is within 1% of the FP64 solve's."""
    N, nl, bc, c, tol = case
    arr = make_arrays(config_problem(c), N, bc)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    u = torch.empty_like(f)
    mode = ex.RELIABLE if refine == "reliable" else ex.RESTART
    rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, tol, u, precision=ex.MIXED, refine=mode,
                         fp32_min_unknowns=1)
    assert rc == ex.OK, ex.last_error()
    print(refine, [(l["iterations"], l["runs"]) for l in st.levels()], flush=True)
    ug = host(u).reshape((N + 1,) * 3)
    b = O.rhs(N, bc, arr.f, arr.g1, arr.g2)
    r = O.residual(N, bc, b, O.interior(ug))
    assert np.sqrt(O.dot(r, r) / O.dot(b, b)) <= tol
    ref = O.excmg(N, nl, bc, arr.f, arr.g1, arr.g2, tol)
    assert abs(O.norm2(ug - arr.u) - O.norm2(ref.u - arr.u)) <= 0.01 * O.norm2(ref.u - arr.u)


def test_mixed_default_runs_small_levels_in_fp64(ex):
    """Residual replacement keeps levels under 2^18 unknowns in FP64: those levels equal
    the FP64 solve's bit for bit, the 128^3 level runs FP32 with replacements, and the
    threshold can be moved (1: FP32 everywhere)."""
    N, nl, bc = 128, 5, 2          # levels of 8, 16, 32, 64 (250047 unknowns), 128 cells
    arr = make_arrays(config_problem(2), N, bc)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    sols = {}
    for name, kw in (("fp64", dict()), ("mixed", dict(precision=ex.MIXED)),
                     ("fp32all", dict(precision=ex.MIXED, fp32_min_unknowns=1))):
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u, **kw)
        assert rc == ex.OK, ex.last_error()
        levels = []
        for lv in range(nl):
            n = N >> (nl - 1 - lv)
            w = torch.empty((n + 1) ** 3, dtype=torch.float64, device="cuda")
            ex.get_level_solution(lv, w)
            levels.append(host(w))
        sols[name] = (st.levels(), levels)
    (s64, l64), (smx, lmx), (s32, l32) = sols["fp64"], sols["mixed"], sols["fp32all"]
    for lv in range(nl - 1):
        np.testing.assert_array_equal(lmx[lv], l64[lv])
        assert smx[lv]["iterations"] == s64[lv]["iterations"]
    assert smx[-1]["runs"] > 1                       # FP32 with residual replacements
    assert s32[3]["runs"] > 1                        # the 64^3 level too when asked
    assert not np.array_equal(l32[3], l64[3])
    with pytest.raises(ex.ExcmgError):
        ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, torch.empty_like(f), precision=ex.MIXED,
                    fp32_min_unknowns=-1)


@pytest.mark.parametrize("refine", ["reliable", "restart"])
def test_padded_rows_keep_the_mixed_solve(ex, refine):
    """The FP32 Bi-CG vectors (with the FP64 iterate and right-hand side they are solved
    with) on padded rows (row_pad = 1, every 3D level): the stencil sweeps see the same
    operator and the vector kernels walk the unknowns in the contiguous order, so the cascade
    gives the contiguous layout's iterates and counts; an invalid row_pad is refused."""
    N, nl, bc = 128, 6, 2
    arr = make_arrays(config_problem(2), N, bc)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    mode = ex.RELIABLE if refine == "reliable" else ex.RESTART
    outs, its = [], []
    for pad in (0, 1):
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u, precision=ex.MIXED, refine=mode,
                             fp32_min_unknowns=1, row_pad=pad)
        assert rc == ex.OK, ex.last_error()
        outs.append(host(u))
        its.append([(l["iterations"], l["runs"]) for l in st.levels()])
    assert its[0] == its[1]
    np.testing.assert_array_equal(outs[0], outs[1])
    with pytest.raises(ex.ExcmgError):
        ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, torch.empty_like(f), precision=ex.MIXED,
                    row_pad=3)


@pytest.mark.parametrize("refine", ["reliable", "restart"])
@pytest.mark.parametrize("case", [(48, 4, 1, 3, 1e-9), (80, 5, 2, 2, 1e-9), (112, 5, 1, 4, 1e-9),
                                  (160, 6, 2, 1, 1e-6)])
def test_two_point_sweeps_keep_the_mixed_solve(ex, refine, case):
    """row_pad = 2: the levels that take the recomputing form (here every level, FP32
    everywhere) run its two sweeps with two adjacent points per lane on padded rows: 128-wide
    tiles, ragged in x (47, 79, 111 and 159 unknowns per axis: partial tiles whose last lane
    holds one point), boundary pairs that mix fictitious points, boundary nodes and points
    beyond the grid, z-chunks shorter than the grid and whole-depth ones.  Per point the arithmetic is that of the single-point
    sweeps, so the cascade gives the same iterates, counts and solution bit for bit."""
    N, nl, bc, c, tol = case
    arr = make_arrays(config_problem(c), N, bc)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    mode = ex.RELIABLE if refine == "reliable" else ex.RESTART
    outs, its = [], []
    for pad in (0, 2):
        print(f"two-point sweeps N={N} bc={bc} {refine} row_pad={pad}", flush=True)
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, tol, u, precision=ex.MIXED, refine=mode,
                             fp32_min_unknowns=1, recompute_min_unknowns=1, row_pad=pad)
        assert rc == ex.OK, ex.last_error()
        outs.append(host(u))
        its.append([(l["iterations"], l["runs"]) for l in st.levels()])
    assert its[0] == its[1]
    np.testing.assert_array_equal(outs[0], outs[1])


def test_autotuned_shape_keeps_results(ex):
    N, bc = 40, 2
    ty, zc, ms = ex.autotune(N, 0, ex.FP64, reps=3)
    assert ty in (4, 8, 16) and 1 <= zc <= N - 1 and ms > 0
    assert ex.get_shape(N, 0) == (ty, zc)
    x = np.random.default_rng(8).standard_normal((N - 1) ** 3)
    y = torch.empty_like(dev(x))
    ex.apply_operator(N, bc, 0, dev(x), y)
    np.testing.assert_array_equal(host(y), O.apply(N, bc, x))
    ty1, zc1, _ = ex.autotune(N, 1, ex.MIXED, reps=3)
    assert ty1 in (4, 8, 16)
    assert ex.get_shape(N, 2) == (ty1, zc1)
    for kind in (0, 1, 2):
        ex.set_shape(N, kind, 0, 0)


def test_autotune_on_recomputing_grids_keeps_results(ex):
    """On grids of 2^22 unknowns and up (here 192^3 cells: 191^3 = 6.97e6 unknowns) the
    autotuner's kind 1 times the pair of sweeps Bi-CG runs there (sweep A marching p, sweep B
    forming q, q* again).  The shape it records leaves the mixed and the FP64 solve exactly as
    they are with the built-in shape."""
    N, nl, bc = 192, 7, 1
    print(f"autotune recomputing pair {N}^3", flush=True)
    arr = make_arrays(config_problem(3), N, bc, with_u=False)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)

    def solve(prec):
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-8, u, precision=prec)
        assert rc == ex.OK, ex.last_error()
        return host(u), [(lv["iterations"], lv["runs"]) for lv in st.levels()]

    for prec, kind, tys in ((ex.MIXED, 2, (4, 8, 16)), (ex.FP64, 1, (4, 8))):
        u0, it0 = solve(prec)
        ty, zc, ms = ex.autotune(N, 1, prec, reps=2)
        try:
            assert ty in tys and 1 <= zc <= N - 1 and ms > 0
            assert ex.get_shape(N, kind) == (ty, zc)
            u1, it1 = solve(prec)
        finally:
            ex.set_shape(N, kind, 0, 0)
        assert it1 == it0
        np.testing.assert_array_equal(u1, u0)


# ------------------------------------------------------------------ CG specialisation

def test_deferred_update_keeps_bicg_equal_to_cg(ex):
    """On the 64^3 and 128^3 grids the mixed Bi-CG moves x += alpha p from sweep B into the
    next sweep A (same arithmetic, applied one launch later, and on its own when a run stops);
    the CG form keeps it in its update sweep.  Both must give the same iterates bit for bit,
    through residual replacements and window ends."""
    N, nl, bc = 128, 6, 2
    arr = make_arrays(config_problem(2), N, bc)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    u_b, u_c = torch.empty_like(f), torch.empty_like(f)
    rc1, st1 = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u_b, precision=ex.MIXED, method=ex.BICG,
                           fp32_min_unknowns=1)
    rc2, st2 = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u_c, precision=ex.MIXED, method=ex.CG,
                           fp32_min_unknowns=1)
    assert rc1 == rc2 == ex.OK
    assert [(l["iterations"], l["runs"]) for l in st1.levels()] == \
        [(l["iterations"], l["runs"]) for l in st2.levels()]
    assert st1.levels()[-1]["runs"] > 1
    np.testing.assert_array_equal(host(u_b), host(u_c))

def test_recomputing_form_keeps_the_mixed_solve(ex):
    """On large 3D grids the mixed Bi-CG forms q = A p and q* = A^T p* again in its update
    sweep instead of storing them (same roundings, same update arithmetic), and its sweeps B
    update the FP64 iterate once per two iterations (x += alpha' p' + alpha p, rounded as two
    updates).  Forced on every level at 128^3 (recompute_min_unknowns = 1) it gives the stored
    form's iterates and counts bit for bit, and the CG form's; launch by launch (event timing)
    too, one sweep A and one sweep B per iteration, the sweeps B of odd and even iterations
    counted apart; a negative threshold is refused."""
    N, nl, bc = 128, 6, 2
    arr = make_arrays(config_problem(2), N, bc)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    outs, its = [], []
    for kw in (dict(recompute_min_unknowns=1 << 30), dict(recompute_min_unknowns=1),
               dict(method=ex.CG)):
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u, precision=ex.MIXED,
                             fp32_min_unknowns=1, **kw)
        assert rc == ex.OK, ex.last_error()
        outs.append(host(u))
        its.append([(l["iterations"], l["runs"]) for l in st.levels()])
    assert its[0] == its[1] == its[2]
    assert its[1][-1][1] > 1                      # residual replacements happened
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[2], outs[1])
    ex.set_timing(True)
    u = torch.empty_like(f)
    rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u, precision=ex.MIXED,
                         fp32_min_unknowns=1, recompute_min_unknowns=1)
    _, n_a = ex.get_timing(nl - 1, 0)
    _, n_b = ex.get_timing(nl - 1, 1)
    _, n_x = ex.get_timing(nl - 1, 2)
    _, n_keep = ex.get_timing(nl - 1, 3)   # odd iterations: x left to the next sweep B
    _, n_pair = ex.get_timing(nl - 1, 4)   # even iterations: both updates
    ex.set_timing(False)
    assert rc == ex.OK
    assert n_x == 0 and n_a == n_b + n_keep + n_pair == its[1][-1][0]
    assert n_keep > 0 and n_pair > 0
    # per run or resumed run, the odd and even sweeps alternate (one leading sweep B may
    # update x once)
    assert abs(n_keep - n_pair) <= its[1][-1][1] + 1 and n_b <= its[1][-1][1] + 1
    np.testing.assert_array_equal(host(u), outs[1])
    with pytest.raises(ex.ExcmgError):
        ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, torch.empty_like(f), precision=ex.MIXED,
                    recompute_min_unknowns=-1)


def test_event_timed_solve_equals_the_graph_solve(ex):
    """With per-sweep timing on, a solve runs its iterations launch by launch (no captured
    graphs), the deferred update of the mixed form included; it must give the same
    iterates, and the timings must count every sweep that did work."""
    N, nl, bc = 128, 6, 2
    arr = make_arrays(config_problem(2), N, bc)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    outs, its = [], []
    for timing in (False, True):
        ex.set_timing(timing)
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u, precision=ex.MIXED,
                             fp32_min_unknowns=1)
        assert rc == ex.OK, ex.last_error()
        outs.append(host(u))
        its.append([(l["iterations"], l["runs"]) for l in st.levels()])
    ms_a, n_a = ex.get_timing(nl - 1, 0)   # sweeps A owing no update (first of each run)
    ms_b, n_b = ex.get_timing(nl - 1, 1)
    ms_x, n_x = ex.get_timing(nl - 1, 2)   # sweeps A applying the deferred update
    ex.set_timing(False)
    assert its[0] == its[1]
    np.testing.assert_array_equal(outs[0], outs[1])
    assert n_a + n_x == n_b == its[1][-1][0]
    assert n_x > n_a > 0 and ms_x > 0 and ms_b > 0

@pytest.mark.parametrize("form", ["stored", "recomputing"])
@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed-restart"])
@pytest.mark.parametrize("case", [(32, 4, 1, 1), (48, 5, 2, 2)])
def test_cg_specialisation_is_bit_identical_to_bicg(ex, prec, case, form):
    """With A_h = A_h^T and r*_0 = r_0 the shadow vectors of Algorithm 2 equal the primal
    ones, so the CG form (one operator product per iteration) reproduces Bi-CG exactly; also
    when Bi-CG takes the recomputing form (forced on every level here; CG keeps the stored
    one)."""
    N, nl, bc, c = case
    p = ex.FP64 if prec == "fp64" else ex.MIXED
    mode = ex.RESTART if prec == "mixed-restart" else ex.RELIABLE
    rq = 1 if form == "recomputing" else 1 << 30
    arr = make_arrays(config_problem(c), N, bc)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    u_b, u_c = torch.empty_like(f), torch.empty_like(f)
    rc1, st1 = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u_b, precision=p, method=ex.BICG,
                           refine=mode, fp32_min_unknowns=1, recompute_min_unknowns=rq)
    rc2, st2 = ex.solve_ex(N, nl, bc, f, g1, g2, 1e-9, u_c, precision=p, method=ex.CG,
                           refine=mode, fp32_min_unknowns=1, recompute_min_unknowns=rq)
    assert rc1 == rc2 == ex.OK
    assert [l["iterations"] for l in st1.levels()] == [l["iterations"] for l in st2.levels()]
    np.testing.assert_array_equal(host(u_b), host(u_c))
    # against the oracle (Algorithm 2 with r*_0 = r_0, both products, in FP64)
    ref = _cg_oracle(N, nl, bc, c)
    uc = host(u_c).reshape((N + 1,) * 3)
    if prec == "fp64":
        assert [l["iterations"] for l in st2.levels()[2:]] == [l.iters for l in ref.levels]
        assert rel_l2(uc, ref.u) <= 1e-10
    else:
        b = O.rhs(N, bc, arr.f, arr.g1, arr.g2)
        r = O.residual(N, bc, b, O.interior(uc))
        assert np.sqrt(O.dot(r, r) / O.dot(b, b)) <= 1e-9
        e_ref = O.norm2(ref.u - arr.u)
        assert abs(O.norm2(uc - arr.u) - e_ref) <= 0.01 * e_ref


_CG_ORACLE = {}


def _cg_oracle(N, nl, bc, c):
    key = (N, nl, bc, c)
    if key not in _CG_ORACLE:
        arr = make_arrays(config_problem(c), N, bc)
        _CG_ORACLE[key] = O.excmg(N, nl, bc, arr.f, arr.g1, arr.g2, 1e-9)
    return _CG_ORACLE[key]
