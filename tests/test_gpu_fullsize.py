"""Parity at the benchmark's full size (512^3 cells, second kind, the benchmark's problem and
launch shapes): the operator element by element, the first Bi-CG iterations of the finest
level bit for bit against the oracle, and the benchmark's solves through properties that
hold at any size (the oracle's FP64 residual of the returned solution, the discretisation
error against the exact solution).  The 256^3 first-kind case is solved at its full size too."""
import numpy as np
import pytest

import oracle as O
from manufactured import config_problem, make_arrays

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, NL, BC = 512, 8, 2
NU = (N - 1) ** 3


@pytest.fixture(scope="module")
def ex():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_05118_amd as ex
    ex.load()
    yield ex
    ex.finalize()


@pytest.fixture(scope="module")
def problem():
    print("generating the 512^3 problem", flush=True)
    arr = make_arrays(config_problem(4), N, BC)
    b = O.rhs(N, BC, arr.f, arr.g1, arr.g2)
    return arr, b


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def test_operator_at_full_size(ex):
    print("operator 512^3", flush=True)
    x = np.random.default_rng(512).standard_normal(NU)
    y = torch.empty(NU, dtype=torch.float64, device="cuda")
    ex.apply_operator(N, BC, 0, dev(x), y)
    np.testing.assert_array_equal(host(y), O.apply(N, BC, x))


def test_first_bicg_iterations_at_full_size(ex, problem):
    """Two iterations of Algorithm 2 on the 512^3 level of the benchmark's hierarchy: the
    FP64 sweeps in their tuned launch shapes give the oracle's iterate bit for bit."""
    print("bicg 512^3", flush=True)
    arr, b = problem
    ex.setup(N, NL, BC)
    x = torch.zeros(NU, dtype=torch.float64, device="cuda")
    rc, it, rr = ex.bicg(NL - 1, dev(b), x, 1e-30, max_iters=2)
    xo, ito, rro, rco = O.bicg(N, BC, b, np.zeros(NU), 1e-30, maxit=2)
    assert it == ito == 2 and rr == rro
    np.testing.assert_array_equal(host(x), xo)


def test_benchmark_solves_meet_tolerance(ex, problem):
    """The benchmark's solves: for both precisions the oracle's FP64 residual of the returned
    solution meets 1e-8 (the exact solution's own residual is 1.6e-8: the tolerance sits at
    the discretisation floor), and the mixed solve's RMS error against the exact solution is
    the FP64 solve's within 1%."""
    arr, b = problem
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    errs = {}
    for name, p in (("fp64", ex.FP64), ("mixed", ex.MIXED)):
        print(f"solve 512^3 {name}", flush=True)
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(N, NL, BC, f, g1, g2, 1e-8, u, precision=p)
        assert rc == ex.OK, ex.last_error()
        ug = host(u).reshape((N + 1,) * 3)
        del u
        r = O.residual(N, BC, b, O.interior(ug))
        assert np.sqrt(O.dot(r, r) / O.dot(b, b)) <= 1e-8
        errs[name] = O.norm2(ug - arr.u)
    assert abs(errs["mixed"] - errs["fp64"]) <= 0.01 * errs["fp64"]


def test_first_kind_256_mixed_against_fp64(ex):
    """256^3 cells, first kind, the seeded four-mode family, tol 1e-8, 7 levels: both solves
    leave an FP64 residual (the oracle's) within the tolerance; the mixed solution is within
    1% of the FP64 solution's max-norm error against the exact u, and so is its distance from
    the FP64 solution."""
    n, nl, bc = 256, 7, 1
    print("generating the 256^3 first-kind problem", flush=True)
    arr = make_arrays(config_problem(3), n, bc)
    b = O.rhs(n, bc, arr.f, arr.g1, arr.g2)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    sols, errs = {}, {}
    for name, p in (("fp64", ex.FP64), ("mixed", ex.MIXED)):
        print(f"solve 256^3 first kind {name}", flush=True)
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(n, nl, bc, f, g1, g2, 1e-8, u, precision=p)
        assert rc == ex.OK, ex.last_error()
        ug = host(u).reshape((n + 1,) * 3)
        del u
        r = O.residual(n, bc, b, O.interior(ug))
        assert np.sqrt(O.dot(r, r) / O.dot(b, b)) <= 1e-8
        sols[name] = ug
        errs[name] = float(np.abs(ug - arr.u).max())
    assert abs(errs["mixed"] - errs["fp64"]) <= 0.01 * errs["fp64"]
    assert float(np.abs(sols["mixed"] - sols["fp64"]).max()) <= 0.01 * errs["fp64"]


def test_mixed_bicg_equals_cg_at_full_size(ex, problem):
    """The mixed Bi-CG takes the recomputing form on the 256^3 and 512^3 levels (q and q*
    formed again in the update sweep, whose partials are per tile).  The CG form, which
    stores q, must match bit for bit, and so must the solves on padded rows (row_pad = 1)
    and with the two-point sweeps on those levels (row_pad = 2)."""
    print("mixed bicg vs cg 512^3", flush=True)
    arr, b = problem
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    outs, its = [], []
    for m, pad in ((ex.BICG, 0), (ex.CG, 0), (ex.BICG, 1), (ex.BICG, 2)):
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(N, NL, BC, f, g1, g2, 1e-8, u, precision=ex.MIXED, method=m,
                             row_pad=pad)
        assert rc == ex.OK, ex.last_error()
        outs.append(host(u))
        its.append([(l["iterations"], l["runs"]) for l in st.levels()])
        del u
    assert its[0] == its[1] == its[2] == its[3]
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])
    np.testing.assert_array_equal(outs[0], outs[3])


def test_fp64_bicg_equals_cg_at_full_size(ex, problem):
    """The FP64 Bi-CG of the benchmark takes the recomputing form on the 256^3 and 512^3
    levels, with the iterate updated once per two iterations and, on the 256^3 level, its
    update sweep marching each chunk from the top plane down.  The CG form (stored q, one
    x update per iteration, upward sweeps) must match bit for bit."""
    print("fp64 bicg vs cg 512^3", flush=True)
    arr, b = problem
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    outs, its = [], []
    for m in (ex.BICG, ex.CG):
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(N, NL, BC, f, g1, g2, 1e-8, u, precision=ex.FP64, method=m)
        assert rc == ex.OK, ex.last_error()
        outs.append(host(u))
        its.append([(l["iterations"], l["runs"]) for l in st.levels()])
        del u
    assert its[0] == its[1]
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_profiled_sweeps_of_the_recomputing_form(ex, prec):
    """The launcher of single sweeps (excmg_profile_sweep 7-10: sweep A, and sweep B with one,
    no and two x updates) runs the solver's sweeps on the 256^3 level and reports their
    algorithmic bytes per unknown."""
    p = ex.FP64 if prec == "fp64" else ex.MIXED
    ex.setup(256, 7, BC)
    nu = 255 ** 3
    want = {7: 48, 8: 64, 9: 48, 10: 72} if prec == "fp64" else {7: 24, 8: 40, 9: 24, 10: 44}
    for which, bpu in want.items():
        ms, nb = ex.profile_sweep(which, p, reps=2)
        assert ms > 0 and nb == bpu * nu
    with pytest.raises(ex.ExcmgError):
        ex.profile_sweep(11, p, reps=1)
