"""Failure handling and determinism of the HIP library, forced from the host (no kernel is
made to fault or hang: every case ends through the library's own status checks)."""
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


def _inputs(k=2, N=32, bc=1):
    arr = make_arrays(config_problem(k), N, bc)
    return arr, dev(arr.f), dev(arr.g1), dev(arr.g2)


def test_nan_forcing_reports_breakdown(ex):
    arr, f, g1, g2 = _inputs()
    f[16, 16, 16] = float("nan")
    u = torch.empty_like(f)
    rc, st = ex.solve_ex(32, 4, 1, f, g1, g2, 1e-8, u)
    assert rc == ex.EBREAKDOWN
    broken = [l for l in st.levels() if l["status"] == ex.EBREAKDOWN]
    assert broken and all(l["exit"] == ex.EXIT_BREAKDOWN for l in broken)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_breakdown_ends_the_level_as_a_single_solve_does(ex, prec):
    """A NaN in one problem of a batch: that problem's levels end as in a single solve (FP64:
    the Bi-CG run breaks down, the level reports EBREAKDOWN and the cascade goes on; mixed
    precision with restarts, FP32 on every level: the FP64 residual is not finite, so
    refinement stops at once), and the other problem is unharmed."""
    p = ex.FP64 if prec == "fp64" else ex.MIXED
    arr, f, g1, g2 = _inputs()
    f[16, 16, 16] = float("nan")
    arr2, f2, g12, g22 = _inputs(3, 32, 2)
    u_single = torch.empty_like(f)
    rc1, st1 = ex.solve_ex(32, 4, 1, f, g1, g2, 1e-8, u_single, precision=p, refine=ex.RESTART,
                           inner_tol=1e-5)
    assert rc1 == (ex.EBREAKDOWN if prec == "fp64" else ex.ENOCONV)
    ub, ub2 = torch.empty_like(f), torch.empty_like(f2)
    probs = [dict(n_finest=32, n_levels=4, bc_kind=1, f=f, g1=g1, g2=g2, u_out=ub),
             dict(n_finest=32, n_levels=4, bc_kind=2, f=f2, g1=g12, g2=g22, u_out=ub2)]
    rc, sts = ex.solve_batch(probs, 1e-8, precision=p, fp32_min_unknowns=1, refine=ex.RESTART)
    assert rc == rc1
    single = st1.levels()
    batched = sts[0].levels()
    assert [l["status"] for l in batched] == [l["status"] for l in single]
    assert [l["exit"] for l in batched] == [l["exit"] for l in single]
    assert [l["iterations"] for l in batched] == [l["iterations"] for l in single]
    assert all(l["status"] == ex.OK for l in sts[1].levels())
    if prec == "fp64":
        np.testing.assert_array_equal(ub.cpu().numpy(), u_single.cpu().numpy())


def test_call_without_context_returns_enoctx(ex):
    ex.finalize()
    x = torch.zeros(27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(ex.ExcmgError) as e:
        ex.apply_stencil(0, 0, x, y)
    assert e.value.code == ex.ENOCTX
    assert ex.load().excmg_profile_sweep(0, ex.FP64, 1, None, None) == ex.ENOCTX
    # a context made afterwards works again
    ex.setup(16, 3, 1)
    ex.apply_stencil(0, 0, x, y)


def test_iteration_cap_reports_no_convergence(ex):
    arr, f, g1, g2 = _inputs()
    u = torch.empty_like(f)
    rc, st = ex.solve_ex(32, 4, 1, f, g1, g2, 1e-10, u, max_iters=3, max_runs=2)
    assert rc == ex.ENOCONV
    lv = st.levels()
    assert all(l["iterations"] <= 6 for l in lv[2:])
    # the tolerances are far above the floor: the caps stopped these levels
    assert all(l["exit"] == ex.EXIT_CAP and l["eps"] > 10 * l["floor"] > 0 for l in lv[2:])
    assert np.isfinite(u.cpu().numpy()).all()


def test_tolerance_below_the_fp64_floor_stops(ex):
    """Problem 1 has zero boundary data; at 32^3 its relative-residual floor is ~4e-12, so
    1e-14 cannot be met: the level stops after max_runs Bi-CG runs instead of looping."""
    arr = make_arrays(paper_problem(1), 32, 1)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    u = torch.empty_like(f)
    rc, st = ex.solve_ex(32, 3, 1, f, g1, g2, 1e-14, u, max_runs=5)
    assert rc == ex.ENOCONV
    last = st.levels()[-1]
    assert last["rel_residual"] > 1e-14
    # the level's tolerance is below 10x the estimated floor, and the level stops as soon
    # as a further run no longer halves the squared residual
    assert 1e-14 < 10 * last["floor"] and last["exit"] == ex.EXIT_FLOOR
    assert last["runs"] < 5
    for mode in (ex.RELIABLE, ex.RESTART):
        # refinement stops when a step no longer reduces the FP64 residual
        rc, st = ex.solve_ex(32, 3, 1, f, g1, g2, 1e-14, u, precision=ex.MIXED, refine=mode,
                             fp32_min_unknowns=1)
        assert rc == ex.ENOCONV
        last = st.levels()[-1]
        assert last["rel_residual"] < 1e-9
        assert last["exit"] == ex.EXIT_FLOOR


def test_solves_are_deterministic(ex):
    arr, f, g1, g2 = _inputs(3, 48, 2)
    outs = []
    for prec in (ex.FP64, ex.FP64, ex.MIXED, ex.MIXED):  # mixed: reliable updates
        u = torch.empty_like(f)
        rc, st = ex.solve_ex(48, 5, 2, f, g1, g2, 1e-9, u, precision=prec, fp32_min_unknowns=1)
        assert rc == ex.OK
        outs.append(u.cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[2], outs[3])


def test_host_arrays_through_solve(ex):
    arr, f, g1, g2 = _inputs(1, 32, 1)
    u_host = np.empty_like(arr.f)
    rc, st = ex.solve_ex(32, 4, 1, arr.f, arr.g1, arr.g2, 1e-10, u_host)
    assert rc == ex.OK
    u_dev = torch.empty_like(f)
    ex.solve_ex(32, 4, 1, f, g1, g2, 1e-10, u_dev)
    np.testing.assert_array_equal(u_host, u_dev.cpu().numpy())


def test_level_solutions_form_the_tables_w_column(ex, golden_tables):
    """||w_h - u_h||_2 of Table 2 at 32^3 from the per-level solutions of one GPU solve."""
    arr = make_arrays(paper_problem(2), 32, 1)
    f, g1, g2 = dev(arr.f), dev(arr.g1), dev(arr.g2)
    u = torch.empty_like(f)
    rc, st = ex.solve_ex(32, 3, 1, f, g1, g2, 1e-12, u)
    assert rc == ex.OK
    u8 = torch.empty((9,) * 3, dtype=torch.float64, device="cuda")
    u16 = torch.empty((17,) * 3, dtype=torch.float64, device="cuda")
    ex.get_level_solution(0, u8)
    ex.get_level_solution(1, u16)
    w = torch.empty_like(f)
    ex.exp_finite(32, u16, u8, w)
    e = w.cpu().numpy() - u.cpu().numpy()
    assert float(f"{O.norm2(e):.2e}") == golden_tables["problems"]["2"]["w_err2"][0]


def test_hierarchy_beyond_device_memory_is_refused_and_released(ex):
    """2048^3 cells (nine vectors of 68.6 GB each) does not fit in HBM: set-up reports
    ENOMEM, frees what it had allocated, and a later solve equals one made before it."""
    arr, f, g1, g2 = _inputs()
    u0 = torch.empty_like(f)
    assert ex.solve_ex(32, 4, 1, f, g1, g2, 1e-8, u0)[0] == ex.OK
    free0, _ = torch.cuda.mem_get_info()
    rc = ex.load().excmg_setup(2048, 9, 1)
    assert rc == ex.ENOMEM
    assert "allocation" in ex.last_error()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0 - (1 << 30)
    u1 = torch.empty_like(f)
    assert ex.solve_ex(32, 4, 1, f, g1, g2, 1e-8, u1)[0] == ex.OK
    assert torch.equal(u0, u1)
