"""Algorithm 2 with its options on the GPU against the oracle: diagonal preconditioner M,
a chosen shadow residual, the dual system A^T x* = b* with its iterate x*.  Both sides
evaluate every formula in the same order, so iterates, iteration counts and residuals are
compared for exact equality."""
import numpy as np
import pytest

import oracle as O
from manufactured import config_problem, make_arrays

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


@pytest.mark.parametrize("bc", [1, 2])
@pytest.mark.parametrize("N", [8, 16, 64])
def test_diagonal_equals_the_oracle(ex, N, bc):
    nl = {8: 3, 16: 3, 64: 4}[N]
    ex.setup(N, nl, bc)
    d = torch.empty((N - 1) ** 3, dtype=torch.float64, device="cuda")
    ex.diagonal(nl - 1, d)
    np.testing.assert_array_equal(host(d), O.diagonal(N, bc))


def _system(N, bc, seed):
    rng = np.random.default_rng(seed)
    n = (N - 1) ** 3
    arr = make_arrays(config_problem(2), N, bc)
    b = O.rhs(N, bc, arr.f, arr.g1, arr.g2)
    return rng, n, b


@pytest.mark.parametrize("variant", ["jacobi", "shadow", "dual", "jacobi+dual"])
@pytest.mark.parametrize("case", [(16, 1), (32, 2), (40, 1)])
def test_bicg_variants_equal_the_oracle(ex, variant, case):
    N, bc = case
    rng, n, b = _system(N, bc, N + bc)
    x0 = rng.standard_normal(n) * 1e-3
    md = O.diagonal(N, bc) if "jacobi" in variant else None
    shadow = rng.standard_normal(n) if variant == "shadow" else None
    bstar = rng.standard_normal(n) if "dual" in variant else None
    xs0 = rng.standard_normal(n) if "dual" in variant else None
    maxit = 60
    xo, xso, ito, rro, rco = O.bicg_ex(N, bc, b, x0, 1e-9, maxit=maxit, shadow=shadow,
                                       bstar=bstar, xstar0=xs0, mdiag=md)
    levels = {16: 3, 32: 3, 40: 4}[N]
    ex.setup(N, levels, bc)
    x = dev(x0)
    xs = dev(xs0) if xs0 is not None else None
    rc, it, rr = ex.bicg_ex(levels - 1, dev(b), x, 1e-9, max_iters=maxit,
                            shadow=None if shadow is None else dev(shadow),
                            bstar=None if bstar is None else dev(bstar), xstar=xs,
                            mdiag=None if md is None else dev(md))
    print(variant, N, bc, "iterations", it, ito, flush=True)
    assert it == ito and rr == rro
    assert (rc == ex.OK) == (rco == O.OK)
    np.testing.assert_array_equal(host(x), xo)
    if xs is not None:
        np.testing.assert_array_equal(host(xs), xso)


def test_bicg_ex_argument_checks(ex):
    ex.setup(16, 3, 1)
    n = 15 ** 3
    b, x, v = dev(np.ones(n)), dev(np.zeros(n)), dev(np.ones(n))
    with pytest.raises(ex.ExcmgError):
        ex.bicg_ex(2, b, x, 1e-8, bstar=v)               # no xstar
    with pytest.raises(ex.ExcmgError):
        ex.bicg_ex(2, b, x, 1e-8, shadow=v, bstar=v, xstar=dev(np.zeros(n)))


@pytest.mark.parametrize("case", [(32, 4, 1, 1), (48, 5, 2, 2)])
def test_jacobi_cascade_equals_the_oracle(ex, case):
    N, nl, bc, c = case
    arr = make_arrays(config_problem(c), N, bc)
    u = torch.empty((N + 1,) * 3, dtype=torch.float64, device="cuda")
    rc, st = ex.solve_ex(N, nl, bc, dev(arr.f), dev(arr.g1), dev(arr.g2), 1e-9, u,
                         precond=ex.PRECOND_JACOBI)
    assert rc == ex.OK, ex.last_error()
    ref = O.excmg(N, nl, bc, arr.f, arr.g1, arr.g2, 1e-9, jacobi=True)
    assert [l["iterations"] for l in st.levels()[2:]] == [s.iters for s in ref.levels]
    np.testing.assert_array_equal(host(u), ref.u)


def test_jacobi_needs_fp64_bicg(ex):
    arr = make_arrays(config_problem(1), 16, 1)
    u = torch.empty((17,) * 3, dtype=torch.float64, device="cuda")
    for kw in (dict(precision=ex.MIXED), dict(method=ex.CG)):
        with pytest.raises(ex.ExcmgError):
            ex.solve_ex(16, 3, 1, dev(arr.f), dev(arr.g1), dev(arr.g2), 1e-9, u,
                        precond=ex.PRECOND_JACOBI, **kw)
