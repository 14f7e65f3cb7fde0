"""EXP_finite without allocation (excmg_exp_finite_noalloc, for callers that cannot allocate
device memory) against the allocating entry point excmg_exp_finite: the same kernels, so
the results must be equal bit for bit, on two calls in a row (the second on a smaller grid,
which reuses the fixed array the first one filled)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ex():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_05118_amd as ex
    ex.load()
    yield ex


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _coarse(n, seed):
    """Node arrays of n/2 and n/4 cells (seeded)."""
    rng = np.random.default_rng(seed)
    m1, m0 = n // 2 + 1, n // 4 + 1
    return (torch.from_numpy(rng.standard_normal(m1 ** 3)).cuda(),
            torch.from_numpy(rng.standard_normal(m0 ** 3)).cuda())


def test_noalloc_exp_finite_matches_the_allocating_call(ex):
    lib = ex.load()
    for n, seed in ((256, 11), (36, 12)):
        u1, u0 = _coarse(n, seed)
        w_ref = torch.empty((n + 1) ** 3, dtype=torch.float64, device="cuda")
        w = torch.full_like(w_ref, float("nan"))
        ex.exp_finite(n, u1, u0, w_ref)
        print(f"exp_finite_noalloc n={n}", flush=True)
        rc = lib.excmg_exp_finite_noalloc(n, _p(u1), _p(u0), _p(w))
        assert rc == ex.OK, ex.last_error()
        torch.cuda.synchronize()
        assert torch.equal(w, w_ref)


def test_noalloc_exp_finite_rejects_what_it_cannot_do(ex):
    lib = ex.load()
    u1, u0 = _coarse(8, 1)
    w = torch.empty(9 ** 3, dtype=torch.float64, device="cuda")
    assert lib.excmg_exp_finite_noalloc(260, _p(u1), _p(u0), _p(w)) == ex.EINVAL  # > 256
    assert lib.excmg_exp_finite_noalloc(10, _p(u1), _p(u0), _p(w)) == ex.EINVAL   # not 4k
    assert lib.excmg_exp_finite_noalloc(8, None, _p(u0), _p(w)) == ex.EINVAL
    host = np.zeros(9 ** 3)
    rc = lib.excmg_exp_finite_noalloc(8, _p(u1), _p(u0), ctypes.c_void_p(host.ctypes.data))
    assert rc == ex.EINVAL and "device" in ex.last_error()
