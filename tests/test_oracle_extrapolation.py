"""Pins of the oracle's EXP_finite (Sec. 4.2.2-4.2.3, Steps 1-5) and EXP_true (Sec. 4.2.1).

References: the paper's 1D formulas eqs. (secfff), (bfsec), (sifen1), (sifen2), (t1) and
(chenlin) typed from the text; polynomial reproduction; an independent separable
(tensor-product) formulation; the observed convergence orders."""
import numpy as np
import pytest

import oracle as O


def _nodes_1d(vals, N):
    """Node array on N cells whose values depend on x only."""
    return np.broadcast_to(np.asarray(vals)[None, None, :], (N + 1, N + 1, N + 1)).copy()


@pytest.mark.parametrize("N", [4, 8, 12])
def test_exp_finite_reduces_to_paper_1d_formulas(N):
    rng = np.random.default_rng(N)
    u1 = rng.standard_normal(N // 2 + 1)   # Z1 values (cells of size 2h)
    u0 = rng.standard_normal(N // 4 + 1)   # Z0 values (cells of size 4h)
    w = O.exp_finite(N, _nodes_1d(u1, N // 2), _nodes_1d(u0, N // 4))
    # every yz line must carry the same 1D result
    assert np.ptp(w, axis=(0, 1)).max() <= 1e-13 * np.abs(w).max()
    w1 = w[0, 0, :]
    for c in range(N // 4):   # Z0 cell (x_j, x_{j+1})
        U1j, U1m, U1k = u1[2 * c], u1[2 * c + 1], u1[2 * c + 2]
        U0j, U0k = u0[c], u0[c + 1]
        secfff_j = (5 * U1j - U0j) / 4
        secfff_k = (5 * U1k - U0k) / 4
        bfsec = U1m + (U1j - U0j + U1k - U0k) / 8
        sifen1 = ((9 * U1j + 12 * U1m - U1k) - (3 * U0j + U0k)) / 16
        sifen2 = ((9 * U1k + 12 * U1m - U1j) - (3 * U0k + U0j)) / 16
        got = w1[4 * c: 4 * c + 5]
        np.testing.assert_allclose(got, [secfff_j, sifen1, bfsec, sifen2, secfff_k],
                                   rtol=0, atol=1e-14 * 8)


@pytest.mark.parametrize("N", [4, 8])
def test_exp_finite_reproduces_triquadratics(N):
    """With u1 = u0 at the coarse nodes the extrapolation terms vanish and Step 5 is
    tri-quadratic interpolation, exact for polynomials of degree <= 2 in each variable."""
    q = lambda X, Y, Z: 1 + X - 2 * Y * Z + 3 * X**2 * Y**2 * Z**2 - X * Z**2  # noqa: E731
    def grid(M):
        t = np.arange(M + 1) / M
        Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
        return q(X, Y, Z)
    w = O.exp_finite(N, grid(N // 2), grid(N // 4))
    np.testing.assert_allclose(w, grid(N), rtol=0, atol=1e-13)


def _separable_exp_finite(N, u1, u0):
    """Independent tensor-product form: w = Q(u1 + 1/4 T(u1|Z0 - u0)), T trilinear Z0->Z1,
    Q piecewise quadratic Z1->Z2 on Z0 cells, applied axis by axis."""
    d = u1[::2, ::2, ::2] - u0
    def lin_up(a, axis):  # Z0 -> Z1 along one axis
        a = np.moveaxis(a, axis, 0)
        out = np.empty((2 * a.shape[0] - 1,) + a.shape[1:])
        out[::2] = a
        out[1::2] = 0.5 * (a[:-1] + a[1:])
        return np.moveaxis(out, 0, axis)
    t = d
    for ax in range(3):
        t = lin_up(t, ax)
    v = u1 + 0.25 * t
    def quad_up(a, axis):  # Z1 -> Z2 along one axis, quadratic on each pair of Z1 cells
        a = np.moveaxis(a, axis, 0)
        m = a.shape[0]
        out = np.empty((2 * m - 1,) + a.shape[1:])
        out[::2] = a
        for c in range((m - 1) // 2):
            a0, a1, a2 = a[2 * c], a[2 * c + 1], a[2 * c + 2]
            out[4 * c + 1] = 0.375 * a0 + 0.75 * a1 - 0.125 * a2
            out[4 * c + 3] = -0.125 * a0 + 0.75 * a1 + 0.375 * a2
        return np.moveaxis(out, 0, axis)
    for ax in range(3):
        v = quad_up(v, ax)
    return v


@pytest.mark.parametrize("N", [4, 8, 16])
def test_exp_finite_equals_separable_form(N):
    rng = np.random.default_rng(N + 1)
    u1 = rng.standard_normal((N // 2 + 1,) * 3)
    u0 = rng.standard_normal((N // 4 + 1,) * 3)
    w = O.exp_finite(N, u1, u0)
    np.testing.assert_allclose(w, _separable_exp_finite(N, u1, u0), rtol=0, atol=1e-13)


@pytest.mark.parametrize("N", [2, 6, 8])
def test_exp_true_reduces_to_paper_1d_formulas(N):
    rng = np.random.default_rng(40 + N)
    uh = rng.standard_normal(N + 1)
    u2h = rng.standard_normal(N // 2 + 1)
    ut = O.exp_true(N, _nodes_1d(uh, N), _nodes_1d(u2h, N // 2))
    assert np.ptp(ut, axis=(0, 1)).max() <= 1e-13 * np.abs(ut).max()
    line = ut[0, 0, :]
    for j in range(N // 2):
        t1 = (4 * uh[2 * j] - u2h[j]) / 3
        chenlin = uh[2 * j + 1] + (uh[2 * j] - u2h[j] + uh[2 * j + 2] - u2h[j + 1]) / 6
        np.testing.assert_allclose(line[2 * j: 2 * j + 2], [t1, chenlin], rtol=0, atol=1e-14 * 8)


def test_exp_true_identity_and_trilinear_correction():
    """ut = uh + (1/3) * trilinear interpolation of (uh - u2h) over the coarse grid: with
    uh = u2h on coarse nodes nothing changes, and a trilinear difference is reproduced."""
    N = 8
    rng = np.random.default_rng(9)
    uh = rng.standard_normal((N + 1,) * 3)
    ut = O.exp_true(N, uh, uh[::2, ::2, ::2].copy())
    np.testing.assert_allclose(ut, uh, rtol=0, atol=1e-15)
    t = np.arange(N + 1) / N
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    lin = 1 + 2 * X - Y + 3 * X * Y * Z - Z * X
    u2h = uh[::2, ::2, ::2] - lin[::2, ::2, ::2]
    ut = O.exp_true(N, uh, u2h)
    np.testing.assert_allclose(ut, uh + lin / 3, rtol=0, atol=1e-14)
