"""Seeded manufactured solutions of the 2D biharmonic problem, eq. (bvp2d), on (0,1)^2.

Only closed-form functions: u, f = Delta^2 u and the boundary data.  Node arrays have shape
(N+1, N+1), indexed [j, i] (x fastest), x_i = i/N.  g1 holds u on boundary nodes; g2 holds
on the four edges the outward normal derivative (first kind) or the second normal
derivative (second kind); interior nodes of both are 0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Arrays2D:
    N: int
    bc: int
    f: np.ndarray
    g1: np.ndarray
    g2: np.ndarray
    u: np.ndarray


class Family2D:
    """u = exp(a x + b y) + sum_m A_m sin(k_m pi x) sin(l_m pi y), evaluated exactly."""

    def __init__(self, ab, modes, name="family2d"):
        self.ab = ab            # (a, b) or None for no exponential
        self.modes = modes      # [(A, k, l)]
        self.name = name

    def _parts(self, X, Y):
        """u, u_x, u_y, u_xx, u_yy, Delta^2 u on the meshgrid (X, Y)."""
        u = np.zeros_like(X)
        ux, uy, uxx, uyy, bih = (np.zeros_like(X) for _ in range(5))
        if self.ab is not None:
            a, b = self.ab
            e = np.exp(a * X + b * Y)
            u += e
            ux += a * e
            uy += b * e
            uxx += a * a * e
            uyy += b * b * e
            bih += (a * a + b * b) ** 2 * e
        for A, k, l in self.modes:
            kx, ly = k * np.pi, l * np.pi
            sx, cx = np.sin(kx * X), np.cos(kx * X)
            sy, cy = np.sin(ly * Y), np.cos(ly * Y)
            u += A * sx * sy
            ux += A * kx * cx * sy
            uy += A * ly * sx * cy
            uxx += -A * kx * kx * sx * sy
            uyy += -A * ly * ly * sx * sy
            bih += A * (kx * kx + ly * ly) ** 2 * sx * sy
        return u, ux, uy, uxx, uyy, bih


def family_2d(seed: int, n_modes: int = 4, kmax: int = 4) -> Family2D:
    """a, b ~ U(-1, 1); wave numbers uniform on 1..kmax; amplitudes ~ N(0, 1); drawn in this
    order from numpy.random.default_rng(seed)."""
    rng = np.random.default_rng(seed)
    ab = tuple(rng.uniform(-1.0, 1.0, size=2))
    ks = rng.integers(1, kmax + 1, size=(n_modes, 2))
    amps = rng.standard_normal(n_modes)
    return Family2D(ab, [(amps[m], ks[m, 0], ks[m, 1]) for m in range(n_modes)])


def sine_2d() -> Family2D:
    """u = sin(pi x) sin(pi y), Delta^2 u = 4 pi^4 u."""
    return Family2D(None, [(1.0, 1, 1)], name="sine2d")


def make_arrays_2d(problem: Family2D, N: int, bc: int) -> Arrays2D:
    if bc not in (1, 2):
        raise ValueError("bc must be 1 or 2")
    x = np.arange(N + 1, dtype=np.float64) / N
    X, Y = np.meshgrid(x, x)          # [j, i]
    u, ux, uy, uxx, uyy, bih = problem._parts(X, Y)
    g1 = np.zeros_like(u)
    g2 = np.zeros_like(u)
    edges = [(np.s_[:, 0], -ux, uxx), (np.s_[:, N], ux, uxx),
             (np.s_[0, :], -uy, uyy), (np.s_[N, :], uy, uyy)]
    for sl, dn, dnn in edges:
        g1[sl] = u[sl]
        g2[sl] = dn[sl] if bc == 1 else dnn[sl]
    return Arrays2D(N=N, bc=bc, f=bih, g1=g1, g2=g2, u=u)
