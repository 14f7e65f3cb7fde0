"""Seeded manufactured-solution inputs for the 3D biharmonic problem on (0,1)^3.

This module only evaluates closed-form functions: the exact solution u, the forcing
f = Delta^2 u and the boundary data.  It contains none of the solver's arithmetic, and both
the GPU library and the CPU oracle receive the arrays it produces.

Array conventions (shared with the library's C ABI):
  * node arrays have shape (N+1, N+1, N+1), indexed [k, j, i] so that x is fastest, with
    x_i = i/N;
  * ``g1`` holds u on the boundary nodes (interior nodes are 0, or NaN with ``poison``);
  * ``g2`` holds, on the six faces, the outward normal derivative du/dn (first kind) or the
    second normal derivative d2u/dn2 (second kind); interior nodes are 0 (NaN with
    ``poison``).  Only face-interior nodes of g2 are meaningful to the solver.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .problems import (Problem, SeparableFamily, SympyProblem, paper_problem, config_problem,
                       batch_problems, BatchItem, polynomial_problem)

__all__ = ["Problem", "SeparableFamily", "SympyProblem", "paper_problem", "config_problem",
           "batch_problems", "BatchItem", "polynomial_problem", "Arrays", "make_arrays",
           "CONFIGS"]


@dataclass
class Arrays:
    N: int
    bc: int
    f: np.ndarray
    g1: np.ndarray
    g2: np.ndarray
    u: np.ndarray | None  # exact solution at all nodes (if requested)


def make_arrays(problem: Problem, N: int, bc: int, *, with_u: bool = True,
                poison: bool = False) -> Arrays:
    """Node arrays f, g1, g2 (and the exact u) of ``problem`` on the grid with N cells."""
    if bc not in (1, 2):
        raise ValueError("bc must be 1 (u, du/dn given) or 2 (u, d2u/dn2 given)")
    M = N + 1
    x = np.arange(M, dtype=np.float64) / N
    f = problem.f_grid(x)
    u = problem.u_grid(x) if with_u else None
    fill = np.nan if poison else 0.0
    g1 = np.full((M, M, M), fill)
    g2 = np.full((M, M, M), fill)
    # faces: axis 0 is z, 1 is y, 2 is x
    for axis in range(3):
        for side in (0, N):
            val = problem.u_face(x, axis, side)
            d = problem.normal_data(x, axis, side, bc)
            sl = [slice(None)] * 3
            sl[axis] = side
            g1[tuple(sl)] = val
            g2[tuple(sl)] = d
    return Arrays(N=N, bc=bc, f=f, g1=g1, g2=g2, u=u)


# The five benchmark configurations: (finest N, n_levels, bc, tolerance, problem factory,
# precision mode).  Config 1's forcing is the true Delta^2 of sin(pi x) sin(pi y) sin(pi z),
# which is 9 pi^4 u.
CONFIGS = {
    1: dict(N=32, n_levels=4, bc=1, tol=1e-10, mode="fp64"),
    2: dict(N=128, n_levels=6, bc=2, tol=1e-10, mode="fp64"),
    3: dict(N=256, n_levels=7, bc=1, tol=1e-8, mode="mixed"),
    4: dict(N=512, n_levels=8, bc=2, tol=1e-8, mode="mixed"),
}
