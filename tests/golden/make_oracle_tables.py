"""Write ``oracle_tables.json``: the accuracy columns of the paper's Tables 1-5 (Sec. 6)
computed by the oracle on the 32^3, 64^3 and 128^3 grids, for the GPU table test.

The GPU test runs each problem as one cascade to 512^3 cells (first kind, direct solves on
8^3 and 16^3, seven levels) with the finest-level tolerance ``tol``; its levels up to 128^3
are exactly the oracle's five-level cascade to 128^3 with tolerance tol / 100 (Algorithm 1
tightens the tolerance tenfold per coarser level), so their rows must agree with the
values stored here.  Tolerances: Problem 1 has zero boundary data and a relative-residual
floor that grows about thirty-fold per level (4e-12 at 32^3 to 6e-7 at 256^3), so its
cascade uses 1e-4 on the finest grid, which keeps every level's tolerance above its floor;
Problem 5's steep exponential makes Bi-CG converge slowly (some 33000 iterations on 256^3
at 1e-9), so its cascade uses 1e-6; Problems 2-4 use 1e-9.  Calls only the oracle.

    python tests/golden/make_oracle_tables.py      # about fifteen minutes on eight cores
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from manufactured import make_arrays, paper_problem  # noqa: E402

FINEST_TOL = {1: 1e-4, 2: 1e-9, 3: 1e-9, 4: 1e-9, 5: 1e-6}
N_REF, LEVELS_REF = 128, 5          # 8, 16 direct; 32, 64, 128 Bi-CG
N_GPU, LEVELS_GPU = 512, 7


def rows(k):
    tol = FINEST_TOL[k] / 100.0     # the 128^3 level's tolerance in the 512^3 cascade
    arr = make_arrays(paper_problem(k), N_REF, 1)
    t0 = time.perf_counter()
    res = O.excmg(N_REF, LEVELS_REF, 1, arr.f, arr.g1, arr.g2, tol, keep_levels=True)
    out = []
    for l in range(2, LEVELS_REF):
        n = N_REF >> (LEVELS_REF - 1 - l)
        s = N_REF // n
        u = res.u_levels[l]
        e = u - arr.u[::s, ::s, ::s]
        st = res.levels[l - 2]
        out.append({"n": n, "err2": O.norm2(e), "errinf": O.norminf(e),
                    "w_err2": O.norm2(res.w_levels[l] - u), "iterations": st.iters,
                    "runs": st.runs, "code": st.code,
                    "rel_residual": (st.rr_true / st.bb) ** 0.5})
    print(f"problem {k}: {time.perf_counter() - t0:.0f} s", out, flush=True)
    return out


def main():
    data = {"source": "the oracle (oracle/), Algorithm 1 with first-kind data of the paper's "
                      "Problems 1-5 (Sec. 6), direct solves on 8^3 and 16^3; written by "
                      "tests/golden/make_oracle_tables.py",
            "cascade": {"n_finest": N_GPU, "n_levels": LEVELS_GPU, "bc_kind": 1},
            "finest_tol": {str(k): v for k, v in FINEST_TOL.items()},
            "rows": {str(k): rows(k) for k in sorted(FINEST_TOL)}}
    with open(os.path.join(HERE, "oracle_tables.json"), "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
