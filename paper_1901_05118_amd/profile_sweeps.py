"""Launch single Bi-CG sweeps on the finest level, for profiler and hardware-counter runs.

    python -m paper_1901_05118_amd.profile_sweeps --n 512 --levels 8 --bc 2 \\
        --precision mixed --sweeps 2,3 --reps 5

sets up the level hierarchy, then launches each listed sweep ``reps`` times (after one
warm-up launch) through ``excmg_profile_sweep``, followed by the same number of plain FP64
copies of one finest-level vector: a kernel of known traffic (16 bytes per unknown) against
which HBM byte counters are calibrated.  Sweeps: 0 operator apply, 1 residual, 2 sweep A
(direction update and the pair of operator products), 3 sweep B (x, r, r* updates with the
next rho), 4 copy, 5 sweep A applying the previous iteration's x update and 6 the sweep B
that then leaves x alone (the stored form's pair on grids from 64^3 to 128^3), 7 and 8 the
two sweeps of the recomputing form (mixed-precision solves on grids of 2^22 unknowns and
up: sweep A marches p alone; sweep B marches p and p* again for q and q* and updates x, r,
r*).  Prints one line per sweep: mean ms per launch, algorithmic bytes per launch and the
rate.  Uses no torch: every launch comes from the library.
"""
import argparse
import sys

from . import excmg as ex


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--levels", type=int, default=8)
    ap.add_argument("--bc", type=int, default=2)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="mixed")
    ap.add_argument("--sweeps", default="2,3")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--ty", type=int, default=0, help="tile rows of sweep A (0: library default)")
    ap.add_argument("--zc", type=int, default=0, help="planes per tile of sweep A")
    ap.add_argument("--no-calibrate", action="store_true")
    args = ap.parse_args(argv)
    prec = ex.MIXED if args.precision == "mixed" else ex.FP64
    sweep_a_kind = 2 if prec == ex.MIXED else 1
    if args.ty:
        ex.set_shape(args.n, sweep_a_kind, args.ty, args.zc)
    ex.setup(args.n, args.levels, args.bc)
    ty, zc = ex.get_shape(args.n, sweep_a_kind)
    print(f"n={args.n} bc={args.bc} precision={args.precision} sweep A tile 64x{ty}, "
          f"{zc} planes per tile", flush=True)
    runs = [(int(s), prec) for s in args.sweeps.split(",") if s.strip()]
    if not args.no_calibrate:
        runs.append((4, ex.FP64))
    for which, p in runs:
        ms, nb = ex.profile_sweep(which, p, args.reps)
        print(f"sweep {which} {'fp64' if p == ex.FP64 else 'mixed'}: {args.reps} launches, "
              f"{ms:.4f} ms/launch, {nb:.6g} bytes/launch, {nb / (ms * 1e-3) / 1e9:.1f} GB/s",
              flush=True)
    ex.finalize()
    return 0


if __name__ == "__main__":
    sys.exit(main())
