"""Summarise rocprofv3 output of solver runs as Markdown tables.

    python -m paper_1901_05118_amd.trace_summary trace RESULTS.db --cmd "..."
    python -m paper_1901_05118_amd.trace_summary counters DIR --cmd "..."

``trace`` reads the SQLite database that ``rocprofv3 --kernel-trace`` writes (its
``kernels`` view) and prints the kernels by total time, then, for the Bi-CG sweeps, the
launches grouped by launch grid: the grid tells the levels apart, since every level of the
hierarchy runs the same kernels.  Inside a polling window a converged run issues launches
that return at once; a launch counts as active when it lasts at least half the median of
its group, and the active mean is the per-launch cost of the sweep on that level.

``counters`` reads the ``*counter_collection.csv`` files of ``rocprofv3 --pmc ... -f csv``
below DIR and prints, per kernel and launch grid, the mean of each counter per dispatch.
"""
import argparse
import csv
import glob
import os
import re
import sqlite3
import statistics
import sys


def short_name(n: str) -> str:
    n = re.sub(r"^void ", "", n)
    n = re.sub(r"\((excmg::|long long|int, |unsigned|double|float|const).*$", "", n)
    return n.replace("excmg::", "")


def _grid_rows(durations):
    med = statistics.median(durations)
    act = [v for v in durations if v >= 0.5 * med]
    return len(durations), len(act), sum(act) / len(act), med


def trace(db_path: str, cmd: str, top: int = 16, sweeps: int = 4) -> str:
    db = sqlite3.connect(db_path)
    cur = db.cursor()
    rows = cur.execute(
        "select name, count(*), sum(duration), avg(duration) from kernels group by name "
        "order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows)
    out = [f"Command: `{cmd}`", "",
           "| kernel | calls | total ms | avg us | share |", "|---|---:|---:|---:|---:|"]
    for n, c, s, a in rows[:top]:
        out.append(f"| `{short_name(n)}` | {c} | {s / 1e6:.2f} | {a / 1e3:.2f} | "
                   f"{100 * s / total:.1f}% |")
    out += ["", f"Total kernel time: {total / 1e6:.1f} ms", "",
            "Launches per grid (x*y*z threads) of the busiest kernels; 'active' = lasting at "
            "least half the group's median.", "",
            "| kernel | grid | calls | active | mean active us | median us |",
            "|---|---|---:|---:|---:|---:|"]
    for n, *_ in rows[:sweeps]:
        groups = cur.execute("select grid_x, grid_y, grid_z from kernels where name=? "
                             "group by grid_x, grid_y, grid_z", (n,)).fetchall()
        stats = []
        for gx, gy, gz in groups:
            d = [r[0] for r in cur.execute(
                "select duration from kernels where name=? and grid_x=? and grid_y=? and "
                "grid_z=?", (n, gx, gy, gz))]
            c, na, mean, med = _grid_rows(d)
            stats.append((mean, f"{gx}x{gy}x{gz}", c, na, med))
        for mean, grid, c, na, med in sorted(stats, reverse=True)[:3]:
            out.append(f"| `{short_name(n)}` | {grid} | {c} | {na} | {mean / 1e3:.1f} | "
                       f"{med / 1e3:.1f} |")
    return "\n".join(out)


def _col(row, *names):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(names)


def counters(root: str, cmd: str) -> str:
    files = sorted(glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no counter_collection.csv below {root}")
    groups = {}
    for path in files:
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                key = (short_name(_col(row, "Kernel_Name")), _col(row, "Grid_Size"),
                       _col(row, "Counter_Name"))
                groups.setdefault(key, []).append(float(_col(row, "Counter_Value")))
    out = [f"Command: `{cmd}`", "",
           "| kernel | grid size | counter | dispatches | mean per dispatch | min | max |",
           "|---|---:|---|---:|---:|---:|---:|"]
    for (k, g, c), v in sorted(groups.items(), key=lambda kv: -max(kv[1])):
        out.append(f"| `{k}` | {g} | {c} | {len(v)} | {statistics.fmean(v):.6g} | "
                   f"{min(v):.6g} | {max(v):.6g} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("mode", choices=("trace", "counters"))
    ap.add_argument("path")
    ap.add_argument("--cmd", default="")
    args = ap.parse_args(argv)
    print(trace(args.path, args.cmd) if args.mode == "trace" else counters(args.path, args.cmd))
    return 0


if __name__ == "__main__":
    sys.exit(main())
