"""Summarise rocprofv3 output of solver runs as Markdown tables.

    python -m paper_1901_05118_amd.trace_summary trace RESULTS.db --cmd "..."
    python -m paper_1901_05118_amd.trace_summary counters DIR --cmd "..."
    python -m paper_1901_05118_amd.trace_summary traffic --fetch DIR --write DIR \
        --copy-bytes BYTES --hash SOURCES --cmd "..."

``trace`` reads the SQLite database that ``rocprofv3 --kernel-trace`` writes (its
``kernels`` view) and prints the kernels by total time, then, for the Bi-CG sweeps, the
launches grouped by launch grid: the grid tells the levels apart, since every level of the
hierarchy runs the same kernels.  Inside a polling window a converged run issues launches
that return at once, and a sweep that stops a run may do only part of its work; a launch
counts as active (a full sweep) when it lasts at least half the longest launch of its
group, and the active mean is the per-launch cost of the sweep on that level.

``counters`` reads the ``*counter_collection.csv`` files of ``rocprofv3 --pmc ... -f csv``
below DIR and prints, per kernel and launch grid, the mean of each counter per dispatch.

``traffic`` turns a FETCH_SIZE pass and a WRITE_SIZE pass into HBM bytes per launch: each
counter is scaled by the factor that makes it read right on a plain copy kernel of known
size, and the result is stored, with a hash of the kernel sources it was measured on, in a
``traffic-record`` comment that the benchmark reads back (and ignores once the sources
differ).
"""
import argparse
import csv
import glob
import hashlib
import json
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
    act = [v for v in durations if v >= 0.5 * max(durations)]
    return len(durations), len(act), sum(act) / len(act), med


def trace(db_path: str, cmd: str, top: int = 24, sweeps: int = 8) -> str:
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
            "least half the group's longest launch (full sweeps).", "",
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
        # the three groups with the most active time: the levels that cost the most
        for mean, grid, c, na, med in sorted(stats, key=lambda t: -t[0] * t[3])[:3]:
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


def _counter_means(root: str):
    """{(kernel, grid size): {counter: mean per dispatch}} over the CSV files below root."""
    groups = {}
    for path in sorted(glob.glob(os.path.join(root, "**", "*counter_collection.csv"),
                                 recursive=True)):
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                key = (short_name(_col(row, "Kernel_Name")), int(float(_col(row, "Grid_Size"))))
                groups.setdefault(key, {}).setdefault(_col(row, "Counter_Name"), []).append(
                    float(_col(row, "Counter_Value")))
    return {k: {c: statistics.fmean(v) for c, v in d.items()} for k, d in groups.items()}


def sources_sha256(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(hashlib.sha256(fh.read()).digest())
    return h.hexdigest()


def traffic(fetch_dir: str, write_dir: str, copy_kernel: str, copy_bytes: float,
            hash_files, cmd: str, min_kib: float = 1024.0) -> str:
    """HBM bytes per dispatch from a FETCH_SIZE pass and a WRITE_SIZE pass, each calibrated
    by the same counter on a copy kernel that reads and writes ``copy_bytes`` bytes."""
    fetch, write = _counter_means(fetch_dir), _counter_means(write_dir)
    copy_f = [v["FETCH_SIZE"] for (k, _), v in fetch.items() if k == copy_kernel]
    copy_w = [v["WRITE_SIZE"] for (k, _), v in write.items() if k == copy_kernel]
    if not copy_f or not copy_w:
        raise SystemExit(f"copy kernel {copy_kernel!r} not found in both passes")
    ff = copy_bytes / (copy_f[0] * 1024.0)
    fw = copy_bytes / (copy_w[0] * 1024.0)
    out = [f"Command: `{cmd}`", "",
           f"Calibration on `{copy_kernel}` ({copy_bytes:.6g} bytes read and written): "
           f"FETCH_SIZE x {ff:.4f}, WRITE_SIZE x {fw:.4f}.", "",
           "| kernel | grid size | FETCH_SIZE KiB | WRITE_SIZE KiB | read bytes | written bytes "
           "| HBM bytes per launch |", "|---|---:|---:|---:|---:|---:|---:|"]
    record = {}
    for key in sorted(set(fetch) & set(write), key=lambda k: -fetch[k]["FETCH_SIZE"]):
        fk, wk = fetch[key]["FETCH_SIZE"], write[key]["WRITE_SIZE"]
        if fk + wk < min_kib:
            continue
        rb, wb = fk * 1024.0 * ff, wk * 1024.0 * fw
        record[f"{key[0]}|{key[1]}"] = rb + wb
        out.append(f"| `{key[0]}` | {key[1]} | {fk:.6g} | {wk:.6g} | {rb:.4g} | {wb:.4g} | "
                   f"{rb + wb:.4g} |")
    rec = {"factors": {"fetch": ff, "write": fw}, "sources": list(hash_files),
           "sources_sha256": sources_sha256(hash_files), "bytes_per_launch": record}
    out += ["", "<!-- traffic-record " + json.dumps(rec, sort_keys=True) + " -->"]
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("mode", choices=("trace", "counters", "traffic"))
    ap.add_argument("path", nargs="?", help="database (trace) or directory (counters)")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--fetch", help="traffic: directory of the FETCH_SIZE pass")
    ap.add_argument("--write", help="traffic: directory of the WRITE_SIZE pass")
    ap.add_argument("--copy-kernel", default="k_copy_convert<double, double>")
    ap.add_argument("--copy-bytes", type=float, help="traffic: bytes the copy reads (= writes)")
    ap.add_argument("--hash", default="", help="traffic: comma-separated kernel sources")
    args = ap.parse_args(argv)
    if args.mode == "trace":
        print(trace(args.path, args.cmd))
    elif args.mode == "counters":
        print(counters(args.path, args.cmd))
    else:
        files = [f for f in args.hash.split(",") if f]
        print(traffic(args.fetch, args.write, args.copy_kernel, args.copy_bytes, files, args.cmd))
    return 0


if __name__ == "__main__":
    sys.exit(main())
