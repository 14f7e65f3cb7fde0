"""The profile summariser on small synthetic rocprofv3 outputs (host logic only)."""
import csv
import json
import sqlite3

from paper_1901_05118_amd import trace_summary as ts


def test_trace_groups_by_grid_and_drops_noop_launches(tmp_path):
    db = tmp_path / "r.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, duration integer, grid_x integer, "
                "grid_y integer, grid_z integer)")
    name = "void excmg::zmarch<2, 8, float>(excmg::Geom, float const*)"
    rows = [(name, 1000, 512, 8, 1)] * 5 + [(name, 10, 512, 8, 1)] * 2 + [(name, 100, 64, 8, 1)] * 3
    con.executemany("insert into kernels values (?,?,?,?,?)", rows)
    con.commit()
    con.close()
    md = ts.trace(str(db), "cmd")
    assert "`zmarch<2, 8, float>`" in md
    assert "| `zmarch<2, 8, float>` | 10 | 0.01 |" in md
    # 7 launches on the big grid, 5 active at 1.0 us each
    assert "| 512x8x1 | 7 | 5 | 1.0 | 1.0 |" in md



def test_trace_active_means_full_sweeps_only(tmp_path):
    """Three populations on one grid: no-op launches, sweeps that stop a run after a partial
    pass, full sweeps; only the full ones are active, even when they are not the majority."""
    db = tmp_path / "r.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, duration integer, grid_x integer, "
                "grid_y integer, grid_z integer)")
    name = "void excmg::zmarch<2, 16, float>(excmg::Geom, float const*)"
    rows = ([(name, 20, 512, 16, 1)] * 40 + [(name, 560, 512, 16, 1)] * 12
            + [(name, 1720, 512, 16, 1)] * 45)
    con.executemany("insert into kernels values (?,?,?,?,?)", rows)
    con.commit()
    con.close()
    md = ts.trace(str(db), "cmd")
    assert "| 512x16x1 | 97 | 45 | 1.7 |" in md

def test_counters_mean_per_kernel_and_grid(tmp_path):
    d = tmp_path / "h" / "1"
    d.mkdir(parents=True)
    with open(d / "x_counter_collection.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writerow([1, 4096, "void excmg::k_copy<double>(long long)", "FETCH_SIZE", 100.0])
        w.writerow([2, 4096, "void excmg::k_copy<double>(long long)", "FETCH_SIZE", 300.0])
    md = ts.counters(str(tmp_path), "cmd")
    assert "| `k_copy<double>` | 4096 | FETCH_SIZE | 2 | 200 | 100 | 300 |" in md


def _pass(root, counter, rows):
    d = root / counter
    d.mkdir()
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for g, k, v in rows:
            w.writerow([g, k, counter, v])
    return str(d)


def test_traffic_calibrates_on_the_copy_and_records_a_source_hash(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("kernel")
    copy = "void excmg::k_copy_convert<double, double>(long long, double const*, double*)"
    sweep = "void excmg::zmarch<2, 16, float>(excmg::Geom)"
    # the copy moves 1 MiB each way; FETCH_SIZE reads half of that, WRITE_SIZE all of it
    f = _pass(tmp_path, "FETCH_SIZE", [(4096, copy, 512.0), (2048, sweep, 1000.0)])
    w = _pass(tmp_path, "WRITE_SIZE", [(4096, copy, 1024.0), (2048, sweep, 3000.0)])
    md = ts.traffic(f, w, "k_copy_convert<double, double>", 1024.0 * 1024.0, [str(src)], "cmd")
    assert "FETCH_SIZE x 2.0000, WRITE_SIZE x 1.0000" in md
    rec = json.loads(md.split("<!-- traffic-record ")[1].split(" -->")[0])
    assert rec["bytes_per_launch"]["zmarch<2, 16, float>|2048"] == (2000.0 + 3000.0) * 1024.0
    assert rec["sources_sha256"] == ts.sources_sha256([str(src)])
    src.write_text("changed")
    assert rec["sources_sha256"] != ts.sources_sha256([str(src)])
