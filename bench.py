"""Benchmark of the EXCMG hot path on one MI355X.

One step = one complete EXCMG solve (Algorithm 1: right-hand sides, direct coarse solves,
EXP_finite guesses, Bi-CG on every level, EXP_true) of the 512^3-cell second-kind
manufactured problem (8 seeded sine modes plus an exponential) to the relative residual
1e-8, with the inputs already in HBM.  Prints one JSON line.

Both precisions are timed: plain FP64, and FP32 Bi-CG inside FP64 iterative refinement
(by residual replacement, the library's default; the restarted form is timed alongside).
The headline step is the mixed solve when its discretisation error is within 1% of the FP64
solve's (the accuracy gate), otherwise the FP64 solve.
value = Bi-CG GLUPS of the whole job: sum over levels of (unknowns x Bi-CG iterations)
divided by the wall time of the solve.  The line also carries the time to the 1e-8
residual, the roofline position of the dominant kernel (measured with device events on the
library's stream) and the CPU oracle's throughput on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Bi-CG stencil GLUPS & HBM GB/s; time-to-1e-8 residual, FP64 vs mixed"
HBM_PEAK_GBS = 8000.0
# sources that define the z-marched stencil kernels: a stored counter measurement of sweep A
# holds only while these are unchanged
SWEEP_A_SOURCES = ["paper_1901_05118_amd/csrc/common.hpp",
                   "paper_1901_05118_amd/csrc/step.hpp",
                   "paper_1901_05118_amd/csrc/zmarch.hpp",
                   "paper_1901_05118_amd/csrc/stencil.hip"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Grids from which Bi-CG takes the recomputing form, and from which mixed solves use FP32
# vectors (the library's defaults)
RECOMPUTE_MIN = 1 << 22      # FP32 vectors
RECOMPUTE_MIN64 = 1 << 20    # FP64 vectors
FP32_MIN = 1 << 18
DOWN_MAX = 1 << 26


def update_depth(ty):
    """Planes in flight of the recomputing form's update sweep (the library's choice)."""
    return 2 if ty >= 16 else 3


def update_blocks(nu):
    """Workgroups of the streaming Bi-CG update kernels (the library's choice)."""
    b = -(-nu // (512 * 4)) if nu > (1 << 18) else -(-nu // 512)
    return max(1, min(b, 1024))


def sweep_launch(N, ty, zc, form):
    """Name (as the profiler shows it) and launch size in threads of a Bi-CG sweep on the
    grid of N cells with stencil tiles of 64 x ty columns and zc planes.  form: "sigma" /
    "update" (the two sweeps of the recomputing form, FP32 vectors; "update_keep" /
    "update_pair" its sweep B leaving x or applying two iterations' updates), "sigma64" /
    "update64" / "update_keep64" / "update_pair64" (the same with FP64 vectors), "fp64" / "stored32" (sweep A of the stored form), "deferred"
    (FP32 sweep A that also applies the previous iteration's x update), "update_stored64" /
    "update32" (the stored form's streaming sweep B)."""
    n = N - 1
    if form in ("update32", "update_stored64"):
        t = "float" if form == "update32" else "double"
        return f"k_bicg_update<double, {t}, false>", update_blocks(n ** 3) * 512
    tiles = -(-n // 64) * -(-n // ty) * -(-n // zc)
    tiles = -(-tiles // 8) * 8  # the grid is padded to whole XCD shares
    d = update_depth(ty)
    # FP32 sweeps A, and FP64 sweeps B below 2^26 unknowns, march downwards (the library's
    # choice)
    kern = "zmarch_down" if form == "sigma" or (
        form in ("update64", "update_keep64", "update_pair64") and n ** 3 < DOWN_MAX) \
        else "zmarch"
    # the last template argument: planes in flight
    name = {"fp64": "zmarch<2, {ty}, double, InDirection<double>, OutPairApply<double>, 2>",
            "stored32": "zmarch<2, {ty}, float, InDirection<float>, OutPairApply<float>, 2>",
            "deferred": "zmarch<2, {ty}, float, InDirection<float>, OutPairApplyX<float>, 2>",
            "sigma": "zmarch<1, {ty}, float, InDirection<float>, OutDirSigma<float>, 3>",
            "update": "zmarch<2, {ty}, float, InPlainAlpha<float>, OutPairUpdate<float, 0>, {d}>",
            "update_keep": "zmarch<2, {ty}, float, InPlainAlpha<float>, OutPairUpdate<float, 1>, {d}>",
            "update_pair": "zmarch<2, {ty}, float, InPlainAlpha<float>, OutPairUpdate2<float>, {d}>",
            "sigma64": "zmarch<1, {ty}, double, InDirection<double>, OutDirSigma<double>, 3>",
            "update64": "zmarch<2, {ty}, double, InPlainAlpha<double>, OutPairUpdate<double, 0>, {d}>",
            "update_keep64": "zmarch<2, {ty}, double, InPlainAlpha<double>, OutPairUpdate<double, 1>, {d}>",
            "update_pair64": "zmarch<2, {ty}, double, InPlainAlpha<double>, OutPairUpdate2<double>, {d}>"}[form]
    return kern + name.format(ty=ty, d=d)[len("zmarch"):], tiles * 64 * ty


class _Forms(dict):
    fp32 = False


def sweep_forms(N, mixed):
    """The Bi-CG sweeps a solve runs on the level of N cells, as {timing kind: (kernel form,
    algorithmic bytes per unknown, label)}; timing kinds as excmg_get_timing's (0 sweep A,
    1 sweep B, 2 sweep A applying the deferred iterate update, 3 and 4 the recomputing
    form's sweeps B of odd and even iterations).  Mixed solves run FP32 vectors from 2^18
    unknowns up (smaller levels FP64); the recomputing form is taken from 2^22 unknowns up
    with FP32 vectors and from 2^20 with FP64 ones.  Bytes: recomputing form, sweep A reads r, p, r*, p* and writes p, p* (FP32
    24, FP64 48), sweep B reads p, p*, r, r* and writes r, r* (FP32 24, FP64 48) and updates
    the FP64 iterate once per two iterations: an odd iteration's sweep B leaves it, an even
    one's reads x and the previous p and writes x (FP32 44, FP64 72); the first sweep B of a
    run at an even iteration updates x once (FP32 40, FP64 64); stored form, FP64: sweep A reads r, r*,
    p, p* and writes p, p*, q, q* (64), sweep B reads x, p, r, q, r*, q* and writes x, r, r*
    (72); stored form with FP32 vectors: sweep A 32 (48 when it also applies the previous
    iteration's x += alpha p), sweep B streams r, q, r*, q* and writes r, r* (24)."""
    nu = (N - 1) ** 3
    f = _Forms()
    f.fp32 = mixed and nu >= FP32_MIN
    if nu >= (RECOMPUTE_MIN if f.fp32 else RECOMPUTE_MIN64):
        if f.fp32:
            f.update({0: ("sigma", 24.0, "A; even iterations launch its OutDirSigmaX variant"),
                      1: ("update", 40.0, "B"),
                      3: ("update_keep", 24.0, "B, x left"), 4: ("update_pair", 44.0, "B, x twice")})
        else:
            f.update({0: ("sigma64", 48.0, "A; even iterations launch its OutDirSigmaX variant"),
                      1: ("update64", 64.0, "B"),
                      3: ("update_keep64", 48.0, "B, x left"),
                      4: ("update_pair64", 72.0, "B, x twice")})
    elif f.fp32:
        f.update({0: ("stored32", 32.0, "A"), 2: ("deferred", 48.0, "A+x"),
                  1: ("update32", 24.0, "B")})
    else:
        f.update({0: ("fp64", 64.0, "A"), 1: ("update_stored64", 72.0, "B")})
    return f


def recorded_traffic(kernel, grid):
    """HBM bytes per launch of (kernel, grid) from the traffic records of the committed
    counter summaries, provided they were measured on the current kernel sources."""
    import glob
    import re
    from paper_1901_05118_amd.trace_summary import sources_sha256
    key = f"{kernel}|{grid}"
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            text = fh.read()
        for m in re.finditer(r"<!-- traffic-record (\{.*?\}) -->", text):
            rec = json.loads(m.group(1))
            if key not in rec["bytes_per_launch"]:
                continue
            files = [os.path.join(ROOT, f) for f in rec["sources"]]
            if sorted(rec["sources"]) != sorted(SWEEP_A_SOURCES):
                continue
            if all(os.path.exists(f) for f in files) and \
                    sources_sha256(files) == rec["sources_sha256"]:
                return rec["bytes_per_launch"][key], os.path.basename(path)
    return None, None


def cpu_model():
    """CPU model, physical cores and threads per core of this host (lscpu)."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        phys = int(info["Core(s) per socket"]) * int(info["Socket(s)"])
    except (KeyError, ValueError):
        phys = None
    return info.get("Model name"), phys, info.get("Thread(s) per core")


# FP64 Bi-CG iteration in the algorithmic-bytes convention of the GPU sweeps, with the x update
# in every iteration as the oracle makes it (recomputing form: sweep A 48 + sweep B 64 bytes
# per unknown; the GPU's paired updates move 106)
FP64_ITERATION_BYTES = 112.0


def cpu_baseline(arr, N, nl, bc, iters, cfg_sols):
    """The oracle (plain FP64 C with OpenMP, never tuned for speed) on the host cores:
    (a) Bi-CG iterations on the finest level of the headline problem, median of 3 runs;
    (b) the same on a 128^3 level with one thread, median of 3; (c) its time to solution of
    configurations 1 (32^3, median of 3) and 2 (128^3, one run), with the max-norm
    distance of the GPU's FP64 and mixed solutions of the same inputs to its solution."""
    import statistics

    import numpy as np
    import oracle
    from manufactured import config_problem, make_arrays

    model, phys, tpc = cpu_model()
    threads = oracle.threads()

    def bicg_rate(Nl, bcl, b, its):
        x0 = np.zeros((Nl - 1) ** 3)
        t0 = time.perf_counter()
        _, it, _, _ = oracle.bicg(Nl, bcl, b, x0, 1e-30, maxit=its)
        dt = time.perf_counter() - t0
        return (Nl - 1) ** 3 * it / dt / 1e9, it, dt

    b = oracle.rhs(N, bc, arr.f, arr.g1, arr.g2)
    runs = [bicg_rate(N, bc, b, iters) for _ in range(3)]
    glups = statistics.median(r[0] for r in runs)
    it_done = runs[0][1]
    t_each = statistics.median(r[2] for r in runs)
    del b
    # one thread, 128^3 level of configuration 2
    arr2 = make_arrays(config_problem(2), 128, 2)
    b2 = oracle.rhs(128, 2, arr2.f, arr2.g1, arr2.g2)
    oracle.set_threads(1)
    try:
        one = [bicg_rate(128, 2, b2, 3) for _ in range(3)]
    finally:
        oracle.set_threads(threads)
    glups1 = statistics.median(r[0] for r in one)
    # time to solution of configurations 1 and 2
    tts = {}
    for c, Nc, nlc, bcc, tol, reps in ((1, 32, 4, 1, 1e-10, 3), (2, 128, 6, 2, 1e-10, 1)):
        a = make_arrays(config_problem(c), Nc, bcc)
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            ref = oracle.excmg(Nc, nlc, bcc, a.f, a.g1, a.g2, tol)
            times.append(time.perf_counter() - t0)
        ms = statistics.median(times) * 1e3
        lups = sum((lv.N - 1) ** 3 * lv.iters for lv in ref.levels)
        entry = {"ms": round(ms, 1), "runs": reps, "glups": round(lups / (ms * 1e-3) / 1e9, 4),
                 "iterations": [lv.iters for lv in ref.levels]}
        for name, ug in cfg_sols.get(c, {}).items():
            entry[f"gpu_{name}_max_dist"] = float(np.abs(ug - ref.u.reshape(ug.shape)).max())
        tts[f"config{c}"] = entry
        log(f"oracle config {c}: {entry}")
    return {"value": glups, "unit": "GLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{it_done} Bi-CG iterations (plus the initial residual) of the oracle on "
                      f"the {N}^3-cell finest level of the same problem, median of 3 runs of "
                      f"{t_each:.1f} s on {threads} OpenMP threads",
            "gbs": round(glups * FP64_ITERATION_BYTES, 2),
            "gbs_convention": "FP64 Bi-CG iteration, 112 algorithmic bytes per unknown",
            "cpu_model": model, "physical_cores": phys, "threads_per_core": tpc,
            "one_thread_128": {"value": glups1, "unit": "GLUPS",
                               "gbs": round(glups1 * FP64_ITERATION_BYTES, 3),
                               "sample": "3 Bi-CG iterations on the 128^3 level of "
                                         "configuration 2, median of 3 runs, 1 thread"},
            "time_to_solution": tts}


def plane_leg(ex, torch, np, steps):
    """The 2D equation (eq. bvp2d) through the same pipeline: 4096^2 cells over 8 levels
    (direct levels of 32^2 and 64^2 cells), second kind, seeded exponential-plus-sines
    solution, tol 1e-8, FP64 and mixed."""
    from manufactured.twod import family_2d, make_arrays_2d
    N, nl, bc = 4096, 8, 2
    arr = make_arrays_2d(family_2d(7), N, bc)
    f, g1, g2 = (torch.from_numpy(a).cuda() for a in (arr.f, arr.g1, arr.g2))
    u = torch.empty_like(f)
    res = {"workload": f"2D EXCMG {N}^2 cells, bc kind {bc}, tol 1e-8", "n_finest": N,
           "n_levels": nl}
    for prec, name in ((ex.FP64, "fp64"), (ex.MIXED, "mixed")):
        ex.solve_ex_2d(N, nl, bc, f, g1, g2, 1e-8, u, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rc, st = ex.solve_ex_2d(N, nl, bc, f, g1, g2, 1e-8, u, precision=prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        if rc != ex.OK:
            raise RuntimeError(f"2D solve failed: {rc} {ex.last_error()}")
        lv = st.levels()
        lups = sum(((l["n"] - 1) ** 2) * l["iterations"] for l in lv)
        e = u.cpu().numpy() - arr.u
        res[name] = {"ms": round(ms, 2), "glups": round(lups / (ms * 1e-3) / 1e9, 3),
                     "iterations": [l["iterations"] for l in lv],
                     "u_rms_error": float(np.sqrt(np.mean(e * e)))}
        log(f"2d {name}: {res[name]}")
    return res


def configs_leg(ex, torch, np, steps, kept):
    """The smaller configurations of the same family: 32^3 cells, first kind, FP64 to 1e-10
    (4 levels); 128^3, second kind, to 1e-10 (6 levels); 256^3, first kind, to 1e-8 (7
    levels); each in FP64 and mixed precision.  Time to solution, Bi-CG GLUPS, the max-norm error against the
    exact solution and, for the mixed solve, against the FP64 one.  The solutions of
    configurations 1 and 2 are kept in `kept` for the comparison with the oracle."""
    from manufactured import config_problem, make_arrays
    res = {}
    for c, N, nl, bc, tol, precs in ((1, 32, 4, 1, 1e-10, ("fp64", "mixed")),
                                      (2, 128, 6, 2, 1e-10, ("fp64", "mixed")),
                                      (3, 256, 7, 1, 1e-8, ("fp64", "mixed"))):
        arr = make_arrays(config_problem(c), N, bc)
        f, g1, g2 = (torch.from_numpy(a).cuda() for a in (arr.f, arr.g1, arr.g2))
        u = torch.empty_like(f)
        entry = {"workload": f"EXCMG {N}^3 cells, bc kind {bc}, seeded family {c}, tol {tol:g}"}
        sols = {}
        for name in precs:
            prec = ex.FP64 if name == "fp64" else ex.MIXED
            ex.solve_ex(N, nl, bc, f, g1, g2, tol, u, precision=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, tol, u, precision=prec)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            if rc != ex.OK:
                raise RuntimeError(f"config {c} {name} solve failed: {rc} {ex.last_error()}")
            lv = st.levels()
            lups = sum(((l["n"] - 1) ** 3) * l["iterations"] for l in lv)
            ug = u.view(N + 1, N + 1, N + 1).cpu().numpy()
            sols[name] = ug
            entry[name] = {"ms": round(ms, 2), "glups": round(lups / (ms * 1e-3) / 1e9, 3),
                           "iterations": [l["iterations"] for l in lv],
                           "max_err_vs_exact": float(np.abs(ug - arr.u).max())}
        if "mixed" in sols:
            entry["mixed_vs_fp64_max"] = float(np.abs(sols["mixed"] - sols["fp64"]).max())
            entry["speedup_mixed"] = round(entry["fp64"]["ms"] / entry["mixed"]["ms"], 3)
        log(f"config {c}: {entry}")
        res[f"config{c}"] = entry
        if c in (1, 2):
            kept[c] = sols
        del f, g1, g2, u
    return res


def jacobi_leg(ex, torch, np, N, nl, bc, tol, f, g1, g2, u, steps):
    """Algorithm 2 with the Jacobi preconditioner M = diag(A_h) on the same 3D workload."""
    ex.solve_ex(N, nl, bc, f, g1, g2, tol, u, precond=ex.PRECOND_JACOBI)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, tol, u, precond=ex.PRECOND_JACOBI)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    if rc != ex.OK:
        raise RuntimeError(f"Jacobi solve failed: {rc} {ex.last_error()}")
    res = {"ms": round(ms, 2), "iterations": [l["iterations"] for l in st.levels()],
           "runs": [l["runs"] for l in st.levels()]}
    log(f"jacobi fp64: {res}")
    return res


def batch_leg(ex, torch, np):
    """64 independent problems of 32^3..128^3 cells (mixed boundary kinds), tol 1e-8:
    batched (both forms: four graph-captured phase launches per Bi-CG step, and one
    persistent work-queue launch per step) against one solve after another, FP64 and mixed
    precision."""
    from manufactured import batch_problems, make_arrays
    items = batch_problems(64)
    dev = torch.device("cuda:0")
    data = []
    for it in items:
        arr = make_arrays(it.problem, it.N, it.bc, with_u=False)
        f, g1, g2 = (torch.from_numpy(a).to(dev) for a in (arr.f, arr.g1, arr.g2))
        data.append((it, f, g1, g2, torch.empty_like(f)))
    res = {"problems": len(items), "unknowns": int(sum((it.N - 1) ** 3 for it in items))}
    for prec, name in ((ex.FP64, "fp64"), (ex.MIXED, "mixed")):
        def seq():
            for (it, f, g1, g2, u) in data:
                rc, _ = ex.solve_ex(it.N, it.n_levels, it.bc, f, g1, g2, 1e-8, u, precision=prec)
                if rc != ex.OK:
                    raise RuntimeError(ex.last_error())
        probs = [dict(n_finest=it.N, n_levels=it.n_levels, bc_kind=it.bc, f=f, g1=g1, g2=g2,
                      u_out=u) for (it, f, g1, g2, u) in data]
        # the batched sweep A's shapes, tuned on this batch's own work list
        t0 = time.perf_counter()
        ty, ms_step = ex.autotune_batch(probs, precision=prec, reps=3)
        tune_s = time.perf_counter() - t0
        # a mixed batch runs FP32 Bi-CG on grids of at least 2^18 unknowns, FP64 below
        shapes = {int(N): list(ex.get_batch_shape(
                      int(N), prec if (N - 1) ** 3 >= (1 << 18) else ex.FP64))
                  for N in sorted({it.N for it in items})}
        log(f"batch {name}: tuned tile height {ty}, shapes {shapes}, {ms_step:.3f} ms per step of "
            f"each size alone, summed "
            f"({tune_s:.1f} s)")

        def bat(persistent):
            rc, _ = ex.solve_batch(probs, 1e-8, precision=prec, persistent=persistent)
            if rc != ex.OK:
                raise RuntimeError(ex.last_error())
        times = {}
        for label, fn in (("sequential", seq), ("batched", lambda: bat(False)),
                          ("batched_persistent", lambda: bat(True))):
            fn()  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            times[label] = (time.perf_counter() - t0) * 1e3
        log(f"batch {name}: {times}")
        res[name] = {"tuned_shapes": {"tile_rows": ty, "ty_zc_per_grid": shapes,
                                      "ms_per_step_sum_over_sizes": round(ms_step, 4),
                                      "tuning_s": round(tune_s, 1)},
                     "sequential_ms": round(times["sequential"], 1),
                     "batched_ms": round(times["batched"], 1),
                     "batched_persistent_ms": round(times["batched_persistent"], 1),
                     "speedup": round(times["sequential"] / times["batched"], 2),
                     "speedup_persistent": round(times["sequential"] /
                                                 times["batched_persistent"], 2)}
    return res


def profile_sweeps(ex, args):
    """Launch single solver sweeps for profiler and hardware-counter runs (see --help)."""
    prec = ex.MIXED if args.precision == "mixed" else ex.FP64
    ex.setup(args.n, args.levels, args.bc)
    ty, zc = ex.get_shape(args.n, 2 if prec == ex.MIXED else 1)
    print(f"n={args.n} bc={args.bc} precision={args.precision} sweep A tile 64x{ty}, "
          f"{zc} planes per tile", flush=True)
    runs = [(int(w), prec) for w in args.profile_sweeps.split(",") if w.strip()]
    runs.append((4, ex.FP64))   # the copy of known traffic
    for which, p in runs:
        ms, nb = ex.profile_sweep(which, p, args.reps)
        print(f"sweep {which} {'fp64' if p == ex.FP64 else 'mixed'}: {args.reps} launches, "
              f"{ms:.4f} ms/launch, {nb:.6g} bytes/launch, {nb / (ms * 1e-3) / 1e9:.1f} GB/s",
              flush=True)
    ex.finalize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="finest grid (cells per axis)")
    ap.add_argument("--levels", type=int, default=8)
    ap.add_argument("--bc", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--config", type=int, default=4, help="seeded problem family (1-4)")
    ap.add_argument("--cpu-iters", type=int, default=2,
                    help="oracle Bi-CG iterations per timed run on the finest level")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batch leg")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D (4096^2) leg")
    ap.add_argument("--no-jacobi", action="store_true", help="skip the Jacobi-preconditioned leg")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the smaller configurations (32^3, 128^3, 256^3)")
    ap.add_argument("--only-2d", action="store_true",
                    help="run the 2D (4096^2) leg alone (for profiling it); its line reports "
                         "the 2D mixed solve")
    ap.add_argument("--autotune", action="store_true",
                    help="re-time every tile shape first instead of the built-in tuned table")
    ap.add_argument("--profile-sweeps", default="",
                    help="only launch the listed solver sweeps (excmg_profile_sweep numbers, "
                         "e.g. 7,8) on the finest level of --n/--levels/--bc, --reps times "
                         "each after one warm-up launch, then as many FP64 copies of one "
                         "finest-level vector (the calibration kernel of the HBM byte "
                         "counters); for profiler and counter runs; prints one line per sweep")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="mixed",
                    help="vectors of the --profile-sweeps launches")
    ap.add_argument("--reps", type=int, default=5, help="launches per sweep (--profile-sweeps)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path (one "
              "problem would shard into z-slabs with two-plane halo exchanges and all-reduced "
              "dot products; a batch would split by problem)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1901_05118_amd as ex
    from manufactured import config_problem, make_arrays

    torch.cuda.set_device(0)
    if args.profile_sweeps:
        profile_sweeps(ex, args)
        return
    if args.only_2d:
        ex.set_stream(torch.cuda.current_stream())
        res = plane_leg(ex, torch, np, args.steps)
        print(json.dumps({
            "metric": "2D EXCMG GLUPS, time to a 1e-8 residual", "value": res["mixed"]["glups"],
            "unit": "GLUPS", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": res["mixed"]["ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": res["workload"], "n_finest": res["n_finest"],
                       "n_levels": res["n_levels"], "precision": "mixed"},
            "plane_2d": res}), flush=True)
        return
    N, nl, bc, tol = args.n, args.levels, args.bc, args.tol
    log(f"generating inputs {N}^3 bc={bc}")
    arr = make_arrays(config_problem(args.config), N, bc)
    dev = torch.device("cuda:0")
    f, g1, g2 = (torch.from_numpy(a).to(dev) for a in (arr.f, arr.g1, arr.g2))
    u = torch.empty_like(f)
    ut = torch.empty_like(f)
    stream = torch.cuda.current_stream()
    ex.set_stream(stream)
    tuned = {}
    if args.autotune:
        # tile shapes of every grid the runs use, chosen by timing (the project's autotuner)
        sizes = sorted({N >> k for k in range(nl - 2)} | {32, 48, 64, 96, 128, 24, 12, 16})
        for n in sizes:
            for kind in (0, 1):
                for prec in (ex.FP64, ex.MIXED):
                    if kind == 0 and prec == ex.MIXED:
                        continue
                    ty, zc, ms = ex.autotune(n, kind, prec, reps=3 if n >= 256 else 10)
                    tuned[f"{n}/{'sweepA' if kind else 'operator'}/{'fp32' if prec else 'fp64'}"] = [ty, zc]
        log(f"autotuned shapes: {tuned}")
    ex.setup(N, nl, bc)

    def solve(prec, refine=ex.RELIABLE):
        rc, st = ex.solve_ex(N, nl, bc, f, g1, g2, tol, u, ut, precision=prec, refine=refine)
        if rc != ex.OK:
            raise RuntimeError(f"solve failed: {rc} {ex.last_error()}")
        return st

    def timed(prec, name, refine=ex.RELIABLE):
        for w in range(args.warmup):
            st = solve(prec, refine)
            log(f"{name} warmup {w}: {st.total_ms:.1f} ms, iterations "
                f"{[l['iterations'] for l in st.levels()]}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            st = solve(prec, refine)
            log(f"{name} step {s}: {st.total_ms:.1f} ms")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        levels = st.levels()
        lups = sum(((lv["n"] - 1) ** 3) * lv["iterations"] for lv in levels)
        uu = u.view(N + 1, N + 1, N + 1).cpu().numpy()
        return {"ms": ms, "levels": levels, "glups": lups / (ms * 1e-3) / 1e9, "u": uu,
                "ut": ut.view(N + 1, N + 1, N + 1).cpu().numpy()}

    rms = lambda e: float(np.sqrt(np.mean(e * e)))  # noqa: E731
    r64 = timed(ex.FP64, "fp64")
    r32 = timed(ex.MIXED, "mixed")
    # the classic refinement form (restarted FP32 solves) for comparison
    r32r = timed(ex.MIXED, "mixed-restart", ex.RESTART)
    # the CG specialisation of Algorithm 2 (same iterates, one operator product per iteration)
    cg = {}
    for prec, name in ((ex.FP64, "fp64"), (ex.MIXED, "mixed")):
        method_solve = lambda: ex.solve_ex(N, nl, bc, f, g1, g2, tol, u, ut, precision=prec,  # noqa: E731
                                           method=ex.CG)
        method_solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s_ in range(args.steps):
            rc, stc = method_solve()
        torch.cuda.synchronize()
        cg[name] = round((time.perf_counter() - t0) * 1e3 / args.steps, 2)
        same = bool(np.array_equal(u.view(N + 1, N + 1, N + 1).cpu().numpy(),
                                   (r64 if prec == ex.FP64 else r32)["u"]))
        cg[name + "_bit_identical_to_bicg"] = same
        log(f"cg {name}: {cg[name]} ms, identical to Bi-CG: {same}")
    e64 = rms(r64["u"] - arr.u)
    e32 = rms(r32["u"] - arr.u)
    gate = abs(e32 - e64) <= 0.01 * e64
    head = r32 if gate else r64
    mode = "mixed" if gate else "fp64"
    ms_step = head["ms"]
    glups = head["glups"]
    levels = head["levels"]

    # Roofline: one more solve of the headline form with every Bi-CG sweep bracketed by
    # device events on the library stream; per level and sweep, achieved = algorithmic
    # bytes per launch / mean duration.  The headline kernel is the (level, sweep) with the
    # largest share of the step's time.
    prec = ex.MIXED if gate else ex.FP64
    ex.set_timing(True)
    st_t = solve(prec)
    if [lv["iterations"] for lv in st_t.levels()] != [lv["iterations"] for lv in levels]:
        raise RuntimeError("the event-timed solve took other iterations than the timed one")
    per_level = []
    for li, lv in enumerate(st_t.levels()):
        if li < 2:
            continue
        n_l = lv["n"]
        forms = sweep_forms(n_l, gate)
        for kind, (form, bpu, label) in forms.items():
            ms_tot, nl_ = ex.get_timing(li, kind)
            if nl_ == 0:
                continue
            nu_l = (n_l - 1) ** 3
            ty_l, zc_l = ex.get_shape(n_l, 2 if forms.fp32 else 1)
            kname, grid = sweep_launch(n_l, ty_l, zc_l, form)
            bpl = bpu * nu_l
            avg = ms_tot / nl_
            per_level.append({"n": n_l, "sweep": label, "kernel": kname, "grid": grid,
                              "tile": f"64x{ty_l}, {zc_l} planes", "launches": nl_,
                              "ms_total": round(ms_tot, 3), "ms_per_launch": round(avg, 5),
                              "bytes_per_unknown": bpu, "bytes_per_launch": bpl,
                              "gbs": round(bpl / (avg * 1e-3) / 1e9, 1),
                              "frac": round(bpl / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    ex.set_timing(False)
    swept_ms = sum(e["ms_total"] for e in per_level)
    swept_bytes = sum(e["bytes_per_launch"] * e["launches"] for e in per_level)
    dom = max(per_level, key=lambda e: e["ms_total"])
    traffic, traffic_src = recorded_traffic(dom["kernel"], dom["grid"])
    ms_c, bytes_c = ex.profile_sweep(4, ex.FP64, reps=10)
    # the stencil alone: y = A x on the finest level (FP64, 16 bytes per unknown)
    nu = (N - 1) ** 3
    ms_s, bytes_s = ex.profile_sweep(0, ex.FP64, reps=10)
    finest = [e for e in per_level if e["n"] == N]
    pair_of = lambda n_l: [e for e in per_level if e["n"] == n_l]  # noqa: E731
    dom_pair = pair_of(dom["n"])
    roofline = {"bound": "hbm", "achieved": dom["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": dom["frac"],
                "traffic": None if traffic is None else round(traffic),
                "traffic_source": traffic_src,
                "kernel": f"{dom['kernel']} (Bi-CG sweep {dom['sweep']}, {dom['n']}^3 level, "
                          f"tile {dom['tile']}, {dom['grid']} threads)",
                "share_of_step": round(dom["ms_total"] / ms_step, 4),
                "launches": dom["launches"], "ms_per_launch": dom["ms_per_launch"],
                "bytes_per_launch": dom["bytes_per_launch"],
                # the dominant level's Bi-CG iteration (all its sweeps, time-weighted)
                "dominant_level_iteration": {
                    "n": dom["n"],
                    "gbs": round(sum(e["bytes_per_launch"] * e["launches"] for e in dom_pair)
                                 / (sum(e["ms_total"] for e in dom_pair) * 1e-3) / 1e9, 1),
                    "frac": round(sum(e["bytes_per_launch"] * e["launches"] for e in dom_pair)
                                  / (sum(e["ms_total"] for e in dom_pair) * 1e-3) / 1e9
                                  / HBM_PEAK_GBS, 4)},
                # every timed Bi-CG sweep of the step, weighted by its time
                "all_sweeps_time_weighted": {
                    "ms": round(swept_ms, 2), "share_of_step": round(swept_ms / ms_step, 4),
                    "gbs": round(swept_bytes / (swept_ms * 1e-3) / 1e9, 1),
                    "frac": round(swept_bytes / (swept_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                # the same bytes over the whole step's wall time (direct solves, transfers,
                # residual replacements, polls and launch gaps included)
                "step_effective": {
                    "gbs": round(swept_bytes / (ms_step * 1e-3) / 1e9, 1),
                    "frac": round(swept_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                "levels": per_level,
                "finest_level": finest,
                "stencil_apply": {"n": N, "ms_per_launch": round(ms_s, 4),
                                  "glups": round(nu / (ms_s * 1e-3) / 1e9, 1),
                                  "gbs": round(bytes_s / (ms_s * 1e-3) / 1e9, 1),
                                  "frac": round(bytes_s / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                "copy_gbs": round(bytes_c / (ms_c * 1e-3) / 1e9, 1),
                "copy_frac": round(bytes_c / (ms_c * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    out = {
        "metric": METRIC, "value": round(glups, 3), "unit": "GLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if gate else "f64", "data": "synthetic",
        "config": {"workload": f"EXCMG {N}^3 cells, bc kind {bc}, seeded family {args.config}, "
                               f"tol {tol:g}, {mode}", "n_finest": N, "n_levels": nl,
                   "bc_kind": bc, "tol": tol, "precision": mode},
        "time_to_solution_ms": {"fp64": round(r64["ms"], 2), "mixed": round(r32["ms"], 2),
                                "mixed_restarted_refinement": round(r32r["ms"], 2),
                                "speedup_mixed": round(r64["ms"] / r32["ms"], 3),
                                "cg_specialisation": cg},
        "glups": {"fp64": round(r64["glups"], 3), "mixed": round(r32["glups"], 3)},
        "iterations": {"fp64": [lv["iterations"] for lv in r64["levels"]],
                       "mixed": [lv["iterations"] for lv in r32["levels"]],
                       "mixed_restarted_refinement": [lv["iterations"] for lv in r32r["levels"]]},
        # the paper's cost measure (Sec. 6): iterations on each level weighted by 8^-(levels
        # below the finest), in finest-grid sweeps
        "work_units": {k: round(sum(lv["iterations"] * 8.0 ** -(len(r["levels"]) - 1 - i)
                                    for i, lv in enumerate(r["levels"])), 2)
                       for k, r in (("fp64", r64), ("mixed", r32))},
        "runs": {"fp64": [lv["runs"] for lv in r64["levels"]],
                 "mixed": [lv["runs"] for lv in r32["levels"]]},
        "error_vs_exact": {"fp64_u_rms": e64, "mixed_u_rms": e32,
                           "fp64_ut_rms": rms(r64["ut"] - arr.u),
                           "mixed_vs_fp64_max": float(np.abs(r32["u"] - r64["u"]).max()),
                           "mixed_gate_1pct": bool(gate)},
        "roofline": roofline,
    }
    if tuned:
        out["autotuned_shapes"] = tuned
    if not args.no_jacobi:
        out["jacobi_fp64"] = jacobi_leg(ex, torch, np, N, nl, bc, tol, f, g1, g2, u, args.steps)
    if not args.no_batch:
        out["batch"] = batch_leg(ex, torch, np)
    if not args.no_2d:
        out["plane_2d"] = plane_leg(ex, torch, np, args.steps)
    kept = {}
    if not args.no_configs:
        out["configs"] = configs_leg(ex, torch, np, args.steps, kept)
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(arr, N, nl, bc, args.cpu_iters, kept)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
