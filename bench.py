"""Benchmark: Bloch band path of the parity-blocked solver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--budget S] [--workload cube|fcc]
                    [--n N] [--nk 16] [--nev M]

Workload: two-phase unit cube, n^3 grid (default n = 128), cubic matrix
(C11=1, C12=0.4, C44=0.3, rho=1) with a centred sphere r = 0.35 holding a seeded
SPD stiffness (rho = 4); 16 points on the Gamma-X-M-Gamma-R path; the 20 lowest
eigenpairs per point; shift delta = 0.30 C_max; tolerances 1e-12.
--workload fcc: the paper's FCC cell (quartz matrix, silicon sphere, subpixel
volume-fraction material; dimensionless units) at n = 60 on the 91-point
Gamma-X-W-K-Gamma-L-U-W-L-K path with 40 eigenpairs per point.

One step = one group of 4 consecutive path points, the unit the blocked path
solves in lockstep: at each of the 4 points four parity-block shift-invert Krylov
solves (16 solves advancing together, every launch covering all of them: inner
PCG with the FFT-diagonal preconditioner, the fused stencil matvec, Gamma
projection), merged with certification.  Steps cycle through the path's groups;
every step starts from the same seeded Krylov start vectors (no warm start from
an earlier step), so every visit of a group does the same work.  The reported
value is the path time assembled from the groups' mean step times.  K steps are
timed with a device synchronisation on both sides; W untimed warm-up steps come
first.  A wall-clock budget (--budget, from process start) bounds the run:
steps that would end past it are not started, and the line reports the steps
actually timed beside the requested ones.

Material form: the two-phase cell has two distinct (C21, rho) rows, so by
default the kernels read the palette form (one byte per node naming its row)
instead of 21 stiffness entries and rho per node; --material-form dense forces
the dense form.  Both give the same matvec bit for bit.

Also measured live: the fused matvec (A + delta M) x of the four parity blocks
in one launch (as the blocked path issues it; HIP events on the context stream)
in the dense material form, 272 algorithmic bytes per node (x, the 21 stiffness
entries and rho, y), reported against the MI355X HBM peak as the roofline of the
block matvec; the palette form of the same launch beside it; one block per
launch, the full-space matvec and the block preconditioner; the full-space solve
of the first group of path points (blocked vs full space, same GPU, same
tolerances) when the budget leaves room for it; and the oracle (CPU) cost of the
path extrapolated from a bounded sample (one oracle operator application and one
oracle preconditioner application on a grid with a block's node count,
single-threaded, scaled by the GPU path's PCG iteration count).
"""

import time

T_START = time.perf_counter()  # process start, for the wall-clock budget

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = 48 + 168 + 8 + 48   # x, C (21 doubles), rho, y (dense material form)
PAL_BYTES_PER_NODE = 48 + 1 + 48     # x, palette row (one byte), y (palette form)
PRECOND_BYTES_PER_NODE = 48 + 48     # r in, z out


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=0)
    p.add_argument("--budget", type=float, default=480.0,
                   help="wall-clock seconds from process start that the run may take; "
                        "steps that would end past it are not started")
    p.add_argument("--group", type=int, default=4,
                   help="path points per step (solved in lockstep; 4 = the blocked "
                        "path's own batch)")
    p.add_argument("--study", choices=("refinement", "cells", "gap", "path"), default=None,
                   help="refinement: grouped grid-refinement errors of the FCC workload at "
                        "Gamma, X and W against a 256^3 reference (Sec. 7.5; one JSON line)")
    p.add_argument("--workload", choices=("cube", "fcc"), default="cube",
                   help="cube: the two-phase unit cube (default); fcc: the paper's quartz/Si "
                        "FCC cell on its 91-point path")
    p.add_argument("--n", type=int, default=0, help="grid size (default 128 cube, 60 fcc)")
    p.add_argument("--nk", type=int, default=16, help="path points (cube workload)")
    p.add_argument("--nev", type=int, default=0, help="eigenpairs per k (default 20 cube, 40 fcc)")
    p.add_argument("--range", nargs=2, type=int, metavar=("FROM", "TO"), default=None,
                   help="--study path: solve path points FROM <= i < TO only (a long path in "
                        "several runs)")
    p.add_argument("--first", type=int, default=0,
                   help="time only the first m points of the path (short profiled runs)")
    p.add_argument("--full-every", type=int, default=4,
                   help="compare with the full space on every k-th path point (0: skip)")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle sample")
    p.add_argument("--matvec-only", action="store_true",
                   help="only the four-block matvec launches (dense and palette form) and the "
                        "copy probe, timed (for kernel-trace and hardware-counter runs)")
    p.add_argument("--mv-iters", type=int, default=100)
    p.add_argument("--material-form", choices=("auto", "dense"), default="auto",
                   help="auto: the kernels read the material's palette form when it has one "
                        "(at most 256 distinct rows); dense: always the 21 + 1 doubles per node")
    p.add_argument("--traffic-record", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                   help="write the matvec traffic records under profiles/ from two rocprofv3 "
                        "--pmc runs (FETCH_SIZE, WRITE_SIZE) of --matvec-only")
    p.add_argument("--kernel-stats", metavar="TRACE_DIR",
                   help="print a markdown summary of a rocprofv3 --kernel-trace --stats "
                        "--output-format csv directory: per kernel and per launch grid")
    p.add_argument("--counter-stats", nargs="+", metavar="PMC_DIR",
                   help="print the mean of each hardware counter per (kernel, launch grid) "
                        "from rocprofv3 --pmc --output-format csv directories")
    p.add_argument("--pcg-probe", action="store_true",
                   help="a short lockstep PCG workload for hardware-counter runs: the bench "
                        "cell, one merged solve at the second path point with a 6-vector "
                        "Krylov space and one outer iteration (it stops unconverged)")
    p.add_argument("--serial-blocks", action="store_true",
                   help="solve the four blocks one after another instead of in lockstep")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def ctx_events(torch, ctx):
    """Start / end timing events recorded on the stream the context launches
    on (pbr_stream), not on torch's current stream."""
    h = ctx.stream_handle()
    st = torch.cuda.ExternalStream(h) if h else torch.cuda.default_stream()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    return st, s, e


def kernel_timing(torch, ctx, n, kappa, delta, iters, blocks, op):
    """Average duration (s) of one launch of `op` ("apply": the fused matvec
    (A + delta M) x; "precond": the FFT preconditioner) over `iters` launches that
    rotate through `blocks`, so that consecutive launches touch different data and
    the 256 MB last-level cache cannot serve a repeated block.  HIP events are
    recorded on the context's stream."""
    from synth import complex_gaussian
    xs, ys = [], []
    for blk in blocks:
        N = n ** 3 if blk < 0 else n ** 3 // 4
        xs.append(torch.from_numpy(complex_gaussian(3 * N, seed=12345)).cuda())
        ys.append(torch.zeros_like(xs[-1]))

    def launch(t):
        j = t % len(blocks)
        if op == "apply":
            ctx.apply(kappa, blocks[j], delta, xs[j], ys[j])
        else:
            ctx.precond(kappa, blocks[j], delta, xs[j], ys[j])

    for t in range(4 * len(blocks)):
        launch(t)
    st, s, e = ctx_events(torch, ctx)
    torch.cuda.synchronize()
    s.record(st)
    for t in range(iters):
        launch(t)
    e.record(st)
    torch.cuda.synchronize()
    del xs, ys
    return s.elapsed_time(e) / 1e3 / iters


def blocks_timing(torch, ctx, n, kappa, delta, iters):
    """Average duration (s) of one launch applying (A + delta M) to all four
    parity blocks (pbr_apply_blocks); HIP events on the context's stream.  The four blocks' stiffness alone (352 MB at
    n=128) exceeds the 256 MB last-level cache."""
    from synth import complex_gaussian
    x = torch.from_numpy(complex_gaussian(3 * n ** 3, seed=12345)).cuda()
    y = torch.zeros_like(x)
    for _ in range(5):
        ctx.apply_blocks(kappa, delta, x, y)
    st, s, e = ctx_events(torch, ctx)
    torch.cuda.synchronize()
    s.record(st)
    for _ in range(iters):
        ctx.apply_blocks(kappa, delta, x, y)
    e.record(st)
    torch.cuda.synchronize()
    del x, y
    return s.elapsed_time(e) / 1e3 / iters


def copy_peak(torch, ctx, nbytes=2 << 30, iters=20):
    """Rate (GB/s, bytes read + written) of the library's streaming copy probe
    over a 2 GiB buffer, timed like the operator kernels."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        ctx.copy_probe(a, b)
    st, s, e = ctx_events(torch, ctx)
    torch.cuda.synchronize()
    s.record(st)
    for _ in range(iters):
        ctx.copy_probe(a, b)
    e.record(st)
    torch.cuda.synchronize()
    t = s.elapsed_time(e) / 1e3 / iters
    ok = bool(torch.equal(a, b))
    del a, b
    assert ok, "copy probe produced a wrong copy"
    return 2 * nbytes / t / 1e9


def cpu_sample(n, kappa, C21_full, rho_full, delta, reps=3):
    """Oracle (as written, single-threaded) cost of one PCG iteration's operator
    work on one parity block at grid n: one application of A + delta M (index
    formula) and one preconditioner application (numpy.fft), each timed on a
    grid with a block's node count (n x n/2 x n/2, the two-phase material
    sampled on it), median of `reps` runs.  The oracle has no block-native
    operator (it applies a block through the full-space one on a zero-extended
    vector, four times this cost), so the block-sized grid is the cheaper and
    fairer stand-in."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import fourier as F, pointwise as P
    from synth import complex_gaussian, two_phase_cell
    dims = (n, n // 2, n // 2)
    C21, rho, _ = two_phase_cell(dims, radius=0.35, seed=0)
    x = complex_gaussian(3 * n ** 3 // 4, seed=12345)
    Cref, rref = F.reference_material(C21_full, rho_full)
    t_mv, t_pc = [], []
    with threadpool_limits(limits=1):
        for _ in range(reps):
            t0 = time.perf_counter()
            y = P.apply_A(x, dims, kappa, C21, rho, s=delta)
            t1 = time.perf_counter()
            z = F.precond_fft(y, dims, kappa, -1, Cref, rref, delta)
            t2 = time.perf_counter()
            t_mv.append(t1 - t0)
            t_pc.append(t2 - t1)
    assert np.isfinite(z).all()
    return float(np.median(t_mv)), float(np.median(t_pc)), dims


def kernel_stats(trace_dir, top=16):
    """Markdown summary of a rocprofv3 kernel trace (csv): calls, mean and total
    time per kernel (its stats file), then mean time per (kernel, launch grid)
    from the trace itself."""
    import collections
    import csv
    import glob
    stats = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    trace = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not stats or not trace:
        raise SystemExit(f"no kernel_stats.csv / kernel_trace.csv under {trace_dir}")

    def short(name):
        name = name.replace("(anonymous namespace)::", "").replace("void ", "")
        return name[:name.index(">") + 1] if "<" in name else name.split("(")[0]

    rows = list(csv.DictReader(open(stats[0])))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["| kernel | calls | avg us | total s | % |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e9:.3f} | {float(r['Percentage']):.1f} |")
    out.append(f"\nTotal kernel time {total / 1e9:.3f} s.\n")
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in csv.DictReader(open(trace[0])):
        key = (short(r["Kernel_Name"]), r["Grid_Size_X"], r["Grid_Size_Y"], r["Grid_Size_Z"],
               r["Workgroup_Size_X"])
        agg[key][0] += 1
        agg[key][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    out += ["| kernel | grid (x, y, z) | work-group | launches | avg us |",
            "|---|---|---|---|---|"]
    for k, (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"| {k[0]} | ({k[1]}, {k[2]}, {k[3]}) | {k[4]} | {c} | {t / c:.1f} |")
    return "\n".join(out)


def counter_stats(dirs):
    """Mean value of each hardware counter per (kernel, launch grid, work-group)
    over the dispatches of rocprofv3 --pmc csv runs, one markdown table per run."""
    import collections
    import csv
    import glob
    out = []
    for d in dirs:
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit(f"no counter_collection.csv under {d}")
        agg = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(files[0])):
            nm = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "")
            nm = nm[:nm.index(">") + 1] if "<" in nm else nm.split("(")[0]
            agg[(nm, r.get("Grid_Size", ""), r.get("Workgroup_Size", ""))][r["Counter_Name"]].append(
                float(r["Counter_Value"]))
        names = sorted({c for v in agg.values() for c in v})
        out.append(f"{os.path.basename(os.path.normpath(d))}:\n")
        out.append("| kernel | grid | work-group | dispatches | " + " | ".join(names) + " |")
        out.append("|---" * (4 + len(names)) + "|")
        for key, cs in sorted(agg.items()):
            n = max(len(v) for v in cs.values())
            vals = [f"{sum(cs[c]) / len(cs[c]):.4g}" if cs.get(c) else "" for c in names]
            out.append(f"| {key[0]} | {key[1]} | {key[2]} | {n} | " + " | ".join(vals) + " |")
        out.append("")
    return "\n".join(out)


def pcg_probe(n=128):
    """Short lockstep PCG workload (hardware-counter runs): the bench cell, one
    merged solve at the second path point with a 6-vector Krylov space and a
    single outer iteration, which stops unconverged after a few thousand
    four-layout PCG launches."""
    import torch
    from paper_2606_03599_amd import pbr
    from synth import sc_path, two_phase_cell
    C21, rho, _ = two_phase_cell((n, n, n), radius=0.35, seed=0)
    ctx = pbr.Context((n, n, n))
    ctx.set_material(torch.from_numpy(C21).cuda(), torch.from_numpy(rho).cuda())
    del C21, rho
    kappas, _ = sc_path(16)
    o = pbr.pbr_opts_default()
    o.ncv = 6
    o.maxit_outer = 1
    try:
        ctx.eigs_merged(tuple(kappas[1]), 4, opts=o)
    except pbr.PbrError as e:
        log(f"pcg probe stopped as set up (status {e.status})")
    torch.cuda.synchronize()
    ctx.close()


def traffic_record(kernel_src, name):
    """Hardware-counter traffic of the matvec kernel, if it was measured on the
    current source (profiles/<name>.json records the source hash)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(kernel_src, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != h:
        return None
    return rec


def traffic_records(fetch_dir, write_dir, n=128):
    """Write profiles/matvec_blocks_n<n>_<form>_traffic.json from two rocprofv3
    --pmc runs of `bench.py --matvec-only` (FETCH_SIZE, then WRITE_SIZE; KiB
    per dispatch).  Each counter is scaled by the factor that makes it read
    the true bytes of the copy probe's 2 GiB dispatches in the same run; the
    four-block launches of each material form are the most frequent grid of
    that form's kernel instance."""
    import collections
    import csv
    import glob
    import hashlib
    import statistics

    def rdir(d):  # a run directory as the command lines give it: under the repository root R
        return "$R/" + os.path.relpath(os.path.abspath(d), ROOT)

    def load(d, counter):
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        per = collections.defaultdict(dict)
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name") != counter:
                continue
            key = r["Dispatch_Id"]
            per[key]["name"] = r["Kernel_Name"]
            per[key]["grid"] = int(r.get("Grid_Size", 0) or 0)
            per[key]["v"] = per[key].get("v", 0.0) + float(r["Counter_Value"])
        return list(per.values())

    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy_bytes = (2 << 30)
    cf = [d["v"] for d in fetch if "copy_probe_kernel" in d["name"]]
    cw = [d["v"] for d in write if "copy_probe_kernel" in d["name"]]
    f_factor = copy_bytes / 1024 / statistics.median(cf)
    w_factor = copy_bytes / 1024 / statistics.median(cw)
    src = os.path.join(ROOT, "paper_2606_03599_amd", "csrc", "stencil.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    nb4 = 4 * n ** 3 // 4
    out = {}
    import re
    inst = re.compile(r"apply_stream_kernel<\s*\d+,\s*\d+,\s*(true|false)\s*>")

    def form_of(name):
        m = inst.search(name)
        return None if m is None else ("palette" if m.group(1) == "true" else "dense")

    for form, bpn in (("dense", BYTES_PER_NODE), ("palette", PAL_BYTES_PER_NODE)):
        fk = [d for d in fetch if form_of(d["name"]) == form]
        wk = [d for d in write if form_of(d["name"]) == form]
        if not fk or not wk:
            continue
        grid = collections.Counter(d["grid"] for d in fk).most_common(1)[0][0]
        fv = [d["v"] for d in fk if d["grid"] == grid]
        wv = [d["v"] for d in wk if d["grid"] == grid]
        fb = statistics.mean(fv) * 1024 * f_factor
        wb = statistics.mean(wv) * 1024 * w_factor
        rec = {
            "kernel": f"apply_stream_kernel, {form} material form: fused (A + delta M) x of the "
                      f"four parity blocks in one launch, n={n} (4 x {n ** 3 // 4} nodes)",
            "source": "paper_2606_03599_amd/csrc/stencil.hip", "source_sha256": sha,
            "commands": [
                "cd /tmp && export TMPDIR=/tmp && timeout -s KILL 200 rocprofv3 --pmc FETCH_SIZE "
                f"--output-format csv -d {rdir(fetch_dir)} -o pf -- python3 -u $R/bench.py "
                "--matvec-only --mv-iters 20",
                "cd /tmp && export TMPDIR=/tmp && timeout -s KILL 200 rocprofv3 --pmc WRITE_SIZE "
                f"--output-format csv -d {rdir(write_dir)} -o pw -- python3 -u $R/bench.py "
                "--matvec-only --mv-iters 20",
                f"python3 $R/bench.py --traffic-record {rdir(fetch_dir)} {rdir(write_dir)}"],
            "grid_threads": grid, "launches_averaged": len(fv),
            "fetch_size_kib_raw": round(statistics.mean(fv), 2),
            "write_size_kib_raw": round(statistics.mean(wv), 2),
            "copy_calibration": {
                "kernel": "copy_probe_kernel (pbr_copy_probe of 2 GiB, same runs)",
                "true_kib_each_way": copy_bytes / 1024,
                "fetch_size_kib": round(statistics.median(cf), 2),
                "write_size_kib": round(statistics.median(cw), 2),
                "fetch_factor": round(f_factor, 5), "write_factor": round(w_factor, 5)},
            "algorithmic_bytes_per_node": bpn,
            "hbm_fetch_bytes_per_launch": int(fb), "hbm_write_bytes_per_launch": int(wb),
            "hbm_bytes_per_launch": int(fb + wb),
            "algorithmic_bytes_per_launch": bpn * nb4,
            "traffic_over_algorithmic": round((fb + wb) / (bpn * nb4), 3)}
        path = os.path.join(ROOT, "profiles", f"matvec_blocks_n{n}_{form}_traffic.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        out[form] = rec["traffic_over_algorithmic"]
    return out


def grouped_errors(lam, lam_ref, n_zero=0, bands=40, group=4):
    """Grouped relative frequency errors of one wave vector (the convergence
    diagnostic of the paper's grid-refinement test, Sec. 7.5): of the first
    `bands` bands, the first `n_zero` are the zero modes of the discrete null
    space (Gamma: 12) and are excluded; `lam`, `lam_ref` are the remaining,
    non-zero eigenvalues (lambda = omega^2), ascending, on the coarse grid and on
    the reference grid.  Bands are grouped `group` at a time in band order and a
    group's error is the mean of |f - f_ref| / f_ref over its non-zero members
    (f proportional to sqrt(lambda)); groups holding only zero modes are None."""
    import numpy as np
    out = []
    k = bands - n_zero
    f = np.sqrt(np.asarray(lam, dtype=float)[:k])
    fr = np.sqrt(np.asarray(lam_ref, dtype=float)[:k])
    rel = np.abs(f - fr) / fr
    for g in range(bands // group):
        members = [b - n_zero for b in range(g * group, (g + 1) * group) if b >= n_zero]
        out.append(None if not members else float(np.mean(rel[members])))
    return out


def refinement_study(grids=(8, 16, 32, 64, 128), ref=256, bands=40, points=("G", "X", "W")):
    """Grid refinement of the FCC workload as the paper tests it (Sec. 7.5): the
    first 40 bands at Gamma, X and W on 8^3 ... 128^3 against the 256^3 result
    (blocked: the same spectrum as the full space by Corollary 4.2), averaged in
    10 groups of 4 bands, each group's error the mean relative frequency error of
    its non-zero branches (Gamma's 12 zero modes excluded), and the observed
    orders log2(e_n / e_2n)."""
    import numpy as np
    import torch
    from paper_2606_03599_amd import pbr
    from synth import fcc_point, fcc_quartz_si_cell
    vals = {}
    t0 = time.perf_counter()
    for n in tuple(grids) + (ref,):
        C21, rho, A, _ = fcc_quartz_si_cell((n, n, n), supersample=4)
        ctx = pbr.Context((n, n, n), A_lat=A)
        ctx.set_material(torch.from_numpy(C21).cuda(), torch.from_numpy(rho).cuda())
        del C21, rho
        for p in points:
            nz = 12 if p == "G" else 0
            ev, st = ctx.eigs_merged(tuple(fcc_point(p)), bands - nz)
            vals[(n, p)] = np.asarray(ev)
            log(f"refinement n={n} {p}: {np.round(ev[:4], 6)} ({time.perf_counter() - t0:.0f} s)")
        ctx.close()
        torch.cuda.empty_cache()
    err, order = {}, {}
    for p in points:
        nz = 12 if p == "G" else 0
        err[p] = {n: grouped_errors(vals[(n, p)], vals[(ref, p)], nz, bands) for n in grids}
        order[p] = {}
        for a, b in zip(grids[:-1], grids[1:]):
            order[p][f"{a}->{b}"] = [None if ea is None or eb is None or eb <= 0 else
                                     round(float(np.log2(ea / eb)), 3)
                                     for ea, eb in zip(err[p][a], err[p][b])]
    return {"study": "grid refinement of the FCC quartz/Si cell (Sec. 7.5 metric): first "
                     f"{bands} bands in groups of 4, mean relative frequency error of each "
                     f"group's non-zero branches against {ref}^3 (blocked), Gamma's 12 zero "
                     "modes excluded",
            "reference_n": ref, "grids": list(grids), "points": list(points),
            "group_error": err, "observed_order": order,
            "seconds": round(time.perf_counter() - t0, 1)}


def gap_gradient_study(n, nev, points=("X", "R"), seed=0):
    """Large-grid slice of the batching + differentiation workload: the two-phase
    cell at n^3, the blocked band path at X and R with nev eigenpairs (four
    blocks in lockstep), then the gradient of the gap width lambda_7 - lambda_6
    at X with respect to the nodewise C21 and rho (Hellmann-Feynman, strains
    recomputed on the device), checked along one random direction over 50 nodes
    against a central difference with relative step 1e-6."""
    import numpy as np
    import torch
    from paper_2606_03599_amd import pbr
    from paper_2606_03599_amd.autograd import band_eigenvalues
    from synth import SC_POINTS, two_phase_cell
    dims = (n, n, n)
    C21, rho = two_phase_cell(dims, radius=0.35, seed=seed)[:2]
    ctx = pbr.Context(dims)
    Ct = torch.tensor(C21, device="cuda", requires_grad=True)
    rt = torch.tensor(rho, device="cuda", requires_grad=True)
    ctx.set_material(Ct.detach(), rt.detach())
    kps = [SC_POINTS[p] for p in points]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, st = ctx.band_path(kps, nev)
    t_path = time.perf_counter() - t0
    log(f"n={n} blocked path at {points}, nev={nev}: {t_path:.1f} s, {st.op_applies} solves, "
        f"{st.pcg_avg:.1f} PCG iterations per solve")
    kap = SC_POINTS[points[0]]
    t0 = time.perf_counter()
    lam = band_eigenvalues(ctx, kap, Ct, rt, 8)
    gap = lam[6] - lam[5]
    gC, gr = torch.autograd.grad(gap, [Ct, rt])
    gap = float(gap.detach())
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    log(f"gap lambda_7 - lambda_6 at {points[0]} = {gap:.6e}, eigenvalues and gradient "
        f"{t_grad:.1f} s")
    rng = np.random.default_rng(256)
    nodes = rng.choice(C21.shape[0], size=50, replace=False)
    dC = np.zeros((50, 21)) + rng.standard_normal((50, 21)) * np.abs(C21[nodes]).mean()
    dr = rng.standard_normal(50) * rho[nodes]
    ana = float((gC[nodes].cpu().numpy() * dC).sum() + (gr[nodes].cpu().numpy() * dr).sum())
    h = 1e-6
    fd = 0.0
    for sgn in (1.0, -1.0):
        C2, r2 = C21.copy(), rho.copy()
        C2[nodes] += sgn * h * dC
        r2[nodes] += sgn * h * dr
        l2 = band_eigenvalues(ctx, kap, torch.tensor(C2, device="cuda"),
                              torch.tensor(r2, device="cuda"), 8).cpu().numpy()
        fd += sgn * (l2[6] - l2[5]) / (2 * h)
        del C2, r2
    log(f"directional derivative of the gap: analytic {ana:.6e}, central difference {fd:.6e}")
    ctx.close()
    return {"study": "large grid: blocked band path and the gradient of a gap width",
            "workload": f"two-phase unit cube n={n}^3 ({n ** 3} nodes, {n ** 3 // 4} per block), "
                        f"blocked path at {list(points)}, {nev} lowest eigenpairs per k; gap "
                        f"lambda_7 - lambda_6 at {points[0]}",
            "path_s": round(t_path, 3), "solves": st.op_applies, "pcg_avg": round(st.pcg_avg, 2),
            "eigenvalues": {p: [float(x) for x in e[:8]] for p, e in zip(points, ev)},
            "gap": gap, "eigs_and_gradient_s": round(t_grad, 3),
            "grad_norms": {"C21": float(gC.norm()), "rho": float(gr.norm())},
            "directional_check": {"analytic": ana, "central_difference": fd,
                                  "rel_diff": abs(ana - fd) / max(abs(fd), 1e-300)}}


def path_study(n, nk, nev, rng_pts=None, group=2, seed=0):
    """Blocked band path of the two-phase cell (radius 0.35) at n^3 over the
    nk-point Gamma-X-M-Gamma-R path, nev eigenpairs per k, tolerances 1e-12:
    points FROM <= i < TO (all by default), solved `group` points at a time in
    lockstep (four blocks each), each group logged as it ends."""
    import torch
    from paper_2606_03599_amd import pbr
    from synth import sc_path, two_phase_cell
    kappas, _ = sc_path(nk)
    a, b = (0, nk) if rng_pts is None else (max(0, rng_pts[0]), min(nk, rng_pts[1]))
    dims = (n, n, n)
    t_setup = time.perf_counter()
    C21, rho = two_phase_cell(dims, radius=0.35, seed=seed)[:2]
    ctx = pbr.Context(dims)
    ctx.set_material(torch.from_numpy(C21).cuda(), torch.from_numpy(rho).cuda())
    del C21, rho
    torch.cuda.synchronize()
    log(f"n={n}: material set in {time.perf_counter() - t_setup:.1f} s; points {a}..{b - 1} of "
        f"{nk}, {nev} eigenpairs, {group} points per group")
    total = 0.0
    solves = pcg_sum = 0
    max_resid = 0.0
    groups, evals = [], {}
    for g0 in range(a, b, group):
        ks = kappas[g0:min(g0 + group, b)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, st = ctx.band_path(ks, nev)
        dt = time.perf_counter() - t0
        total += dt
        solves += st.op_applies
        pcg_sum += st.pcg_iters_total
        max_resid = max(max_resid, st.max_rel_resid)
        groups.append({"points": [g0, g0 + len(ks) - 1], "s": round(dt, 3),
                       "solves": st.op_applies, "pcg_avg": round(st.pcg_avg, 2)})
        for q in range(len(ks)):
            evals[g0 + q] = [float(x) for x in ev[q]]
        log(f"points {g0}-{g0 + len(ks) - 1}: {dt:.1f} s, {st.op_applies} solves, "
            f"{st.pcg_avg:.1f} PCG per solve (total {total:.1f} s)")
    ctx.close()
    return {"study": "blocked band path of the two-phase cube, run in ranges of path points",
            "workload": f"two-phase unit cube n={n}^3 ({n ** 3} nodes, four blocks of "
                        f"{n ** 3 // 4}), {nk}-point Gamma-X-M-Gamma-R path, {nev} lowest "
                        f"eigenpairs per k, tolerances 1e-12",
            "n": n, "nk": nk, "nev": nev, "range": [a, b], "group": group,
            "path_s": round(total, 3), "s_per_point": round(total / max(1, b - a), 3),
            "solves": solves, "pcg_avg": round(pcg_sum / max(1, solves), 2),
            "max_rel_resid": max_resid, "groups": groups, "eigenvalues": evals}


def cells_study(nk, nev, count=8, seed=0, first=0):
    """Uneven batch of two-phase cells (n drawn from {64, 96, 128}, inclusion
    radius from U[0.2, 0.4], each with its own seeded inclusion stiffness): the
    blocked band paths of all cells, group of 4 path points by group, first one
    cell after another, then all cells at once (pbr_band_paths: one host thread
    and stream per cell).  Results must agree bit for bit."""
    import numpy as np
    import torch
    from paper_2606_03599_amd import pbr
    from synth import batch_cells, sc_path
    cells = batch_cells(count, seed=seed)
    kappas, _ = sc_path(nk)
    if first > 0:
        kappas = kappas[:first]
    ctxs = []
    for n, r, C21, rho in cells:
        ctx = pbr.Context((n, n, n))
        ctx.set_material(torch.from_numpy(C21).cuda(), torch.from_numpy(rho).cuda())
        ctxs.append(ctx)
    sizes = [c[0] for c in cells]
    radii = [round(c[1], 4) for c in cells]
    del cells
    log(f"cells: n = {sizes}, radius = {radii}, {nk} k-points, nev = {nev}")
    t_serial = t_conc = 0.0
    same = True
    max_diff = 0.0
    solves = 0
    for g0 in range(0, len(kappas), 4):
        ks = kappas[g0:g0 + 4]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        serial = [ctx.band_path(ks, nev)[0] for ctx in ctxs]
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        t0 = time.perf_counter()
        conc, sts = pbr.band_paths(ctxs, [ks] * len(ctxs), nev)
        tc = time.perf_counter() - t0
        t_serial += ts
        t_conc += tc
        solves += int(sum(st.op_applies for st in sts))
        same = same and all(np.array_equal(a, b) for a, b in zip(serial, conc))
        diff = [float(np.max(np.abs(a - b) / np.abs(a))) for a, b in zip(serial, conc)]
        max_diff = max(max_diff, max(diff))
        log(f"points {g0}-{g0 + len(ks) - 1}: one after another {ts:.1f} s, all at once {tc:.1f} s "
            f"(totals {t_serial:.1f} / {t_conc:.1f} s), identical {same}, max rel diff per cell "
            + " ".join(f"{d:.1e}" for d in diff))
    for ctx in ctxs:
        ctx.close()
    return {"study": "uneven batch of cells, blocked band paths, one after another vs all cells "
                     "at once (pbr_band_paths), 4 path points at a time",
            "cells": [{"n": n, "radius": r} for n, r in zip(sizes, radii)],
            "k_points": len(kappas), "nev": nev,
            "one_after_another_s": round(t_serial, 3), "concurrent_s": round(t_conc, 3),
            "speedup": round(t_serial / t_conc, 3), "solves": solves,
            "results_identical": bool(same), "max_rel_diff": max_diff}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: collectives and sharding are "
                                   "not part of this implementation, so --gpus must be 1"}))
        sys.exit(2)
    if args.counter_stats:
        print(counter_stats(args.counter_stats), flush=True)
        return
    if args.pcg_probe:
        pcg_probe(args.n if args.n > 0 else 128)
        return
    if args.kernel_stats:
        print(kernel_stats(args.kernel_stats), flush=True)
        return
    if args.traffic_record:
        print(json.dumps(traffic_records(*args.traffic_record)), flush=True)
        return
    if args.study == "refinement":
        print(json.dumps(refinement_study()), flush=True)
        return
    if args.study == "gap":
        print(json.dumps(gap_gradient_study(args.n if args.n > 0 else 256,
                                            args.nev if args.nev > 0 else 30)), flush=True)
        return
    if args.study == "path":
        print(json.dumps(path_study(args.n if args.n > 0 else 256, args.nk,
                                    args.nev if args.nev > 0 else 30, args.range,
                                    max(1, min(4, args.group)))),
              flush=True)
        return
    if args.study == "cells":
        print(json.dumps(cells_study(args.nk if args.nk != 16 else 24,
                                     args.nev if args.nev > 0 else 16, first=args.first)),
              flush=True)
        return
    import numpy as np
    import torch
    from paper_2606_03599_amd import pbr
    from synth import fcc_path, fcc_quartz_si_cell, sc_path, two_phase_cell

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    fcc = args.workload == "fcc"
    n = args.n if args.n > 0 else (60 if fcc else 128)
    nev = args.nev if args.nev > 0 else (40 if fcc else 20)
    dims = (n, n, n)
    A_lat = None
    if fcc:
        C21, rho, A_lat, _ = fcc_quartz_si_cell(dims, supersample=4)
        kappas, _ = fcc_path(10)
        wl = (f"FCC cell (quartz matrix, silicon sphere R = a0/4, subpixel volume-fraction "
              f"material) n={n}^3, 91-point Gamma-X-W-K-Gamma-L-U-W-L-K path")
    else:
        C21, rho, _ = two_phase_cell(dims, radius=0.35, seed=0)
        kappas, _ = sc_path(args.nk)
        wl = f"two-phase unit cube n={n}^3, {args.nk}-point Gamma-X-M-Gamma-R path"
    log(f"workload: {wl}, nev={nev}")
    ctx = pbr.Context(dims, A_lat=A_lat)
    ctx.set_material(torch.from_numpy(C21).cuda(), torch.from_numpy(rho).cuda())
    delta = ctx.default_shift()
    pal_rows = ctx.palette_size()
    if args.material_form == "dense":
        ctx.set_palette(False)
    form = "palette" if ctx.palette_size() > 0 else "dense"
    log(f"material: {pal_rows} distinct rows, the kernels read the {form} form")
    if args.first > 0:
        kappas = kappas[:args.first]
    kap_mv = (0.15, 0.05, 0.10)
    opts = pbr.pbr_opts_default()
    opts.concurrent = 0 if args.serial_blocks else 1

    # ---- block matvec roofline: the four-block launch, live HIP-event timing ----
    # dense form (the 272 B/node of the metric), then the palette form if the
    # material has one; the solver runs whichever `form` names.
    ctx.set_palette(False)
    t_b4 = blocks_timing(torch, ctx, n, kap_mv, delta, max(10, args.mv_iters // 2))
    t_b4_pal = None
    if pal_rows > 0:
        ctx.set_palette(True)
        t_b4_pal = blocks_timing(torch, ctx, n, kap_mv, delta, max(10, args.mv_iters // 2))
    ctx.set_palette(form == "palette")
    if args.matvec_only:  # counter runs: the four-block launches and the copy probe only
        t_blk = t_full = t_pc = float("nan")
    else:
        t_blk = kernel_timing(torch, ctx, n, kap_mv, delta, args.mv_iters, (0, 1, 2, 3), "apply")
        t_full = kernel_timing(torch, ctx, n, kap_mv, delta, max(8, args.mv_iters // 4), (-1,),
                               "apply")
        t_pc = kernel_timing(torch, ctx, n, kap_mv, delta, max(8, args.mv_iters // 2),
                             (0, 1, 2, 3), "precond")
    nb = n ** 3 // 4
    bpn = PAL_BYTES_PER_NODE if form == "palette" else BYTES_PER_NODE
    b4_bytes = BYTES_PER_NODE * 4 * nb
    b4_gbs = b4_bytes / t_b4 / 1e9
    blk_gbs = bpn * nb / t_blk / 1e9
    full_gbs = bpn * n ** 3 / t_full / 1e9
    pc_gbs = PRECOND_BYTES_PER_NODE * nb / t_pc / 1e9
    cpeak = copy_peak(torch, ctx)
    log(f"4-block matvec launch, dense form: {t_b4*1e6:.1f} us = {b4_gbs:.0f} GB/s"
        + ("" if t_b4_pal is None else f"; palette form {t_b4_pal*1e6:.1f} us"))
    log(f"one block ({form}) {t_blk*1e6:.1f} us = {blk_gbs:.0f} GB/s; full {t_full*1e6:.1f} us "
        f"= {full_gbs:.0f} GB/s; block preconditioner {t_pc*1e6:.1f} us; copy probe "
        f"{cpeak:.0f} GB/s")
    stencil_src = os.path.join(ROOT, "paper_2606_03599_amd", "csrc", "stencil.hip")
    rec = traffic_record(stencil_src, f"matvec_blocks_n{n}_dense_traffic")
    roof = {"bound": "hbm", "achieved": round(b4_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(b4_gbs / HBM_PEAK_GBS, 4),
            "traffic": (None if rec is None else rec["hbm_bytes_per_launch"]),
            "kernel": "apply_stream_kernel, dense material form: fused (A + delta M) x of the "
                      "four parity blocks in one launch (272 algorithmic bytes per node: "
                      "x 48, stiffness 168, rho 8, y 48)",
            "algorithmic_bytes": b4_bytes, "avg_launch_us": round(t_b4 * 1e6, 2),
            "frac_of_copy_probe": round(b4_gbs / cpeak, 4)}
    if t_b4_pal is not None:
        pb = PAL_BYTES_PER_NODE * 4 * nb
        prec = traffic_record(stencil_src, f"matvec_blocks_n{n}_palette_traffic")
        roof["palette_form"] = {
            "kernel": "the same launch in the palette material form (97 algorithmic bytes "
                      "per node: x 48, one palette byte, y 48; what the path runs for this "
                      "two-row material)",
            "achieved": round(pb / t_b4_pal / 1e9, 1), "unit": "GB/s",
            "frac": round(pb / t_b4_pal / 1e9 / HBM_PEAK_GBS, 4),
            "algorithmic_bytes": pb, "avg_launch_us": round(t_b4_pal * 1e6, 2),
            "traffic": (None if prec is None else prec["hbm_bytes_per_launch"])}
    kernels = {"blocks4_matvec_dense_us": round(t_b4 * 1e6, 2),
               "block_matvec_us": round(t_blk * 1e6, 2), "block_matvec_GBps": round(blk_gbs, 1),
               "full_matvec_us": round(t_full * 1e6, 2), "full_matvec_GBps": round(full_gbs, 1),
               "block_precond_us": round(t_pc * 1e6, 2),
               "block_precond_GBps_algorithmic": round(pc_gbs, 1),
               "copy_probe_GBps": round(cpeak, 1), "material_form": form,
               "material_rows": pal_rows}
    if t_b4_pal is not None:
        kernels["blocks4_matvec_palette_us"] = round(t_b4_pal * 1e6, 2)
    if args.matvec_only:
        print(json.dumps({"roofline": roof, "kernels": kernels}), flush=True)
        ctx.close()
        return

    # ---- CPU oracle sample (before the GPU steps: it needs no GPU state) ----
    cpu = None
    if not args.no_cpu and not fcc:
        t_mv_cpu, t_pc_cpu, cdims = cpu_sample(n, kap_mv, C21, rho, delta)
        cpu = (t_mv_cpu, t_pc_cpu, cdims)
        log(f"oracle sample on {cdims}: matvec {t_mv_cpu:.2f} s, preconditioner "
            f"{t_pc_cpu:.2f} s ({time.perf_counter() - T_START:.0f} s elapsed)")
    del C21, rho

    # ---- the timed steps: groups of path points, blocked ----
    G = max(1, args.group)
    groups = [kappas[g:g + G] for g in range(0, len(kappas), G)]
    ng = len(groups)
    budget = args.budget

    def left():
        return budget - (time.perf_counter() - T_START)

    def run_group(g):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, st = ctx.band_path(groups[g], nev, blocked=True, opts=opts)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ev, st

    warm_done, t_est = 0, None
    for w in range(args.warmup):
        if t_est is not None and left() < t_est * (args.steps + 1.5):
            log(f"warmup {w}: skipped (budget: {left():.0f} s left)")
            break
        dt, _, st = run_group(w % ng)
        t_est = dt if t_est is None else max(t_est, dt)
        warm_done += 1
        log(f"warmup {w} (group {w % ng}): {dt:.2f} s")
    times = [[] for _ in range(ng)]
    evs = [None] * ng
    stats = [None] * ng
    done = 0
    t_timed = 0.0
    for k in range(args.steps):
        g = k % ng
        est = t_est if t_est is not None else 0.0
        if done > 0 and left() < 1.2 * est:
            log(f"step {k}: not started (budget: {left():.0f} s left, a step takes ~{est:.1f} s)")
            break
        dt, ev, st = run_group(g)
        t_est = dt if t_est is None else max(t_est, dt)
        t_timed += dt
        times[g].append(dt)
        evs[g], stats[g] = ev, st
        done += 1
        log(f"step {k} (group {g}): {dt:.2f} s, solves {st.op_applies}, pcg avg "
            f"{st.pcg_avg:.1f} ({time.perf_counter() - T_START:.0f} s elapsed)")
    timed_groups = [g for g in range(ng) if times[g]]
    mean_g = {g: sum(times[g]) / len(times[g]) for g in timed_groups}
    if len(timed_groups) == ng:
        path_s = sum(mean_g.values())
        path_note = "sum over the path's groups of their mean step times"
    else:
        path_s = ng * sum(mean_g.values()) / len(timed_groups)
        path_note = (f"only {len(timed_groups)} of {ng} groups timed: their mean step time "
                     f"times {ng}")
    pcg_total = sum(stats[g].pcg_iters_total for g in timed_groups)
    solves = sum(stats[g].op_applies for g in timed_groups)
    pts_timed = sum(len(groups[g]) for g in timed_groups)
    ms_step = 1e3 * t_timed / max(1, done)
    out = {
        "metric": "block matvec GB/s (% HBM peak) + Bloch-path s at n=128, vs full-space, 1 GPU",
        "value": round(path_s, 3), "unit": "s", "n_gpus": 1, "steps": done,
        "warmup": warm_done, "ms_per_step": round(ms_step, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl}{'' if args.first <= 0 else f' (first {len(kappas)} points)'}, "
                               f"{nev} lowest eigenpairs per k, 4 parity blocks with "
                               "certified merge, shift-invert Lanczos + FFT-preconditioned PCG, "
                               f"complex128; one step = {G} path points in lockstep",
                   "n": n, "nk": len(kappas), "nev": nev, "tol": 1e-12, "tol_inner": 1e-12,
                   **({"lattice": "fcc", "supersample": 4} if fcc else {"radius": 0.35, "seed": 0}),
                   "points_per_step": G, "blocks_per_launch": 1 if args.serial_blocks else 4},
        "value_is": f"seconds for the {len(kappas)}-point path: {path_note}",
        "requested": {"steps": args.steps, "warmup": args.warmup, "budget_s": budget},
        "group_mean_s": [round(mean_g[g], 3) if g in mean_g else None for g in range(ng)],
        "solves_per_point": round(solves / max(1, pts_timed), 2),
        "pcg_avg": round(pcg_total / max(1, solves), 2),
        "pcg_max": max(stats[g].pcg_iters_max for g in timed_groups),
        "max_rel_resid": max(stats[g].max_rel_resid for g in timed_groups),
        "kernels": kernels,
        "roofline": roof,
    }
    # ---- blocked vs full space on the same GPU: the first group, if the budget allows ----
    if args.full_every > 0 and 0 in mean_g:
        need = 3.2 * mean_g[0] + 5.0
        if left() > need:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            evf, stf = ctx.band_path(groups[0], nev, blocked=False)
            torch.cuda.synchronize()
            t_f = time.perf_counter() - t0
            diff = float(np.max(np.abs(evs[0] - evf) / np.abs(evf)))
            log(f"group 0 ({len(groups[0])} points): full space {t_f:.2f} s, blocked "
                f"{mean_g[0]:.2f} s, max rel diff {diff:.2e}")
            out["vs_full_space"] = {
                "k_points": len(groups[0]), "full_space_s": round(t_f, 3),
                "blocked_s": round(mean_g[0], 3), "blocked_speedup": round(t_f / mean_g[0], 3),
                "max_rel_diff_eigenvalues": diff, "full_pcg_avg": round(stf.pcg_avg, 2),
                "full_solves": stf.op_applies, "blocked_solves": stats[0].op_applies}
        else:
            log(f"full-space comparison skipped: {left():.0f} s left, needs ~{need:.0f} s")
            out["vs_full_space"] = {"skipped": f"budget ({left():.0f} s left, ~{need:.0f} s needed)"}
    ctx.close()
    if cpu is not None:
        t_mv_cpu, t_pc_cpu, cdims = cpu
        iters_path = pcg_total * len(kappas) / max(1, pts_timed)
        est = iters_path * (t_mv_cpu + t_pc_cpu)
        out["cpu_baseline"] = {
            "value": round(est, 1), "unit": "s", "cores": 1, "kind": "oracle",
            "extrapolated": True,
            "sample": (f"oracle (numpy, one thread) on a {cdims[0]}x{cdims[1]}x{cdims[2]} grid "
                       f"(a block's node count at n={n}): one operator application "
                       f"{t_mv_cpu:.2f} s + one FFT preconditioner application {t_pc_cpu:.2f} s "
                       f"(median of 3), times the {iters_path:.0f} block PCG iterations of the "
                       f"GPU path over {len(kappas)} points; Krylov and orthogonalisation work "
                       "not counted")}
    out["wall_s"] = round(time.perf_counter() - T_START, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
