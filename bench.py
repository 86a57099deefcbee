"""Benchmark: Bloch band path of the parity-blocked solver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cube|fcc] [--n N] [--nk 16] [--nev M]

Workload: two-phase unit cube, n^3 grid (default n = 128), cubic matrix
(C11=1, C12=0.4, C44=0.3, rho=1) with a centred sphere r = 0.35 holding a seeded
SPD stiffness (rho = 4); 16 points on the Gamma-X-M-Gamma-R path; the 20 lowest
eigenpairs per point; shift delta = 0.30 C_max; tolerances 1e-12.
--workload fcc: the paper's FCC cell (quartz matrix, silicon sphere, subpixel
volume-fraction material; dimensionless units) at n = 60 on the 91-point
Gamma-X-W-K-Gamma-L-U-W-L-K path with 40 eigenpairs per point.

One step = the whole hot path over the path: at every k, four parity-block
shift-invert Krylov solves advancing in lockstep (every launch covers all active
blocks: inner PCG with the FFT-diagonal preconditioner, the fused stencil
matvec, Gamma projection), merged with certification.  K steps are timed with a device synchronisation on both
sides.  The full-space form (one solve of 3n^3 unknowns per k) is then compared
with the blocked form on every fourth path point (--full-every), same GPU, same
tolerances.

Material form: the two-phase cell has two distinct (C21, rho) rows, so by
default the kernels read the palette form (one byte per node naming its row)
instead of 21 stiffness entries and rho per node; --material-form dense forces
the dense form.  Both give the same matvec bit for bit.

Also measured live: the fused matvec (A + delta M) x of the four parity blocks
in one launch (as the blocked path issues it; HIP events on the context stream),
in the form the path runs and in the other form, reported against the MI355X
HBM peak (algorithmic bytes: x, y and the material as that form stores it) as
the roofline of the dominant kernel; one
block per launch (rotating through the blocks), the full-space matvec and the
block preconditioner beside it; and the oracle (CPU) cost of the same path
estimated from a bounded sample (one oracle matvec + preconditioner application
at the same n, single-threaded, scaled by the GPU run's PCG iteration count).
"""

import argparse
import json
import os
import sys
import time

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
    p.add_argument("--study", choices=("refinement", "cells", "gap"), default=None,
                   help="refinement: grid-refinement errors of the FCC workload at X, W and L "
                        "against a 256^3 blocked reference (one JSON line)")
    p.add_argument("--workload", choices=("cube", "fcc"), default="cube",
                   help="cube: the two-phase unit cube (default); fcc: the paper's quartz/Si "
                        "FCC cell on its 91-point path")
    p.add_argument("--n", type=int, default=0, help="grid size (default 128 cube, 60 fcc)")
    p.add_argument("--nk", type=int, default=16, help="path points (cube workload)")
    p.add_argument("--nev", type=int, default=0, help="eigenpairs per k (default 20 cube, 40 fcc)")
    p.add_argument("--first", type=int, default=0,
                   help="time only the first m points of the path (short profiled runs)")
    p.add_argument("--full-every", type=int, default=4,
                   help="compare with the full space on every k-th path point (0: skip)")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle sample")
    p.add_argument("--matvec-only", action="store_true",
                   help="only the matvec timing (for hardware-counter runs)")
    p.add_argument("--mv-iters", type=int, default=100)
    p.add_argument("--material-form", choices=("auto", "dense"), default="auto",
                   help="auto: the kernels read the material's palette form when it has one "
                        "(at most 256 distinct rows); dense: always the 21 + 1 doubles per node")
    p.add_argument("--serial-blocks", action="store_true",
                   help="solve the four blocks one after another instead of in lockstep")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_timing(torch, ctx, n, kappa, delta, iters, blocks, op):
    """Average duration (s) of one launch of `op` ("apply": the fused matvec
    (A + delta M) x; "precond": the FFT preconditioner) over `iters` launches that
    rotate through `blocks`, so that consecutive launches touch different data and
    the 256 MB last-level cache cannot serve a repeated block.  HIP events are
    recorded on torch's current stream, which is the stream the context launches
    on."""
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
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for t in range(iters):
        launch(t)
    e.record()
    torch.cuda.synchronize()
    del xs, ys
    return s.elapsed_time(e) / 1e3 / iters


def blocks_timing(torch, ctx, n, kappa, delta, iters):
    """Average duration (s) of one launch applying (A + delta M) to all four
    parity blocks (pbr_apply_blocks); HIP events on torch's current stream, the
    stream the context launches on.  The four blocks' stiffness alone (352 MB at
    n=128) exceeds the 256 MB last-level cache."""
    from synth import complex_gaussian
    x = torch.from_numpy(complex_gaussian(3 * n ** 3, seed=12345)).cuda()
    y = torch.zeros_like(x)
    for _ in range(5):
        ctx.apply_blocks(kappa, delta, x, y)
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(iters):
        ctx.apply_blocks(kappa, delta, x, y)
    e.record()
    torch.cuda.synchronize()
    del x, y
    return s.elapsed_time(e) / 1e3 / iters


def copy_peak(torch, nbytes=2 << 30, iters=20):
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(iters):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    t = s.elapsed_time(e) / 1e3 / iters
    del a, b
    return 2 * nbytes / t / 1e9


def cpu_sample(n, kappa, C21, rho, delta, A_lat=None):
    """Oracle (as written) cost of one PCG iteration's operator work at this n:
    one matvec (index formula) and one preconditioner application (numpy.fft),
    both in the full space, which is how the oracle evaluates a block too."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import fourier as F, pointwise as P
    from synth import complex_gaussian
    x = complex_gaussian(3 * n ** 3, seed=12345)
    Cref, rref = F.reference_material(C21, rho)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        y = P.apply_A(x, (n, n, n), kappa, C21, rho, s=delta, A_lat=A_lat)
        t1 = time.perf_counter()
        z = F.precond_fft(y, (n, n, n), kappa, -1, Cref, rref, delta, A_lat)
        t2 = time.perf_counter()
    assert np.isfinite(z).all()
    return t1 - t0, t2 - t1


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


def refinement_study(grids=(16, 32, 64, 128), ref=256, nev=8, points=("X", "W", "L")):
    """Relative eigenvalue errors of the FCC workload on coarser grids against the
    blocked solve at ref^3, and the observed orders log2(e_n / e_2n)."""
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
            ev, st = ctx.eigs_merged(tuple(fcc_point(p)), nev)
            vals[(n, p)] = np.asarray(ev)
            log(f"refinement n={n} {p}: {np.round(ev[:4], 6)} ({time.perf_counter() - t0:.0f} s)")
        ctx.close()
        torch.cuda.empty_cache()
    err = {p: {n: float(np.max(np.abs(vals[(n, p)] - vals[(ref, p)]) / vals[(ref, p)]))
               for n in grids} for p in points}
    order = {p: {f"{a}->{b}": round(float(np.log2(err[p][a] / err[p][b])), 3)
                 for a, b in zip(grids[:-1], grids[1:])} for p in points}
    return {"study": "grid refinement, FCC quartz/Si cell, blocked solves, max relative "
                     f"error of the {nev} lowest eigenvalues vs {ref}^3",
            "reference_n": ref, "grids": list(grids), "max_rel_error": err,
            "observed_order": order, "seconds": round(time.perf_counter() - t0, 1)}


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


def cells_study(nk, nev, count=8, seed=0):
    """Uneven batch of two-phase cells (n drawn from {64, 96, 128}, inclusion
    radius from U[0.2, 0.4], each with its own seeded inclusion stiffness): the
    blocked band paths of all cells one after another, then all cells at once
    (pbr_band_paths: one host thread and stream per cell).  Results must agree
    bit for bit."""
    import numpy as np
    import torch
    from paper_2606_03599_amd import pbr
    from synth import batch_cells, sc_path
    cells = batch_cells(count, seed=seed)
    kappas, _ = sc_path(nk)
    ctxs = []
    for n, r, C21, rho in cells:
        ctx = pbr.Context((n, n, n))
        ctx.set_material(torch.from_numpy(C21).cuda(), torch.from_numpy(rho).cuda())
        ctxs.append(ctx)
    sizes = [c[0] for c in cells]
    radii = [round(c[1], 4) for c in cells]
    del cells
    log(f"cells: n = {sizes}, radius = {radii}, {nk} k-points, nev = {nev}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    serial = []
    for q, ctx in enumerate(ctxs):
        serial.append(ctx.band_path(kappas, nev)[0])
        log(f"cell {q} (n={sizes[q]}) one after another: {time.perf_counter() - t0:.1f} s")
    t_serial = time.perf_counter() - t0
    t0 = time.perf_counter()
    conc, sts = pbr.band_paths(ctxs, [kappas] * len(ctxs), nev)
    t_conc = time.perf_counter() - t0
    log(f"all cells at once: {t_conc:.1f} s (one after another {t_serial:.1f} s)")
    same = all(np.array_equal(a, b) for a, b in zip(serial, conc))
    for ctx in ctxs:
        ctx.close()
    return {"study": "uneven batch of cells, blocked band paths, one after another vs all cells "
                     "at once (pbr_band_paths)",
            "cells": [{"n": n, "radius": r} for n, r in zip(sizes, radii)],
            "k_points": nk, "nev": nev,
            "one_after_another_s": round(t_serial, 3), "concurrent_s": round(t_conc, 3),
            "speedup": round(t_serial / t_conc, 3),
            "solves": int(sum(s.op_applies for s in sts)),
            "results_identical": bool(same)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU: collectives and sharding are "
                                   "not part of it, so --gpus must be 1"}))
        sys.exit(2)
    if args.study == "refinement":
        print(json.dumps(refinement_study()), flush=True)
        return
    if args.study == "gap":
        print(json.dumps(gap_gradient_study(args.n if args.n > 0 else 256,
                                            args.nev if args.nev > 0 else 30)), flush=True)
        return
    if args.study == "cells":
        print(json.dumps(cells_study(args.nk if args.nk != 16 else 6,
                                     args.nev if args.nev > 0 else 16)), flush=True)
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

    # ---- matvec roofline (dominant kernel), live HIP-event timing ----
    t_b4 = blocks_timing(torch, ctx, n, kap_mv, delta, max(10, args.mv_iters // 2))
    t_b4_other = None
    if pal_rows > 0:  # the other form of the same launch, for comparison
        ctx.set_palette(form == "dense")
        t_b4_other = blocks_timing(torch, ctx, n, kap_mv, delta, max(10, args.mv_iters // 2))
        ctx.set_palette(form == "palette")
    t_blk = kernel_timing(torch, ctx, n, kap_mv, delta, args.mv_iters, (0, 1, 2, 3), "apply")
    t_full = kernel_timing(torch, ctx, n, kap_mv, delta, max(8, args.mv_iters // 4), (-1,),
                           "apply")
    t_pc = kernel_timing(torch, ctx, n, kap_mv, delta, max(8, args.mv_iters // 2), (0, 1, 2, 3),
                         "precond")
    nb = n ** 3 // 4
    bpn = PAL_BYTES_PER_NODE if form == "palette" else BYTES_PER_NODE
    b4_bytes = bpn * 4 * nb
    b4_gbs = b4_bytes / t_b4 / 1e9
    blk_bytes = bpn * nb
    blk_gbs = blk_bytes / t_blk / 1e9
    full_gbs = bpn * n ** 3 / t_full / 1e9
    pc_gbs = PRECOND_BYTES_PER_NODE * nb / t_pc / 1e9
    cpeak = copy_peak(torch)
    if t_b4_other is not None:
        log(f"4-block matvec launch, other material form: {t_b4_other*1e6:.1f} us")
    log(f"4-block matvec launch {t_b4*1e6:.1f} us = {b4_gbs:.0f} GB/s; one block "
        f"{t_blk*1e6:.1f} us = {blk_gbs:.0f} GB/s; full {t_full*1e6:.1f} us = "
        f"{full_gbs:.0f} GB/s; block preconditioner {t_pc*1e6:.1f} us; copy {cpeak:.0f} GB/s")
    rec = traffic_record(os.path.join(ROOT, "paper_2606_03599_amd", "csrc", "stencil.hip"),
                         f"matvec_blocks_n{n}_{form}_traffic")
    roof = {"bound": "hbm", "achieved": round(b4_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(b4_gbs / HBM_PEAK_GBS, 4),
            "traffic": (None if rec is None else rec["hbm_bytes_per_launch"]),
            "kernel": "apply_stream_kernel: fused (A + delta M) x of the four parity blocks "
                      f"in one launch (as the blocked path runs it), {form} material form "
                      f"({bpn} algorithmic bytes per node)",
            "algorithmic_bytes": b4_bytes, "avg_launch_us": round(t_b4 * 1e6, 2)}
    kernels = {"blocks4_matvec_us": round(t_b4 * 1e6, 2), "blocks4_matvec_GBps": round(b4_gbs, 1),
               "blocks4_matvec_frac_copy": round(b4_gbs / cpeak, 4),
               "block_matvec_us": round(t_blk * 1e6, 2), "block_matvec_GBps": round(blk_gbs, 1),
               "block_matvec_frac_copy": round(blk_gbs / cpeak, 4),
               "full_matvec_us": round(t_full * 1e6, 2), "full_matvec_GBps": round(full_gbs, 1),
               "full_matvec_frac_hbm": round(full_gbs / HBM_PEAK_GBS, 4),
               "block_precond_us": round(t_pc * 1e6, 2),
               "block_precond_GBps_algorithmic": round(pc_gbs, 1),
               "copy_peak_GBps": round(cpeak, 1), "material_form": form,
               "material_rows": pal_rows}
    if t_b4_other is not None:
        obpn = BYTES_PER_NODE if form == "palette" else PAL_BYTES_PER_NODE
        ogbs = obpn * 4 * nb / t_b4_other / 1e9
        other = "dense" if form == "palette" else "palette"
        kernels[f"blocks4_matvec_{other}_us"] = round(t_b4_other * 1e6, 2)
        kernels[f"blocks4_matvec_{other}_GBps"] = round(ogbs, 1)
        kernels[f"blocks4_matvec_{other}_frac_hbm"] = round(ogbs / HBM_PEAK_GBS, 4)
    if args.matvec_only:
        print(json.dumps({"roofline": roof, "kernels": kernels}), flush=True)
        ctx.close()
        return

    # ---- the timed steps: blocked band path ----
    for w in range(args.warmup):
        log(f"warmup {w}")
        ctx.band_path(kappas, nev, blocked=True, opts=opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev, st = ctx.band_path(kappas, nev, blocked=True, opts=opts)
        log(f"step {k}: {st.seconds:.2f} s, op_applies {st.op_applies}, pcg avg {st.pcg_avg:.1f}")
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / max(1, args.steps)
    out = {
        "metric": "block matvec GB/s (% HBM peak) + Bloch-path s at n=128, vs full-space, 1 GPU",
        "value": round(t_step, 3), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_step * 1e3, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl}{'' if args.first <= 0 else f' (first {len(kappas)} points)'}, "
                               f"{nev} lowest eigenpairs per k, 4 parity blocks with "
                               "certified merge, shift-invert Lanczos + FFT-preconditioned PCG, "
                               "complex128", "n": n, "nk": len(kappas), "nev": nev,
                   "tol": 1e-12, "tol_inner": 1e-12,
                   **({"lattice": "fcc", "supersample": 4} if fcc else {"radius": 0.35, "seed": 0}),
                   "blocks_per_launch": 1 if args.serial_blocks else 4},
        "kernels": kernels,
        "pcg_avg": round(st.pcg_avg, 2), "pcg_max": st.pcg_iters_max,
        "op_applies": st.op_applies, "outer_restarts": st.outer_iters,
        "max_rel_resid": st.max_rel_resid,
        "roofline": roof,
    }
    # ---- blocked vs full space on the same GPU, on every full_every-th k-point ----
    if args.full_every > 0:
        sub = kappas[::args.full_every]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evb, stb = ctx.band_path(sub, nev, blocked=True, opts=opts)
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
        t0 = time.perf_counter()
        evf, stf = ctx.band_path(sub, nev, blocked=False)
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t0
        diff = float(np.max(np.abs(evb - evf) / np.abs(evf)))
        log(f"{len(sub)} k-points: full space {t_f:.2f} s, blocked {t_b:.2f} s, "
            f"max rel diff {diff:.2e}")
        out["vs_full_space"] = {
            "k_points": len(sub), "full_space_s": round(t_f, 3), "blocked_s": round(t_b, 3),
            "blocked_speedup": round(t_f / t_b, 3), "max_rel_diff_eigenvalues": diff,
            "full_pcg_avg": round(stf.pcg_avg, 2), "full_op_applies": stf.op_applies,
            "blocked_op_applies": stb.op_applies}
    ctx.close()
    # ---- CPU oracle baseline (bounded sample, scaled to the path) ----
    if not args.no_cpu:
        t_mv_cpu, t_pc_cpu = cpu_sample(n, kap_mv, C21, rho, delta, A_lat)
        iters = st.pcg_iters_total
        est = iters * (t_mv_cpu + t_pc_cpu)
        out["cpu_baseline"] = {
            "value": round(est, 1), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"one oracle matvec ({t_mv_cpu:.2f} s) + one oracle FFT preconditioner "
                       f"({t_pc_cpu:.2f} s) at n={n}, single-threaded; scaled by the {iters} PCG "
                       "iterations of the GPU blocked path (the oracle applies a block as the "
                       "full-space operator on a zero-extended vector)")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
