#!/usr/bin/env python3
"""Throughput of the pfb-clean hot path on one MI355X.

One step = one pass of the whole hot path over the resident synthetic data of
the workload (Bester et al. 2021, Section 2):
    I^d   = R^dagger Sigma^-1 V        (dirty image: grid)
    V_mod = R x                        (model visibilities: degrid)
    H x   = R^dagger Sigma^-1 R x      (exact Hessian, eq. 3)
    x    <- prox(x - gamma U^-1 (I^psf * x - I^d)),  U = I^psf * + sigma Id
                                       (eqs. 4, 6, 8: PSF convolution + CG solve + prox)
Each step therefore grids and degrids the active visibilities twice; the value
is that visibility count per second (grid+degrid visibilities/s).  The timed
steps replay one HIP graph holding the whole step (--no-graph: eager launches);
per-kernel times come from the same number of eager steps with HIP events.

Prints ONE JSON line.  Plan creation (bucketing), PSF formation and the
Lipschitz estimate happen before the timed region and are reported apart.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid+degrid visibilities/s at rel-ℓ₂ 1e-5; batched vs plain Hessian apps/s"
PEAK = {"hbm_GBps": 8000.0, "fp32_vector_TFLOPs": 157.3, "fp32_matrix_TFLOPs": 157.3, "fp64_vector_TFLOPs": 78.6}
# The FP32 vector figure counts packed FP32 (two lanes per instruction); every kernel
# here is built without packed FP32, so its vector issue peak is half of it.
FP32_VECTOR_UNPACKED_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched-8x4096")
    ap.add_argument("--cg-iters", type=int, default=20)
    ap.add_argument("--support", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--tuned", default=os.path.join(ROOT, "profiles", "autotune_{workload}.json"),
                    help="autotuner record whose choice (support, tile, chunk) the FP32 plan uses when "
                         "the command line leaves them at 0 (see paper_2101_08072_amd.tune)")
    ap.add_argument("--no-fp64-baseline", action="store_true")
    ap.add_argument("--no-band-batch-compare", action="store_true",
                    help="skip timing the Hessian with one band per launch (FP32)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of one HIP graph per step")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target oracle CPU time")
    ap.add_argument("--traffic-file", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 3 times (HBM counter calibration) and exit")
    ap.add_argument("--write-traffic", nargs=4, default=None,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE csv output of this bench "
                         "and of --copy-calibration into per-launch HBM bytes in --traffic-file")
    ap.add_argument("--copy-mib", type=int, default=2048, help="size used with --copy-calibration")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# algorithmic work per kernel launch (for the roofline fraction)
# ---------------------------------------------------------------------------

def kernel_models(info, prob, M, W, csz, rsz):
    """Algorithmic bytes (HBM-bound passes) or flops (ALU-bound spread/interp)
    per launch, from the method's data structures moved once each."""
    nx, ny = prob.nx, prob.ny
    gx = info["grid_x"]
    T = info["tile"]
    nwt = info["n_wplanes_total"]          # w-planes summed over bands
    P = prob.n_band * nx * ny
    spread_flops = M * (4.0 * W ** 3 + 60.0 * W)
    return {
        # ES spread / interpolation: W^3 complex*real multiply-adds + 3W kernel values per visibility
        "spread_kernel": ("alu", spread_flops),
        "spread_run_kernel": ("alu", spread_flops),
        # same algorithmic work, computed as FP32 matrix products on the matrix cores
        "spread_mfma_kernel": ("mfma", spread_flops),
        "interp_kernel": ("alu", spread_flops),     # FP64 mode
        "interp4_kernel": ("alu", spread_flops),    # FP32
        # row inverse DFT of every w-plane: read its occupied tiles (the rest of the
        # plane is zero), write the cropped rows of tile rows that hold them
        "g1_rows_kernel": ("hbm", (info["occ_tiles"] * T * T + info["occ_tile_rows"] * T * ny) * csz),
        # column passes (plane loop inside): per column and plane two N-point FFTs
        # (N = gx / 2, 5 N log2 N flops each) and about 24 N flops of twiddles, the
        # even/odd combination and the w-phase product (its sincos not counted)
        "wgrid_cols_kernel": ("alu", nwt * ny * (10.0 * (gx // 2) * math.log2(gx // 2) + 24.0 * (gx // 2))),
        "wdegrid_cols_kernel": ("alu", nwt * ny * (10.0 * (gx // 2) * math.log2(gx // 2) + 24.0 * (gx // 2))),
        # forward row DFT: read the cropped rows of tile rows the interpolation
        # reaches, write the tiles it reads
        "d3_rows_kernel": ("hbm", (info["need_tile_rows"] * T * ny + info["need_tiles"] * T * T) * csz),
    }


def kernel_source_sha():
    # the kernels and the device headers they are built from
    h = hashlib.sha256()
    for name in ("pfb_kernels.hip", "pfb_device.h", "pfb_kernels.h"):
        h.update(open(os.path.join(ROOT, "paper_2101_08072_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def copy_calibration(mib):
    """A plain device-to-device copy of known size, the yardstick for the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * 2 ** 20 // 4
    src = torch.empty(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4}), flush=True)


def _pmc_rows(d, counter):
    """(kernel name, value) per dispatch from rocprofv3's counter_collection csv files."""
    import csv
    import glob
    rows = []
    for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(fn, newline="") as f:
            for r in csv.DictReader(f):
                r = {k.lower(): v for k, v in r.items()}
                if r.get("counter_name") == counter:
                    rows.append((r["kernel_name"], float(r["counter_value"])))
    if not rows:
        raise SystemExit(f"no {counter} rows under {d}")
    return rows


def _base_name(full):
    m = re.search(r"pfb::(\w+)", full)
    return m.group(1) if m else None


def write_traffic(dirs, workload, copy_mib, path, min_dispatches):
    """Per-launch HBM bytes of every library kernel, from one FETCH_SIZE and one
    WRITE_SIZE pass (KiB per dispatch), each scaled by what the same counter
    reads for a plain copy of copy_mib MiB.  A kernel's figure is the mean over
    its template instances that ran at least min_dispatches times (those run in
    every step), each instance averaged over its dispatches."""
    fetch, write, cfetch, cwrite = (_pmc_rows(d, c) for d, c in
                                    zip(dirs, ("FETCH_SIZE", "WRITE_SIZE", "FETCH_SIZE", "WRITE_SIZE")))
    nbytes = copy_mib * 2 ** 20

    def copy_factor(rows):
        vals = [v for k, v in rows if "copy" in k.lower()]
        return nbytes / (max(vals) * 1024.0)

    f_fetch, f_write = copy_factor(cfetch), copy_factor(cwrite)
    out = {}
    for key, rows, fac in (("fetch", fetch, f_fetch), ("write", write, f_write)):
        per_inst = {}
        for k, v in rows:
            per_inst.setdefault(k, []).append(v * 1024.0 * fac)
        for k, vals in per_inst.items():
            b = _base_name(k)
            if b is None or len(vals) < min_dispatches:
                continue
            e = out.setdefault(b, {"instances": {}})
            e["instances"].setdefault(k, {})[key] = sum(vals) / len(vals)
            e["instances"][k]["dispatches"] = len(vals)
    for b, e in out.items():
        inst = [v for v in e["instances"].values() if "fetch" in v and "write" in v]
        e["fetch_bytes_per_launch"] = sum(v["fetch"] for v in inst) / len(inst)
        e["write_bytes_per_launch"] = sum(v["write"] for v in inst) / len(inst)
        e["bytes_per_launch"] = e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]
        e["source_sha"] = kernel_source_sha()
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    rec["copy_calibration"] = {"bytes": nbytes, "fetch_factor": f_fetch, "write_factor": f_write}
    rec[workload] = out
    with open(path, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    log(f"wrote {path}: copy factors fetch {f_fetch:.4f} write {f_write:.4f}")


def traffic_for(kernel, workload, path):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, if it was taken
    on the current kernel source."""
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    entry = rec.get(workload, {}).get(kernel)
    if not entry or entry.get("source_sha") != kernel_source_sha():
        return None
    return entry.get("bytes_per_launch")


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample of the same workload
# ---------------------------------------------------------------------------

def cpu_baseline(prob, vis_host, x_host, M, target_s):
    import oracle
    oracle.build()
    nth = oracle.threads()
    P = prob.nx * prob.ny
    rng = np.random.default_rng(7)
    # grid: whole batches of `nth` pixels (one per thread) against all visibilities
    t0 = time.perf_counter()
    oracle.grid(prob, vis_host, pix=rng.integers(0, P, nth))
    tp = time.perf_counter() - t0
    npix = nth * max(1, min(256, int(0.6 * target_s / max(tp, 1e-3))))
    pix = rng.integers(0, P, npix)
    t0 = time.perf_counter()
    oracle.grid(prob, vis_host, pix=pix)
    tg = time.perf_counter() - t0
    # degrid: visibilities (parallel over visibilities) against the image x
    active = np.flatnonzero(prob.effective_weight().ravel())
    t0 = time.perf_counter()
    oracle.degrid(prob, x_host, sel=active[:4 * nth])
    tp = time.perf_counter() - t0
    nvis = 4 * nth * max(1, min(4096, int(0.4 * target_s / max(tp, 1e-3))))
    sel = rng.choice(active, nvis, replace=False)
    t0 = time.perf_counter()
    oracle.degrid(prob, x_host, sel=sel)
    td = time.perf_counter() - t0
    t_grid_full = tg / npix * P
    t_degrid_full = td / nvis * M
    t_step = 2.0 * (t_grid_full + t_degrid_full)   # grid+degrid twice per step (FB part neglected)
    return {"value": 2.0 * M / t_step, "unit": "visibilities/s", "cores": nth, "kind": "oracle",
            "sample": (f"FP64 direct sum: grid of {npix} random pixels x {M} visibilities "
                       f"({tg:.1f} s) and degrid of {nvis} random visibilities x the "
                       f"{int(np.count_nonzero(x_host))} non-zero pixels of x ({td:.1f} s), scaled to "
                       f"the full step (2 grids + 2 degrids of all {M} visibilities; the FFT-based "
                       f"FB/CG part is not counted)"),
            "seconds": round(tg + td, 2)}


# ---------------------------------------------------------------------------

def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has "
              f"no multi-GPU path: bands would be sharded across GPUs with no exchange.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.write_traffic:
        write_traffic(args.write_traffic, args.workload, args.copy_mib, args.traffic_file,
                      args.steps + args.warmup)
        return
    import torch

    import synth
    from paper_2101_08072_amd import Options, Plan

    dev = "cuda"
    log(f"workload {args.workload}: generating inputs")
    prob = synth.workload(args.workload)
    n_vis = prob.n_row * prob.n_chan
    x_true = synth.extended_sky(synth.SEED_BASE, prob.n_band, prob.nx, prob.ny)

    tuned = None
    tuned_path = args.tuned.format(workload=args.workload)
    if not (args.support or args.tile or args.chunk) and os.path.exists(tuned_path):
        with open(tuned_path) as f:
            rec = json.load(f)
        if rec.get("workload") == args.workload:
            tuned = rec["choice"]
            args.support, args.tile, args.chunk = tuned["support"], tuned["tile"], tuned["chunk"]
            log(f"autotuned options from {tuned_path}: {tuned}")
    opts = Options(precision="fp32", support=args.support, tile=args.tile, chunk=args.chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = Plan.from_problem(prob, device=dev, options=opts)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan.info()
    M = int(info["n_vis_active"])
    log(f"plan: {plan_s:.2f} s, info {info}")

    xg = torch.as_tensor(x_true, device=dev).contiguous()
    vis = plan.degrid(xg)                      # resident synthetic visibilities V = R x_true
    t0 = time.perf_counter()
    plan.make_psf(want_image=False)
    torch.cuda.synchronize()
    psf_s = time.perf_counter() - t0
    v0 = torch.ones_like(xg)
    lam_max = plan.power_iteration(v0, 20)
    torch.cuda.synchronize()
    lam_max = float(lam_max.max().item())
    sigma, gamma, lam = 1e-3 * lam_max, 1.0, 1e-3

    dirty = plan.image()
    vmod = plan.vis()
    hx = plan.image()
    xk = torch.zeros_like(xg)

    def step():
        plan.grid(vis, out=dirty)
        plan.degrid(xg, out=vmod)
        plan.hessian(xg, out=hx)
        plan.fb_step(dirty, xk, sigma, gamma, lam, args.cg_iters)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    run = step
    if not args.no_graph:
        # the whole step as one HIP graph (same kernels, no launch gaps between them);
        # eager launches if the capture is refused
        try:
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                step()
            torch.cuda.synchronize()
            run = graph.replay
            for _ in range(args.warmup):
                run()
            torch.cuda.synchronize()
        except RuntimeError as exc:
            log(f"graph capture failed ({exc}); timing eager launches")
            torch.cuda.synchronize()
            run = step
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = 2.0 * M / (ms_step * 1e-3)
    used_graph = run is not step
    log(f"step {ms_step:.3f} ms (wall {wall / args.steps * 1e3:.3f} ms, {'graph' if run is not step else 'eager'}); "
        f"{value:.4g} vis/s")
    # per-kernel times: the same steps launched eagerly with HIP events around every kernel
    plan.profile(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = plan.profile_report()
    plan.profile(False)

    # per-operator times (separate short loops, HIP events on the same stream)
    def timed(fn, n=3):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    breakdown = {
        "grid": timed(lambda: plan.grid(vis, out=dirty)),
        "degrid": timed(lambda: plan.degrid(xg, out=vmod)),
        "hessian": timed(lambda: plan.hessian(xg, out=hx)),
        "psf_conv": timed(lambda: plan.psf_conv(xg, out=hx)),
        "cg_solve": timed(lambda: plan.precond_solve(dirty, sigma, args.cg_iters, out=hx)),
    }
    breakdown["fb_step"] = ms_step - breakdown["grid"] - breakdown["degrid"] - breakdown["hessian"]

    # backward step of eq. 7 with the regulariser of eq. 9 (outside the step above, which
    # keeps the Euclidean l1 prox): primal-dual iterations with the Dirac + db1-6
    # dictionary at 3 levels and the PSF metric; per-kernel times from the same profiler
    prox_levels, prox_iters = 3, 10
    prox_ws = plan.prox_workspace(7)
    xp = plan.image()
    lam_prox = 1e-3 * float(dirty.abs().max().item())
    plan.prox(dirty, xp, prox_ws, lam_prox, gamma, sigma, 1.05 * lam_max, 1, 7, prox_levels)
    breakdown["prox_iteration"] = timed(lambda: plan.prox(dirty, xp, prox_ws, lam_prox, gamma, sigma, 1.05 * lam_max,
                                                          prox_iters, 7, prox_levels), n=2) / prox_iters
    plan.profile(True)
    plan.prox(dirty, xp, prox_ws, lam_prox, gamma, sigma, 1.05 * lam_max, prox_iters, 7, prox_levels)
    torch.cuda.synchronize()
    prox_prof = plan.profile_report()
    plan.profile(False)
    # pfb-clean with the exact gradient: 8 forward-backward steps (the paper's Cygnus A run
    # used eight gradient evaluations), each one Hessian, a 20-step CG and 10 primal-dual steps
    n_major = 8
    xc = torch.zeros_like(xp)
    a_ev, b_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a_ev.record()
    plan.clean(dirty, xc, prox_ws, sigma, gamma, lam_prox, 1.05 * lam_max, args.cg_iters, prox_iters, n_major, 7,
               prox_levels)
    b_ev.record()
    torch.cuda.synchronize()
    clean_out = {"n_major": n_major, "ms": round(a_ev.elapsed_time(b_ev), 2), "hessian_applications": n_major,
                 "cg_iters": args.cg_iters, "pd_iters": prox_iters, "nbasis": 7, "levels": prox_levels}
    log("clean:", json.dumps(clean_out))
    del prox_ws
    grid_degrid_vis_s = M / ((breakdown["grid"] + breakdown["degrid"]) * 1e-3)
    hess_apps = 1e3 / breakdown["hessian"]
    # PSF convolution (eq. 4) and one CG step (eq. 8) against HBM: algorithmic bytes of
    # the three-pass zero-padded FFT convolution, 48 B per pixel and band (x read, the
    # row spectrum written and read twice, the PSF spectrum read, y written), and for a
    # CG step that plus 36 B per pixel of vector updates
    Pb = prob.n_band * prob.nx * prob.ny

    def hbm(bytes_, ms):
        ach = bytes_ / (ms * 1e-3) / 1e9
        return {"bytes": bytes_, "ms": round(ms, 4), "achieved_GBps": round(ach, 1),
                "frac": round(ach / PEAK["hbm_GBps"], 4)}
    psf_hbm = hbm(48 * Pb, breakdown["psf_conv"])
    cg_hbm = hbm(84 * Pb, breakdown["cg_solve"] / max(args.cg_iters, 1))

    # dominant kernel and its roofline
    W = info["support"]
    models = kernel_models(info, prob, M, W, 8, 4)
    name, (n_launch, tot_ms) = max(prof.items(), key=lambda kv: kv[1][1])
    avg_ms = tot_ms / n_launch
    roof = None
    if name in models:
        bound, work = models[name]
        if bound == "hbm":
            ach = work / (avg_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK["hbm_GBps"], "unit": "GB/s",
                    "frac": round(ach / PEAK["hbm_GBps"], 4)}
        else:
            ach = work / (avg_ms * 1e-3) / 1e12
            peak = PEAK["fp32_matrix_TFLOPs"] if bound == "mfma" else PEAK["fp32_vector_TFLOPs"]
            roof = {"bound": bound, "achieved": round(ach, 3), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(ach / peak, 4)}
            if bound == "alu":
                roof["frac_of_unpacked_fp32"] = round(ach / FP32_VECTOR_UNPACKED_TFLOPS, 4)
        roof["kernel"] = name
        roof["avg_ms"] = round(avg_ms, 4)
        roof["launches_per_step"] = n_launch / args.steps
        roof["traffic"] = traffic_for(name, args.workload, args.traffic_file)
    kernels = {k: {"launches_per_step": n / args.steps, "ms_per_step": round(t / args.steps, 4)}
               for k, (n, t) in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    # every modelled kernel against its own bound (same event timings)
    for k, (n, t) in prof.items():
        if k in models and n:
            bound, work = models[k]
            a_ms = t / n
            if bound == "hbm":
                ach = work / (a_ms * 1e-3) / 1e9
                kernels[k].update(bound="hbm", achieved_GBps=round(ach, 1),
                                  frac=round(ach / PEAK["hbm_GBps"], 4))
            else:
                ach = work / (a_ms * 1e-3) / 1e12
                peak = PEAK["fp32_matrix_TFLOPs"] if bound == "mfma" else PEAK["fp32_vector_TFLOPs"]
                kernels[k].update(bound=bound, achieved_TFLOPs=round(ach, 3), frac=round(ach / peak, 4))
                if bound == "alu":
                    kernels[k]["frac_of_unpacked_fp32"] = round(ach / FP32_VECTOR_UNPACKED_TFLOPS, 4)
    log("kernels:", json.dumps(kernels))

    # backward step: per-kernel ms per primal-dual iteration; the wavelet levels against
    # HBM with algorithmic bytes = one read and one write of every level block, six
    # wavelet bases, analysis and synthesis each
    rsz = 4
    blk = sum(prob.n_band * (prob.nx >> l) * (prob.ny >> l) for l in range(prox_levels))
    level_bytes = 6 * 2 * blk * rsz
    prox_k = {k: {"launches_per_iteration": n / prox_iters, "ms_per_iteration": round(t / prox_iters, 4)}
              for k, (n, t) in sorted(prox_prof.items(), key=lambda kv: -kv[1][1])}
    for k in ("wavelet_ana2_kernel", "wavelet_syn2_kernel"):
        if k in prox_k:
            ach = level_bytes / (prox_k[k]["ms_per_iteration"] * 1e-3) / 1e9
            prox_k[k].update(bound="hbm", achieved_GBps=round(ach, 1), frac=round(ach / PEAK["hbm_GBps"], 4))
    prox_out = {"ms_per_iteration": round(breakdown["prox_iteration"], 4), "nbasis": 7, "levels": prox_levels,
                "kernels": prox_k}
    log("prox:", json.dumps(prox_out))

    # sampled parity against the FP64 oracle at the full size (every band sampled)
    parity = None
    vis_host = None
    if not args.no_parity or not args.no_cpu_baseline:
        vis_host = vis.cpu().numpy()
    if not args.no_parity:
        import oracle
        rng = np.random.default_rng(3)
        P = prob.nx * prob.ny
        pix = np.concatenate([b * P + rng.integers(0, P, 16) for b in range(prob.n_band)])
        plan.grid(vis, out=dirty)
        d = dirty.cpu().numpy().ravel()[pix]
        d_ref = oracle.grid(prob, vis_host, pix=pix)
        active = np.flatnonzero(prob.effective_weight().ravel())
        sel = rng.choice(active, 128, replace=False)
        v_ref = oracle.degrid(prob, x_true.astype(np.float64), sel=sel)
        xs = np.zeros_like(x_true)
        for b in range(prob.n_band):
            xs[b].ravel()[rng.integers(0, P, 40)] = rng.uniform(0.1, 1.0, 40)
        hs = plan.hessian(torch.as_tensor(xs, device=dev)).cpu().numpy().ravel()[pix]
        hs_ref = oracle.hessian(prob, xs, pix=pix)
        parity = {"dirty_image": oracle.rel_l2(d, d_ref), "degrid": oracle.rel_l2(vis_host.ravel()[sel], v_ref),
                  "hessian": oracle.rel_l2(hs, hs_ref),
                  "sample": f"16 random pixels per band ({pix.size} in all: dirty image, Hessian of a "
                            f"40-source sparse sky per band), 128 random visibilities (degrid)"}
        log("parity", parity)

    # the FP32 Hessian of x_true for the precision comparison, then free the batched plan
    h32_host = plan.hessian(xg, out=hx).double().cpu().numpy()
    graph = None
    del plan, step, run, graph, vis, dirty, vmod, hx, xk, xp, xc
    import gc
    gc.collect()
    torch.cuda.empty_cache()

    # plain per-band FP64 path on the same GPU (Hessian applications/s): one band per
    # launch (band_batch = 1), everything in FP64 with W = 13
    plain = None
    if not args.no_fp64_baseline:
        try:
            p64 = Plan.from_problem(prob, device=dev, options=Options(precision="fp64", band_batch=1))
            x64 = xg.double()
            h64 = p64.image()
            t64 = timed(lambda: p64.hessian(x64, out=h64), n=2)
            i64 = p64.info()
            plain = {"precision": "fp64", "support": i64["support"], "tile": i64["tile"], "band_batch": 1,
                     "hessian_ms": round(t64, 3), "hessian_apps_per_s": round(1e3 / t64, 3),
                     "speedup_batched_fp32_over_plain_fp64": round(t64 / breakdown["hessian"], 2)}
            b64 = h64.cpu().numpy()
            plain["fp32_vs_fp64_hessian_rel_l2"] = float(np.linalg.norm(h32_host - b64) / np.linalg.norm(b64))
            log("plain fp64", plain)
            del p64, x64, h64
        except Exception as exc:  # report, do not hide
            plain = {"error": str(exc)}
        torch.cuda.empty_cache()

    # all bands in one launch vs one band per launch (same FP32 kernels)
    per_band = None
    if not args.no_band_batch_compare and prob.n_band > 1:
        pb = Plan.from_problem(prob, device=dev, options=Options(precision="fp32", band_batch=1,
                                                                 support=args.support, tile=args.tile))
        hb = pb.image()
        t_pb = timed(lambda: pb.hessian(xg, out=hb), n=2)
        per_band = {"hessian_ms": round(t_pb, 3), "hessian_apps_per_s": round(1e3 / t_pb, 3),
                    "batched_speedup": round(t_pb / breakdown["hessian"], 3)}
        del pb, hb
        torch.cuda.empty_cache()
        log("one band per launch", per_band)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, vis_host, x_true.astype(np.float64), M, args.cpu_seconds)
        log("cpu", cpu)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "visibilities/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "hip_graph": used_graph,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded VLA-like earth-rotation uvw, 10% flags, 500 points + 20 blobs)",
        "config": {"workload": args.workload, "nx": prob.nx, "ny": prob.ny, "n_band": prob.n_band,
                   "n_row": prob.n_row, "n_chan": prob.n_chan, "visibilities": n_vis,
                   "active_visibilities": M, "cg_iters": args.cg_iters, "support": W,
                   "tile": info["tile"], "w_planes": info["n_wplanes_max"], "oversample": 2.0,
                   "autotuned": tuned},
        "roofline": roof,
        "cpu_baseline": cpu,
        "grid_degrid_vis_per_s": round(grid_degrid_vis_s, 1),
        "hessian_apps_per_s": round(hess_apps, 3),
        "plain_fp64": plain,
        "one_band_per_launch": per_band,
        "breakdown_ms": {k: round(v, 4) for k, v in breakdown.items()},
        "psf_conv_hbm": psf_hbm,
        "cg_iteration_hbm": cg_hbm,
        "kernels": kernels,
        "prox": prox_out,
        "clean": clean_out,
        "parity_rel_l2": parity,
        "setup_s": {"plan": round(plan_s, 3), "psf": round(psf_s, 3)},
        "lambda_max": lam_max,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
