"""Autotuner for the operator's accuracy/speed parameters.

Picks ES support W, uv tile T and work-item size for a given problem: every
candidate is built, timed on grid + degrid of the resident data, and its error
is measured against a reference computed on the same GPU in FP64 mode (support
13, relative error ~1e-12 against the direct sum; FP64 plans serve grid and
degrid up to 4096^2 images, one band at a time); the fastest candidate whose
dirty-image and degrid errors both stay within the budget wins.  The grid
oversampling is fixed at 2 (the FFTs are power-of-two only).

    python -m paper_2101_08072_amd.tune --workload batched-8x4096 --out tune.json

writes the choice and the candidate table as JSON (the benchmark can load it).
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

from .plan import Options, Plan


def _rel(a: torch.Tensor, b: torch.Tensor) -> float:
    a = torch.view_as_real(a) if a.is_complex() else a
    b = torch.view_as_real(b) if b.is_complex() else b
    return float(torch.linalg.vector_norm((a.double() - b.double()).ravel())
                 / torch.linalg.vector_norm(b.double().ravel()))


def _time(fn, reps):
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def autotune(prob, err_budget: float = 3e-6, supports=(6, 7, 8), tiles=(16, 32), chunks=(0,),
             reps: int = 3, seed: int = 0, device="cuda"):
    """Returns (best Options, table of candidates).  `prob` is a synth.Problem."""
    gen = torch.Generator(device=device).manual_seed(seed)
    ref_plan = Plan.from_problem(prob, device=device, options=Options(precision="fp64", band_batch=1))
    vis64 = torch.complex(torch.randn((prob.n_row, prob.n_chan), generator=gen, device=device, dtype=torch.float64),
                          torch.randn((prob.n_row, prob.n_chan), generator=gen, device=device, dtype=torch.float64))
    x64 = torch.randn((prob.n_band, prob.nx, prob.ny), generator=gen, device=device, dtype=torch.float64)
    dirty_ref = ref_plan.grid(vis64)
    degrid_ref = ref_plan.degrid(x64)
    torch.cuda.synchronize()
    del ref_plan
    torch.cuda.empty_cache()
    vis, x = vis64.to(torch.complex64), x64.float()
    table = []
    for W, T, K in itertools.product(supports, tiles, chunks):
        opt = Options(precision="fp32", support=W, tile=T, chunk=K)
        try:
            plan = Plan.from_problem(prob, device=device, options=opt)
        except Exception as exc:  # an invalid combination for this problem
            table.append(dict(support=W, tile=T, chunk=K, error=str(exc)))
            continue
        d, v = plan.image(), plan.vis()
        t_grid = _time(lambda: plan.grid(vis, out=d), reps)
        t_degrid = _time(lambda: plan.degrid(x, out=v), reps)
        e_grid, e_degrid = _rel(d, dirty_ref), _rel(v, degrid_ref)
        table.append(dict(support=W, tile=T, chunk=K, grid_ms=t_grid, degrid_ms=t_degrid,
                          err_grid=e_grid, err_degrid=e_degrid,
                          ok=bool(e_grid <= err_budget and e_degrid <= err_budget)))
        del plan, d, v
        torch.cuda.empty_cache()
    ok = [r for r in table if r.get("ok")]
    if not ok:
        raise RuntimeError(f"no candidate meets the error budget {err_budget}: {table}")
    best = min(ok, key=lambda r: r["grid_ms"] + r["degrid_ms"])
    return Options(precision="fp32", support=best["support"], tile=best["tile"], chunk=best["chunk"]), table


def main(argv=None):
    import argparse
    import json
    import sys
    import os
    ap = argparse.ArgumentParser(prog="python -m paper_2101_08072_amd.tune")
    ap.add_argument("--workload", default="batched-8x4096")
    ap.add_argument("--budget", type=float, default=3e-6)
    ap.add_argument("--supports", default="6,7,8")
    ap.add_argument("--tiles", default="16,32")
    ap.add_argument("--chunks", default="0")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth
    prob = synth.workload(a.workload)
    ints = lambda t: tuple(int(v) for v in t.split(","))  # noqa: E731
    best, table = autotune(prob, err_budget=a.budget, supports=ints(a.supports), tiles=ints(a.tiles),
                           chunks=ints(a.chunks))
    rec = {"workload": a.workload, "err_budget": a.budget,
           "choice": {"support": best.support, "tile": best.tile, "chunk": best.chunk}, "candidates": table}
    text = json.dumps(rec, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()
