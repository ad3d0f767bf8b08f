"""Serving: continuous batching of imaging jobs on one GPU.

A job is one pfb-clean run on its own data (Bester et al. 2021, Sec. 2): dirty
image and PSF, power iteration for the step size, `n_fb` forward-backward
iterations with PSF-approximate gradients and CG preconditioner solves (eqs. 4,
6, 8 + prox), then one exact Hessian for the final residual gradient (eq. 3).

The scheduler admits queued jobs whenever a slot and enough of the HBM budget
are free (not only when a batch finishes), keeps each admitted job's
visibilities, weights, PSF spectrum and iterates resident, and advances every
active job by one stage per tick.  On the GPU each job runs on its own stream,
so the kernels of different jobs overlap on the device; the host never waits
for a job — completion is polled with events — and a job's set-up (input
generation and plan creation, which reads uvw and the bucket counts back on the
host) runs on a worker thread, so admissions do not stall the other jobs.  The
slot count defaults to the device's four hardware queues.

The scheduling core (`Scheduler`) is independent of the executor, so the
admission logic is tested on the CPU with a fake executor.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable

import numpy as np


@dataclasses.dataclass
class JobSpec:
    job_id: int
    arrival: float            # seconds since the start of the stream
    nx: int
    n_band: int
    n_vis: int                # visibilities (rows x channels) before flagging
    n_fb: int = 10
    cg_iters: int = 20
    seed: int = 0


@dataclasses.dataclass
class JobResult:
    job_id: int
    arrival: float
    admitted: float
    finished: float
    bytes: int
    n_vis_active: int
    passes: int               # grid/degrid passes over the visibilities

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Scheduler:
    """Continuous-batching admission by HBM budget and slots.

    executor interface:
      estimate(spec) -> bytes                 (upper bound the job will hold)
      start(spec) -> handle                   (allocates, enqueues the first stage)
      advance(handle) -> bool                 (enqueue next stage; True when all enqueued)
      done(handle) -> bool                    (all enqueued work finished)
      finish(handle) -> (n_vis_active, passes) and release memory
      now() -> float
    """

    def __init__(self, executor, hbm_budget: int, max_slots: int = 4, backfill: bool = True):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.backfill = backfill
        self.used = 0
        self.peak_used = 0
        self.active = {}          # job_id -> (spec, handle, bytes, admitted, fully_enqueued)
        self.results: list[JobResult] = []
        self.rejected: list[int] = []
        self.failed: list[tuple[int, str]] = []

    def _admit(self, queue: list[JobSpec]):
        i = 0
        while i < len(queue) and len(self.active) < self.max_slots:
            spec = queue[i]
            need = self.ex.estimate(spec)
            if need > self.budget:
                self.rejected.append(spec.job_id)        # can never fit
                queue.pop(i)
                continue
            if self.used + need <= self.budget:
                queue.pop(i)
                try:
                    handle = self.ex.start(spec)
                except Exception as exc:                  # a job that cannot start frees its slot
                    self.failed.append((spec.job_id, str(exc)))
                    continue
                self.used += need
                self.peak_used = max(self.peak_used, self.used)
                self.active[spec.job_id] = [spec, handle, need, self.ex.now(), False]
                continue
            if not self.backfill:
                break                                     # strict FIFO: wait for memory
            i += 1                                        # let a smaller later job in

    def run(self, jobs: list[JobSpec], on_tick: Callable | None = None) -> list[JobResult]:
        pending = sorted(jobs, key=lambda j: j.arrival)
        queue: list[JobSpec] = []
        t0 = self.ex.now()
        while pending or queue or self.active:
            now = self.ex.now() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.pop(0))
            self._admit(queue)
            progressed = False
            for jid in list(self.active):
                spec, handle, need, admitted, enq = self.active[jid]
                if not enq:
                    try:
                        self.active[jid][4] = self.ex.advance(handle)
                    except Exception as exc:              # set-up or a stage failed: free the slot
                        self.failed.append((jid, str(exc)))
                        self.used -= need
                        del self.active[jid]
                    progressed = True
                elif self.ex.done(handle):
                    n_act, passes = self.ex.finish(handle)
                    self.used -= need
                    self.results.append(JobResult(jid, spec.arrival + t0, admitted, self.ex.now(), need,
                                                  n_act, passes))
                    del self.active[jid]
                    progressed = True
            if on_tick:
                on_tick(self)
            if not progressed:
                self.ex.idle(pending[0].arrival + t0 if pending else None)
        return self.results


def latency_summary(results: list[JobResult]) -> dict:
    lat = np.array([r.latency for r in results])
    span = max(r.finished for r in results) - min(r.arrival for r in results)
    vis = sum(r.n_vis_active * r.passes for r in results)
    return {"jobs": len(results), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "makespan_s": float(span),
            "vis_per_s": float(vis / span) if span > 0 else float("nan")}


def poisson_jobs(n: int, rate_hz: float, seed: int = 7, sides=(512, 1024, 2048, 4096),
                 vis_range=(1e5, 1e8), max_band: int = 8, n_fb: int = 10, cg_iters: int = 20) -> list[JobSpec]:
    """Poisson arrivals; side uniform over `sides`, visibilities log-uniform, bands 1..max_band."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    lo, hi = math.log(vis_range[0]), math.log(vis_range[1])
    jobs = []
    for k in range(n):
        jobs.append(JobSpec(job_id=k, arrival=float(t[k]), nx=int(rng.choice(sides)),
                            n_band=int(rng.integers(1, max_band + 1)),
                            n_vis=int(math.exp(rng.uniform(lo, hi))), n_fb=n_fb, cg_iters=cg_iters,
                            seed=int(rng.integers(0, 2 ** 31))))
    return jobs


# ---------------------------------------------------------------------------
# executors
# ---------------------------------------------------------------------------

class FakeExecutor:
    """Virtual-clock executor for testing the scheduler on the CPU.  Each job holds
    `bytes_fn(spec)` bytes and needs `stages` advance() calls, then `work_fn(spec)`
    seconds of device time shared equally by the active jobs (processor sharing)."""

    def __init__(self, bytes_fn, work_fn, stages: int = 3, fail_ids=()):
        self.t = 0.0
        self.bytes_fn, self.work_fn, self.stages = bytes_fn, work_fn, stages
        self.jobs = {}
        self.fail_ids = set(fail_ids)
        self.log = []

    def now(self):
        return self.t

    def estimate(self, spec):
        return self.bytes_fn(spec)

    def start(self, spec):
        if spec.job_id in self.fail_ids:
            raise RuntimeError(f"job {spec.job_id} failed to start")
        h = {"spec": spec, "left": self.work_fn(spec), "stage": 0}
        self.jobs[spec.job_id] = h
        self.log.append(("start", spec.job_id, self.t))
        return h

    def advance(self, h):
        h["stage"] += 1
        return h["stage"] >= self.stages

    def done(self, h):
        return h["left"] <= 1e-12

    def finish(self, h):
        del self.jobs[h["spec"].job_id]
        self.log.append(("finish", h["spec"].job_id, self.t))
        return h["spec"].n_vis, 2

    def idle(self, until):
        # advance the virtual clock to the next completion or arrival
        running = [h for h in self.jobs.values() if h["left"] > 0]
        dt_done = min((h["left"] * len(running) for h in running), default=math.inf)
        dt_arr = (until - self.t) if until is not None else math.inf
        dt = min(dt_done, dt_arr)
        if not math.isfinite(dt):
            dt = 1e-3
        for h in running:
            h["left"] -= dt / len(running)
        self.t += max(dt, 1e-9)


class GpuExecutor:
    """Runs jobs through the C ABI, one HIP stream per job.  Inputs are generated
    on the device from the seeded earth-rotation uvw (synth) and a seeded torch
    generator for weights, flags and visibilities.  Set-up (inputs, plan) runs on
    a pool of `setup_workers` threads; the first stage waits for it without
    blocking the tick.  Large jobs keep at most `max_plane_bytes` of w-planes
    resident (the plan's band batch)."""

    def __init__(self, device="cuda", cell_fov_deg: float = 1.0, keep_results: bool = False,
                 setup_workers: int = 2, max_plane_bytes: int = 48 << 30):
        import concurrent.futures as cf
        import torch
        self.torch = torch
        dev = torch.device(device)
        self.device = torch.device("cuda", dev.index if dev.index is not None else torch.cuda.current_device())
        self.fov = cell_fov_deg
        self.keep = keep_results
        self.outputs = {}
        self.pool = cf.ThreadPoolExecutor(max_workers=setup_workers)
        self.max_plane_bytes = int(max_plane_bytes)

    def now(self):
        return time.perf_counter()

    def _shape(self, spec):
        n_chan = 16 * spec.n_band
        n_row = max(1, -(-spec.n_vis // n_chan))
        return n_row, n_chan

    def _band_batch(self, spec):
        """Bands whose w-planes are resident at once (planes + two intermediates)."""
        per_band = self._per_band_planes(spec) * 3
        return max(1, min(spec.n_band, self.max_plane_bytes // per_band))

    @staticmethod
    def _per_band_planes(spec):
        g = 2 * spec.nx
        nw = 24                                    # generous w-plane bound for a 1 degree field
        return max(nw * g * g, 4 * g * g) * 8

    def estimate(self, spec):
        """Upper bound of the device bytes of a job (inputs + workspace), from shapes."""
        n_row, n_chan = self._shape(spec)
        nv = n_row * n_chan
        nx = spec.nx
        planes = self._per_band_planes(spec) * 3 * self._band_batch(spec)  # planes + two intermediates
        recs = int(nv * 2.2) * 28 * 2              # two gridders, up to 2.2 copies per visibility
        inputs = nv * (8 + 4 + 1 + 8) + n_row * 24
        images = spec.n_band * nx * nx * 4 * 40    # images, PSF, row spectra, CG vectors
        return int(planes + recs + inputs + images + (256 << 20))

    def start(self, spec):
        """Hands the job's set-up to a worker thread; the handle's first stage waits for it."""
        stream = self.torch.cuda.Stream(device=self.device)
        return {"spec": spec, "stream": stream, "stage": -1, "setup": self.pool.submit(self._setup, spec, stream)}

    def _setup(self, spec, stream):
        import synth
        torch = self.torch
        from .plan import Options, Plan
        torch.cuda.set_device(self.device)   # the worker thread's current device
        n_row, n_chan = self._shape(spec)
        with torch.cuda.stream(stream):
            uvw = torch.as_tensor(synth.earth_rotation_uvw(synth.antenna_enu(spec.seed), n_row),
                                  device=self.device)
            freq = np.linspace(0.9e9, 1.7e9, n_chan)
            gen = torch.Generator(device=self.device).manual_seed(spec.seed)
            weight = (0.5 + torch.rand((n_row, n_chan), generator=gen, device=self.device)).contiguous()
            flag = (torch.rand((n_row, n_chan), generator=gen, device=self.device) < 0.1).to(torch.uint8)
            cell = math.radians(self.fov) / spec.nx
            plan = Plan(uvw, freq, weight, flag, synth.contiguous_bands(n_chan, spec.n_band), spec.n_band,
                        spec.nx, spec.nx, cell, cell, Options(precision="fp32", band_batch=self._band_batch(spec)))
            vis = torch.complex(torch.randn((n_row, n_chan), generator=gen, device=self.device),
                                torch.randn((n_row, n_chan), generator=gen, device=self.device)).contiguous()
            job = {"plan": plan, "vis": vis, "x": plan.image().zero_(), "n_act": plan.info()["n_vis_active"],
                   "graph": None, "uvw": uvw, "freq": freq, "weight": weight, "flag": flag, "cell": cell}
        return job

    def advance(self, job):
        torch = self.torch
        if job["stage"] < 0:
            if not job["setup"].done():
                return False                                   # set-up still running on its worker
            job.update(job.pop("setup").result())             # re-raises a set-up failure
            job["stage"] = 0
        plan, spec = job["plan"], job["spec"]
        with torch.cuda.stream(job["stream"]):
            s = job["stage"]
            if s == 0:
                job["dirty"] = plan.grid(job["vis"])
                plan.make_psf(want_image=False)
                job["lam"] = plan.power_iteration(torch.ones_like(job["dirty"]), 15)
                job["ev_lam"] = torch.cuda.Event()
                job["ev_lam"].record()
            elif s == 1:
                if not job["ev_lam"].query():
                    return False                               # step size not known yet
                lam_max = float(job["lam"].cpu().numpy().max())
                sigma = 1e-3 * lam_max
                job["graph"] = plan.fb_graph(job["dirty"], job["x"], sigma, 1.0, 1e-3, spec.cg_iters, 1)
            elif s < 2 + spec.n_fb:
                job["graph"].launch()
            else:
                job["resid"] = plan.hessian(job["x"])          # exact gradient part R^T S R x (eq. 3)
                job["ev_done"] = torch.cuda.Event()
                job["ev_done"].record()
                job["stage"] += 1
                return True
            job["stage"] += 1
        return False

    def done(self, job):
        return job["ev_done"].query()

    def finish(self, job):
        spec = job["spec"]
        if self.keep:
            out = {k: job[k].detach().cpu().numpy() for k in ("dirty", "x", "resid", "vis", "uvw", "weight", "flag")}
            out.update(freq=job["freq"], cell=job["cell"])
            self.outputs[spec.job_id] = out
        n_act = job["n_act"]
        job.clear()
        return n_act, 4        # dirty-image grid, PSF grid, Hessian degrid + grid

    def idle(self, until):
        if until is None:
            time.sleep(2e-4)
        else:
            time.sleep(max(0.0, min(until - self.now(), 2e-3)))


def main(argv=None):
    """Serving benchmark: a Poisson stream of imaging jobs through the scheduler."""
    import argparse
    import json
    ap = argparse.ArgumentParser(prog="python -m paper_2101_08072_amd.serve")
    ap.add_argument("--jobs", type=int, default=40)
    ap.add_argument("--rate", type=float, default=4.0, help="arrivals per second")
    ap.add_argument("--sides", default="512,1024,2048")
    ap.add_argument("--vis-min", type=float, default=1e5)
    ap.add_argument("--vis-max", type=float, default=2e7)
    ap.add_argument("--max-band", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--n-fb", type=int, default=10)
    ap.add_argument("--cg-iters", type=int, default=20)
    a = ap.parse_args(argv)
    jobs = poisson_jobs(a.jobs, a.rate, sides=tuple(int(s) for s in a.sides.split(",")),
                        vis_range=(a.vis_min, a.vis_max), max_band=a.max_band, n_fb=a.n_fb,
                        cg_iters=a.cg_iters)
    ex = GpuExecutor()
    sch = Scheduler(ex, hbm_budget=int(a.budget_gb * (1 << 30)), max_slots=a.slots)
    done = [0]

    def tick(s):
        if len(s.results) != done[0]:
            done[0] = len(s.results)
            r = s.results[-1]
            print(f"job {r.job_id} done: latency {r.latency:.3f} s, active {len(s.active)}, "
                  f"used {s.used / 2**30:.1f} GB", flush=True)

    res = sch.run(jobs, on_tick=tick)
    out = latency_summary(res)
    out.update({"rejected": sch.rejected, "failed": [f[0] for f in sch.failed],
                "peak_budget_gb": sch.peak_used / 2 ** 30, "config": vars(a)})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
