"""Serving on the GPU: jobs admitted together overlap on the device and each
job's results (dirty image, FB iterate, final Hessian) are the same alone and in
the mix."""
import numpy as np
import pytest

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def test_results_same_alone_and_in_mix():
    from paper_2101_08072_amd.serve import GpuExecutor, JobSpec, Scheduler, latency_summary
    jobs = [JobSpec(0, 0.0, 128, 1, 60_000, n_fb=3, cg_iters=5, seed=11),
            JobSpec(1, 0.0, 64, 2, 40_000, n_fb=3, cg_iters=5, seed=12),
            JobSpec(2, 0.0, 128, 2, 90_000, n_fb=3, cg_iters=5, seed=13),
            JobSpec(3, 0.0, 64, 1, 20_000, n_fb=3, cg_iters=5, seed=14)]
    alone = {}
    for j in jobs:
        ex = GpuExecutor(keep_results=True)
        Scheduler(ex, hbm_budget=64 << 30, max_slots=1).run([j])
        alone[j.job_id] = ex.outputs[j.job_id]
        say(f"alone job {j.job_id} done")
    ex = GpuExecutor(keep_results=True)
    sch = Scheduler(ex, hbm_budget=64 << 30, max_slots=4)
    res = sch.run(jobs)
    say("mix", latency_summary(res))
    first_finish = min(r.finished for r in res)
    assert all(r.admitted < first_finish for r in res)       # all four were in flight together
    for j in jobs:
        for k in ("dirty", "x", "resid"):
            a, b = alone[j.job_id][k], ex.outputs[j.job_id][k]
            den = np.linalg.norm(a.ravel()) or 1.0
            assert np.linalg.norm((a - b).ravel()) / den <= 1e-6, (j.job_id, k)
