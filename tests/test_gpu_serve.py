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
        sch = Scheduler(ex, hbm_budget=64 << 30, max_slots=1)
        sch.run([j])
        assert not sch.failed, sch.failed
        alone[j.job_id] = ex.outputs[j.job_id]
        say(f"alone job {j.job_id} done")
    ex = GpuExecutor(keep_results=True)
    sch = Scheduler(ex, hbm_budget=64 << 30, max_slots=4)
    res = sch.run(jobs)
    assert not sch.failed, sch.failed
    say("mix", latency_summary(res))
    first_finish = min(r.finished for r in res)
    assert all(r.admitted < first_finish for r in res)       # all four were in flight together
    for j in jobs:
        for k in ("dirty", "x", "resid"):
            a, b = alone[j.job_id][k], ex.outputs[j.job_id][k]
            den = np.linalg.norm(a.ravel()) or 1.0
            assert np.linalg.norm((a - b).ravel()) / den <= 1e-6, (j.job_id, k)


def test_served_job_matches_the_oracle():
    """One job through the scheduler (set-up on its worker thread) against the FP64
    oracle run on the same synthetic inputs: the dirty image (after eq. 3), the FB
    iterate after its steps (eqs. 4, 6, 8, l1 prox) with sigma from the oracle's own
    per-band power iteration, and the final Hessian (eq. 3) of the oracle's iterate
    against the served one, at sampled pixels."""
    import oracle
    import synth
    from paper_2101_08072_amd.serve import GpuExecutor, JobSpec, Scheduler
    spec = JobSpec(0, 0.0, 128, 2, 60_000, n_fb=3, cg_iters=5, seed=21)
    ex = GpuExecutor(keep_results=True)
    sch = Scheduler(ex, hbm_budget=64 << 30)
    sch.run([spec])
    assert not sch.failed and len(sch.results) == 1, sch.failed
    o = ex.outputs[0]
    n_chan = o["freq"].size
    prob = synth.Problem(uvw=o["uvw"], freq=o["freq"], weight=o["weight"], flag=o["flag"],
                         chan_band=synth.contiguous_bands(n_chan, 2), n_band=2, nx=128, ny=128,
                         cellx=o["cell"], celly=o["cell"])
    rng = np.random.default_rng(5)
    pix = rng.choice(2 * 128 * 128, 256, replace=False)
    dirty = oracle.grid(prob, o["vis"])
    e_dirty = oracle.rel_l2(o["dirty"].ravel()[pix], dirty.ravel()[pix])
    psf = oracle.psf(prob)
    lam = max(oracle.power_iteration(lambda v, b=b: oracle.psf_conv(psf[b:b + 1], v[None])[0],
                                     np.ones((128, 128)), 15)[0] for b in range(2))
    x = np.zeros((2, 128, 128))
    for _ in range(spec.n_fb):
        x = oracle.fb_step(psf, dirty, x, 1e-3 * lam, 1.0, 1e-3, spec.cg_iters)
    e_x = oracle.rel_l2(o["x"], x)
    e_h = oracle.rel_l2(o["resid"].ravel()[pix], oracle.hessian(prob, x, pix=pix))
    say(f"served job vs oracle: dirty {e_dirty:.2e}, FB iterate {e_x:.2e}, final Hessian {e_h:.2e}")
    assert e_dirty < 1e-5
    assert e_x < 1e-4 and e_h < 1e-4
