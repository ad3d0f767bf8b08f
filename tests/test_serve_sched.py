"""Continuous-batching scheduler (host logic) on a virtual-clock fake executor."""
from paper_2101_08072_amd.serve import FakeExecutor, JobSpec, Scheduler, latency_summary, poisson_jobs

GB = 1 << 30


def _ex(**kw):
    return FakeExecutor(bytes_fn=lambda s: s.nx * GB // 1024, work_fn=lambda s: s.n_vis * 1e-8, **kw)


def test_budget_never_exceeded_and_all_jobs_finish():
    jobs = poisson_jobs(60, rate_hz=50.0, seed=3, sides=(512, 1024, 2048), vis_range=(1e5, 1e7))
    ex = _ex()
    seen = []
    sch = Scheduler(ex, hbm_budget=4 * GB, max_slots=6)
    res = sch.run(jobs, on_tick=lambda s: seen.append(s.used))
    assert len(res) == 60
    assert max(seen) <= 4 * GB and sch.peak_used <= 4 * GB
    assert sch.used == 0 and not sch.active
    summ = latency_summary(res)
    assert summ["p99_s"] >= summ["p50_s"] > 0


def test_admission_is_continuous_not_batch_synchronous():
    """A job arriving while others run is admitted as soon as memory allows, before
    the running ones finish."""
    jobs = [JobSpec(0, 0.0, 1024, 1, 10_000_000), JobSpec(1, 0.01, 1024, 1, 10_000_000)]
    ex = _ex()
    Scheduler(ex, hbm_budget=3 * GB, max_slots=4).run(jobs)
    order = [(k, j) for k, j, _ in ex.log]
    assert order.index(("start", 1)) < order.index(("finish", 0))


def test_fifo_blocks_and_backfill_admits_smaller_jobs():
    jobs = [JobSpec(0, 0.0, 2048, 1, 5_000_000), JobSpec(1, 0.001, 2048, 1, 1_000_000),
            JobSpec(2, 0.002, 512, 1, 1_000_000)]
    ex = _ex()
    Scheduler(ex, hbm_budget=3 * GB, max_slots=4, backfill=False).run(jobs)
    starts = [j for k, j, _ in ex.log if k == "start"]
    assert starts == [0, 1, 2]
    t_start = {j: t for k, j, t in ex.log if k == "start"}
    t_fin = {j: t for k, j, t in ex.log if k == "finish"}
    assert t_start[2] >= t_fin[0]                 # 2 waited behind 1 in strict FIFO
    ex2 = _ex()
    Scheduler(ex2, hbm_budget=3 * GB, max_slots=4, backfill=True).run(jobs)
    t_start2 = {j: t for k, j, t in ex2.log if k == "start"}
    t_fin2 = {j: t for k, j, t in ex2.log if k == "finish"}
    assert t_start2[2] < t_fin2[0]                # the small job backfilled


def test_oversized_job_rejected_and_failing_start_releases_nothing():
    jobs = [JobSpec(0, 0.0, 4096, 1, 1000), JobSpec(1, 0.0, 512, 1, 1000), JobSpec(2, 0.0, 512, 1, 1000)]
    ex = _ex(fail_ids={2})
    sch = Scheduler(ex, hbm_budget=1 * GB, max_slots=4)
    res = sch.run(jobs)
    assert sch.rejected == [0]
    assert [f[0] for f in sch.failed] == [2]
    assert [r.job_id for r in res] == [1]
    assert sch.used == 0
