"""pfb_plan_count_static: the counting pass of plan set-up in the library's fixed
device buffer, for callers that cannot allocate device memory.

Called through the C ABI (the binding's count_scratch="static"), it must give the
same plan and bit-for-bit the same operator results as pfb_plan_count with a
caller buffer: on two calls in a row, the second on a smaller problem (the fixed
buffer still holds the first call's counts), and it must refuse a plan whose
counting pass needs more than the buffer holds.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import host, say, to_dev

pytestmark = pytest.mark.gpu


def _same_results(prob, seed):
    import torch
    from paper_2101_08072_amd import Plan
    a = Plan.from_problem(prob, count_scratch="static")
    b = Plan.from_problem(prob)
    ia, ib = a.info(), b.info()
    assert ia == ib
    rng = np.random.default_rng(seed)
    vis = to_dev(rng.normal(size=(prob.n_row, prob.n_chan)) + 1j * rng.normal(size=(prob.n_row, prob.n_chan)),
                 torch.complex64)
    x = to_dev(rng.normal(size=(prob.n_band, prob.nx, prob.ny)), torch.float32)
    for name, fa, fb in (("dirty", a.grid(vis), b.grid(vis)), ("hessian", a.hessian(x), b.hessian(x)),
                         ("degrid", a.degrid(x), b.degrid(x)), ("psf", a.make_psf(), b.make_psf())):
        ha, hb = host(fa), host(fb)
        assert np.isfinite(ha).all() and np.abs(ha).max() > 0, name
        assert np.array_equal(ha, hb), name
    say(f"static count: {prob.n_band} band(s) {prob.nx}x{prob.ny}, {ia['n_vis_active']} visibilities, "
        f"{ia['n_entries']} entries: identical plans and results")


def test_static_count_matches_caller_buffer_twice_second_smaller():
    big = synth.tiny_problem(seed=synth.SEED_BASE + 40, nx=128, ny=128, n_row=4096, n_band=2,
                             freqs=(1.0e9, 1.05e9, 1.1e9, 1.15e9), flag_frac=0.1)
    small = synth.tiny_problem(seed=synth.SEED_BASE + 41, nx=64, ny=32, n_row=700, flag_frac=0.05)
    _same_results(big, 1)
    _same_results(small, 2)


def test_static_count_refuses_plans_beyond_its_buffer():
    from paper_2101_08072_amd import Options, Plan, _lib
    # 8-cell tiles of a 8192^2 grid (1M tiles) times ~20 w base planes need ~170 MB of counters
    prob = synth.tiny_problem(seed=synth.SEED_BASE + 42, nx=4096, ny=4096, n_row=200, cell_arcsec=2.0)
    with pytest.raises(_lib.PfbError) as exc:
        Plan.from_problem(prob, options=Options(tile=8), count_scratch="static")
    assert exc.value.status == -2 and "fixed buffer" in str(exc.value)
