"""hipGraph capture of forward-backward iterations (eqs. 4, 6, 8 + prox): every
replay, with eager work and synchronisation between replays, equals the eager
iterations."""
import numpy as np
import pytest

import synth
from gpu_helpers import host, make_plan, say, to_dev

pytestmark = pytest.mark.gpu


def test_fb_graph_replays_match_eager():
    import torch
    prob = synth.tiny_problem(seed=31, nx=64, ny=64, n_row=800, cell_arcsec=20.0)
    plan = make_plan(prob, "fp32")
    plan.make_psf(want_image=False)
    rng = np.random.default_rng(32)
    vis = to_dev(rng.normal(size=(prob.n_row, prob.n_chan)) + 1j * rng.normal(size=(prob.n_row, prob.n_chan)),
                 torch.complex64)
    dirty = plan.grid(vis)
    lam_max = float(host(plan.power_iteration(torch.ones_like(dirty), 20))[0])
    sigma, gamma, lam, iters, steps = 1e-2 * lam_max, 1.0, 1e-3, 8, 3
    x0 = to_dev(np.abs(rng.normal(size=(1, 64, 64))) * 1e-3, torch.float32)
    xe = x0.clone()
    for _ in range(steps):
        plan.fb_step(dirty, xe, sigma, gamma, lam, iters)
    ref = host(xe)
    xg = x0.clone()
    say("capture")
    g = plan.fb_graph(dirty, xg, sigma, gamma, lam, iters, n_steps=steps)
    for rep in range(3):
        xg.copy_(x0)
        torch.cuda.synchronize()
        g.launch()
        got = host(xg)
        say(f"replay {rep}: max |diff| {np.abs(got - ref).max():.3g}")
        assert np.array_equal(got, ref)
        plan.psf_conv(dirty)                    # eager work between replays
        torch.cuda.synchronize()
