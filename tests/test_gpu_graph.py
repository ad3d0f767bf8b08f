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


def test_whole_step_graph_replays_match_eager():
    """The benchmark's step (dirty image, degrid, Hessian, one FB step) captured as
    one graph: every replay, with eager work and synchronisation between replays,
    equals the eager step bit for bit."""
    import torch
    prob = synth.tiny_problem(seed=33, nx=64, ny=64, n_row=800, cell_arcsec=20.0)
    plan = make_plan(prob, "fp32")
    plan.make_psf(want_image=False)
    rng = np.random.default_rng(34)
    vis = to_dev(rng.normal(size=(prob.n_row, prob.n_chan)) + 1j * rng.normal(size=(prob.n_row, prob.n_chan)),
                 torch.complex64)
    x = to_dev(np.abs(rng.normal(size=(1, 64, 64))), torch.float32)
    dirty, hx, xk = plan.image(), plan.image(), plan.image()
    vmod = plan.vis()
    x0 = to_dev(np.abs(rng.normal(size=(1, 64, 64))) * 1e-3, torch.float32)
    sigma, gamma, lam, iters = 1e-2, 1e-3, 1e-3, 6

    def step():
        plan.grid(vis, out=dirty)
        plan.degrid(x, out=vmod)
        plan.hessian(x, out=hx)
        plan.fb_step(dirty, xk, sigma, gamma, lam, iters)

    xk.copy_(x0)
    step()
    ref = [host(t).copy() for t in (dirty, vmod, hx, xk)]
    xk.copy_(x0)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in (dirty, hx):
            t.zero_()
        vmod.zero_()
        xk.copy_(x0)
        torch.cuda.synchronize()
        graph.replay()
        got = [host(t) for t in (dirty, vmod, hx, xk)]
        say(f"replay {rep}: max |diff| {max(float(np.abs(g - r).max()) for g, r in zip(got, ref)):.3g}")
        for g, r in zip(got, ref):
            assert np.array_equal(g, r)
        plan.psf_conv(dirty)                    # eager work between replays
        plan.degrid(x, out=vmod)
        torch.cuda.synchronize()
