"""GPU parity at the full workload sizes (FP32 path, the launch configuration the
benchmark times), on outputs the FP64 oracle computes one at a time.

* single-band-2048: 2048^2 image, 6.4e7 visibilities (the benchmark workload)
* precision-4096:   4096^2 image, 2.56e8 visibilities
* batched-8x4096:   8 bands of 4096^2 in one launch, 2.56e8 visibilities with
                    uneven per-band flag fractions

Sampled: dirty image R^dagger Sigma^-1 V at random pixels, degridded visibilities
R x of a point-source sky at random active visibilities, and the Hessian of a
sparse sky at random pixels, each within rel-l2 1e-5 of the oracle.  On the
two 4096^2 workloads the uv coverage leaves most tiles and tile rows empty, so
the occupancy pruning of the transforms is exercised at its real shape.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, make_plan, rel, say

pytestmark = pytest.mark.gpu

SAMPLES = {  # pixels, visibilities, point sources
    "single-band-2048": (12, 96, 24),
    "precision-4096": (6, 64, 12),
    "batched-8x4096": (8, 64, 16),
}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", list(SAMPLES))
def test_full_size_sampled(name):
    import torch
    n_pix, n_vis, n_src = SAMPLES[name]
    say(f"full size {name}: building the workload")
    prob = synth.workload(name)
    P = prob.n_band * prob.nx * prob.ny
    rng = np.random.default_rng(210)
    plan = make_plan(prob, "fp32")
    inf = plan.info()
    say(f"full size {name}: {inf['n_vis_active']} active visibilities, {inf['n_wplanes_max']} w-planes, "
        f"occupied tiles {inf['occ_tiles']}")

    # dirty image of seeded visibilities
    g = torch.Generator(device="cuda").manual_seed(211)
    vis = torch.randn((prob.n_row, prob.n_chan), dtype=torch.complex64, device="cuda", generator=g)
    pix = rng.integers(0, P, n_pix)
    d = plan.grid(vis).reshape(-1)[torch.as_tensor(pix, device="cuda")].cpu().numpy()
    vis_host = vis.cpu().numpy()
    del vis
    e = rel(d, oracle.grid(prob, vis_host, pix=pix))
    say(f"full size {name}: dirty image at {n_pix} pixels, rel-l2 {e:.2e}")
    assert e < TOL["fp32"]
    del vis_host

    # degrid and Hessian of sparse skies
    x = np.zeros((prob.n_band, prob.nx, prob.ny))
    x.ravel()[rng.integers(0, P, n_src)] = rng.uniform(0.1, 1.0, n_src)
    xd = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    active = np.flatnonzero(prob.effective_weight().ravel())
    sel = rng.choice(active, n_vis, replace=False)
    v = plan.degrid(xd).reshape(-1)[torch.as_tensor(sel, device="cuda")].cpu().numpy()
    e = rel(v, oracle.degrid(prob, x, sel=sel))
    say(f"full size {name}: degrid at {n_vis} visibilities, rel-l2 {e:.2e}")
    assert e < TOL["fp32"]
    h = plan.hessian(xd).reshape(-1)[torch.as_tensor(pix, device="cuda")].cpu().numpy()
    e = rel(h, oracle.hessian(prob, x, pix=pix))
    say(f"full size {name}: Hessian at {n_pix} pixels, rel-l2 {e:.2e}")
    assert e < TOL["fp32"]
