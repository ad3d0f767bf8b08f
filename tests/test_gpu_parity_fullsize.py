"""GPU parity at the full workload sizes (FP32 path, the launch configuration the
benchmark times), on outputs the FP64 oracle computes one at a time.

* single-band-2048: 2048^2 image, 6.4e7 visibilities (the benchmark workload)
* precision-4096:   4096^2 image, 2.56e8 visibilities
* batched-8x4096:   8 bands of 4096^2 in one launch, 2.56e8 visibilities with
                    uneven per-band flag fractions

Sampled, stratified: the dirty image R^dagger Sigma^-1 V at pixels of every band
(corners and edge midpoints, where |l|, |m| and n - 1 are largest, the phase
centre and random pixels; each band also on its own), the degridded
visibilities R x of a point-source sky at the entries with the largest |w|, the
longest baselines, negative u and v (wrapped to the far side of the periodic
uv grid) and random ones, and the Hessian of that sky at stratified pixels,
each within rel-l2 1e-5 of the oracle.  On the
two 4096^2 workloads the uv coverage leaves most tiles and tile rows empty, so
the occupancy pruning of the transforms is exercised at its real shape.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, make_plan, rel, say

pytestmark = pytest.mark.gpu

SAMPLES = {  # dirty-image pixels per band, Hessian pixels per band, visibilities, point sources
    "single-band-2048": (256, 64, 1024, 24),
    "precision-4096": (64, 32, 1024, 12),
    "batched-8x4096": (32, 8, 1024, 16),
}


def _pixels(prob, n_per_band, rng):
    """Stratified pixel sample: in every band the four corners (largest |l|, |m| and
    n - 1), the middle of each edge, the phase centre, then random pixels."""
    nx, ny = prob.nx, prob.ny
    fixed = [(0, 0), (0, ny - 1), (nx - 1, 0), (nx - 1, ny - 1), (0, ny // 2), (nx - 1, ny // 2),
             (nx // 2, 0), (nx // 2, ny - 1), (nx // 2, ny // 2)]
    out = []
    for b in range(prob.n_band):
        ij = fixed + [tuple(t) for t in np.stack([rng.integers(0, nx, n_per_band), rng.integers(0, ny, n_per_band)],
                                                 axis=1)[: n_per_band - len(fixed)]]
        out += [(b * nx + i) * ny + j for i, j in ij]
    return np.array(out, dtype=np.int64)


def _visibilities(prob, n, rng):
    """Stratified visibility sample: the largest |w|, the longest baselines, entries with
    u < 0 and v < 0 (they wrap to the far side of the periodic uv grid), then random."""
    w = prob.effective_weight()
    rr, cc = np.nonzero(w)
    flat = rr * prob.n_chan + cc
    s = prob.freq[cc] / synth.C_LIGHT
    u, v, ww = prob.uvw[rr, 0] * s, prob.uvw[rr, 1] * s, prob.uvw[rr, 2] * s
    k = n // 8
    pick = [flat[np.argsort(-np.abs(ww))[:k]], flat[np.argsort(-np.hypot(u, v))[:k]],
            rng.choice(flat[(u < 0) & (v < 0)], k, replace=False)]
    rest = rng.choice(flat, n, replace=False)
    sel = np.unique(np.concatenate(pick + [rest]))
    return sel[:n] if sel.size >= n else sel


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", list(SAMPLES))
def test_full_size_sampled(name):
    import torch
    n_pix, n_hpix, n_vis, n_src = SAMPLES[name]
    say(f"full size {name}: building the workload")
    prob = synth.workload(name)
    P = prob.n_band * prob.nx * prob.ny
    rng = np.random.default_rng(210)
    plan = make_plan(prob, "fp32")
    inf = plan.info()
    say(f"full size {name}: {inf['n_vis_active']} active visibilities, {inf['n_wplanes_max']} w-planes, "
        f"occupied tiles {inf['occ_tiles']}")

    # dirty image of seeded visibilities, every band sampled
    g = torch.Generator(device="cuda").manual_seed(211)
    vis = torch.randn((prob.n_row, prob.n_chan), dtype=torch.complex64, device="cuda", generator=g)
    pix = _pixels(prob, n_pix, rng)
    d = plan.grid(vis).reshape(-1)[torch.as_tensor(pix, device="cuda")].cpu().numpy()
    vis_host = vis.cpu().numpy()
    del vis
    d_ref = oracle.grid(prob, vis_host, pix=pix)
    e = rel(d, d_ref)
    say(f"full size {name}: dirty image at {pix.size} pixels, rel-l2 {e:.2e}")
    assert e < TOL["fp32"]
    for b in range(prob.n_band):
        sl = slice(b * n_pix, (b + 1) * n_pix)
        assert rel(d[sl], d_ref[sl]) < TOL["fp32"], f"band {b}"
    del vis_host

    # degrid of a point-source sky at stratified visibilities, Hessian at stratified pixels
    x = np.zeros((prob.n_band, prob.nx, prob.ny))
    x.ravel()[rng.integers(0, P, n_src)] = rng.uniform(0.1, 1.0, n_src)
    for b in range(prob.n_band):   # every band holds at least one source
        x[b, rng.integers(0, prob.nx), rng.integers(0, prob.ny)] = 0.5
    xd = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    sel = _visibilities(prob, n_vis, rng)
    v = plan.degrid(xd).reshape(-1)[torch.as_tensor(sel, device="cuda")].cpu().numpy()
    e = rel(v, oracle.degrid(prob, x, sel=sel))
    say(f"full size {name}: degrid at {sel.size} visibilities, rel-l2 {e:.2e}")
    assert e < TOL["fp32"]
    hpix = _pixels(prob, n_hpix, rng)
    h = plan.hessian(xd).reshape(-1)[torch.as_tensor(hpix, device="cuda")].cpu().numpy()
    e = rel(h, oracle.hessian(prob, x, pix=hpix))
    say(f"full size {name}: Hessian at {hpix.size} pixels, rel-l2 {e:.2e}")
    assert e < TOL["fp32"]
