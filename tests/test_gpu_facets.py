"""Faceting: an image as a grid of facets, each with its own plan (its own w-range of
n - 1, its own w-planes and smaller FFTs), against the un-faceted FP64 oracle.

The dirty image R^dagger Sigma^-1 V (after eq. 3), the model visibilities R x
(eq. 1) and the Hessian R^dagger Sigma^-1 R x (eq. 3) of the whole image, built
from 2 x 2 and 4 x 4 facets, match the oracle's direct sums over the whole image
within rel-l2 1e-5 (FP32 path).  The field is wide and |w| large, so the w term
matters and the facets away from the phase centre get fewer w-planes.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, host, say, to_dev

pytestmark = pytest.mark.gpu

N = 256


@pytest.fixture(scope="module")
def fc():
    prob = synth.tiny_problem(seed=synth.SEED_BASE + 50, nx=N, ny=N, n_row=2000, cell_arcsec=40.0,
                              w_frac=1.0, n_band=2, freqs=(1.0e9, 1.05e9, 1.1e9, 1.15e9), flag_frac=0.1)
    rng = np.random.default_rng(51)
    vis = rng.normal(size=(prob.n_row, prob.n_chan)) + 1j * rng.normal(size=(prob.n_row, prob.n_chan))
    x = rng.normal(size=(2, N, N))
    pix = rng.choice(2 * N * N, 512, replace=False)
    say("facets: oracle references (whole image)")
    return dict(prob=prob, vis=vis, x=x, pix=pix, dirty=oracle.grid(prob, vis), degrid=oracle.degrid(prob, x),
                hess=oracle.hessian(prob, x, pix=pix))


@pytest.mark.parametrize("nf", [2, 4])
def test_faceted_operators_match_the_unfaceted_oracle(fc, nf):
    import torch
    from paper_2101_08072_amd import Plan
    from paper_2101_08072_amd.facets import FacetedPlan
    prob = fc["prob"]
    fp = FacetedPlan.from_problem(prob, nf, nf)
    whole = Plan.from_problem(prob).info()
    inf = fp.info()
    nw = [i["n_wplanes_max"] for i in inf]
    say(f"facets {nf}x{nf}: w-planes per facet {nw} (whole image {whole['n_wplanes_max']}), grid "
        f"{inf[0]['grid_x']}^2 per facet (whole image {whole['grid_x']}^2)")
    assert max(nw) <= whole["n_wplanes_max"]
    if nf == 4:   # the outer facets span a narrower range of n - 1
        assert sum(nw) < nf * nf * whole["n_wplanes_max"]
    d = host(fp.grid(to_dev(fc["vis"], torch.complex64)))
    v = host(fp.degrid(to_dev(fc["x"], torch.float32)))
    h = host(fp.hessian(to_dev(fc["x"], torch.float32))).ravel()[fc["pix"]]
    e = (oracle.rel_l2(d, fc["dirty"]), oracle.rel_l2(v, fc["degrid"]), oracle.rel_l2(h, fc["hess"]))
    say(f"facets {nf}x{nf}: dirty {e[0]:.2e}, degrid {e[1]:.2e}, Hessian {e[2]:.2e}")
    assert max(e) < TOL["fp32"]
    w = prob.effective_weight()
    assert np.all(v[w == 0] == 0)
