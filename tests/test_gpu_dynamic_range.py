"""FP32 gridding over a wide range of magnitudes, and loud failure on bad input.

The FP32 spread accumulates in 64-bit fixed point with a step set by the largest
|w V| of the call, so the dirty image (Section 2, after eq. 3) and the Hessian
(eq. 3) are checked against the FP64 oracle with every visibility scaled by
1e-20 and by 1e+18, and with one visibility 1e5 times the rest plus a few
weights 1e3 times larger.  A NaN in an unflagged visibility makes the image NaN
(never silently finite); a NaN in a flagged one is ignored; a NaN or negative
unflagged weight is refused when the plan is counted.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, host, make_plan, rel, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dr():
    prob = synth.tiny_problem(seed=synth.SEED_BASE + 30, nx=64, ny=64, n_row=2048, cell_arcsec=20.0,
                              flag_frac=0.1)
    rng = np.random.default_rng(31)
    vis = rng.normal(size=(prob.n_row, prob.n_chan)) + 1j * rng.normal(size=(prob.n_row, prob.n_chan))
    x = rng.normal(size=(1, 64, 64))
    say("dynamic range: oracle references")
    return dict(prob=prob, vis=vis, x=x, dirty=oracle.grid(prob, vis), hess=oracle.hessian(prob, x))


@pytest.mark.parametrize("scale", [1e-20, 1e18])
def test_scaled_inputs(dr, scale):
    import torch
    plan = make_plan(dr["prob"], "fp32")
    d = host(plan.grid(to_dev(dr["vis"] * scale, torch.complex64)))
    e = rel(d, dr["dirty"] * scale)
    h = host(plan.hessian(to_dev(dr["x"] * scale, torch.float32)))
    eh = rel(h, dr["hess"] * scale)
    say(f"dynamic range: scale {scale:g}: dirty {e:.2e}, Hessian {eh:.2e}")
    assert np.isfinite(d).all() and np.isfinite(h).all()
    assert e < TOL["fp32"] and eh < TOL["fp32"]


def test_one_bright_visibility_and_heavy_weights(dr):
    import torch
    prob = dr["prob"]
    on = np.flatnonzero(prob.effective_weight().ravel())
    rng = np.random.default_rng(32)
    vis = dr["vis"].copy()
    vis.ravel()[on[17]] *= 1e5
    p2 = synth.Problem(uvw=prob.uvw, freq=prob.freq, weight=prob.weight.copy(), flag=prob.flag,
                       chan_band=prob.chan_band, n_band=1, nx=prob.nx, ny=prob.ny, cellx=prob.cellx,
                       celly=prob.celly)
    heavy = rng.choice(on, 5, replace=False)
    p2.weight.ravel()[heavy] *= 1e3
    plan = make_plan(p2, "fp32")
    d = host(plan.grid(to_dev(vis, torch.complex64)))
    ref = oracle.grid(p2, vis)
    e = rel(d, ref)
    # the faint part: the image of all visibilities but the bright one
    faint = vis.copy()
    faint.ravel()[on[17]] = 0
    ef = rel(host(plan.grid(to_dev(faint, torch.complex64))), oracle.grid(p2, faint))
    say(f"dynamic range: bright visibility + heavy weights: dirty {e:.2e}, without the bright one {ef:.2e}")
    assert e < TOL["fp32"] and ef < TOL["fp32"]


def test_nan_visibility_is_loud_and_flagged_nan_is_ignored(dr):
    import torch
    prob = dr["prob"]
    plan = make_plan(prob, "fp32")
    w = prob.effective_weight().ravel()
    vis = dr["vis"].copy()
    vis.ravel()[np.flatnonzero(w == 0)[0]] = np.nan          # flagged: must not matter
    d = host(plan.grid(to_dev(vis, torch.complex64)))
    assert np.isfinite(d).all() and rel(d, dr["dirty"]) < TOL["fp32"]
    vis.ravel()[np.flatnonzero(w)[3]] = np.nan + 1j          # unflagged: must not be gridded silently
    d = host(plan.grid(to_dev(vis, torch.complex64)))
    assert np.isnan(d).all()
    # the plan stays usable
    d = host(plan.grid(to_dev(dr["vis"], torch.complex64)))
    assert rel(d, dr["dirty"]) < TOL["fp32"]


@pytest.mark.parametrize("bad", [np.nan, -1.0, np.inf])
def test_bad_unflagged_weight_refused(dr, bad):
    from paper_2101_08072_amd import _lib
    prob = dr["prob"]
    wt = prob.weight.copy()
    w = prob.effective_weight().ravel()
    wt.ravel()[np.flatnonzero(w)[5]] = bad
    p2 = synth.Problem(uvw=prob.uvw, freq=prob.freq, weight=wt, flag=prob.flag, chan_band=prob.chan_band,
                       n_band=1, nx=prob.nx, ny=prob.ny, cellx=prob.cellx, celly=prob.celly)
    with pytest.raises(_lib.PfbError) as exc:
        make_plan(p2, "fp32")
    assert exc.value.status == -1 and "weight" in str(exc.value)
    # the same value under a flag is ignored
    fl = np.zeros_like(wt, dtype=np.uint8) if prob.flag is None else prob.flag.copy()
    fl.ravel()[np.flatnonzero(w)[5]] = 1
    p3 = synth.Problem(uvw=prob.uvw, freq=prob.freq, weight=wt, flag=fl, chan_band=prob.chan_band,
                       n_band=1, nx=prob.nx, ny=prob.ny, cellx=prob.cellx, celly=prob.celly)
    make_plan(p3, "fp32")


def test_epsilon_picks_the_support(dr):
    """epsilon = 3e-6 asks for W = 8 in FP32 (tabulated 3-D kernel error 3e-7 plus the
    FP32 rounding floor of 2e-6), 1e-5 for the default W = 7; each result meets its epsilon."""
    import torch
    for eps, W in ((3e-6, 8), (1e-5, 7)):
        plan = make_plan(dr["prob"], "fp32", epsilon=eps)
        assert plan.info()["support"] == W
        d = host(plan.grid(to_dev(dr["vis"], torch.complex64)))
        e = rel(d, dr["dirty"])
        say(f"epsilon {eps:g}: W = {W}, dirty rel-l2 {e:.2e}")
        assert e < eps
