"""Image sides that are even but not powers of two (the paper's Cygnus A image is
1728 x 1200, Sec. 3).  The library pads to power-of-two grids: the NUFFT grid is
the smallest power of two >= 2n per axis (oversampling 2 .. 4), the PSF
convolution's zero-padded grid likewise (a circular convolution of period >= 2n
has no wrap-around inside the n x n crop).  Every operator against the FP64
oracle, element by element, FP32 and FP64:

* 96 x 80, two bands: dirty image, degrid, Hessian, PSF, PSF convolution, CG,
  FB step, wavelet analysis (3 levels) and the primal-dual prox of eq. 7;
* 1728 x 1200: dirty image, degrid and Hessian sampled, PSF and PSF convolution
  on the whole image, 10 CG steps.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, host, make_plan, rel, say, to_dev
from oracle import wavelets as wv

pytestmark = pytest.mark.gpu


def _dt(prec):
    import torch
    return (torch.float64, torch.complex128) if prec == "fp64" else (torch.float32, torch.complex64)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_small_non_power_of_two_all_operators(prec):
    R, C = _dt(prec)
    prob = synth.tiny_problem(seed=synth.SEED_BASE + 60, nx=96, ny=80, n_row=1500, cell_arcsec=30.0,
                              n_band=2, freqs=(1.0e9, 1.1e9, 1.2e9, 1.3e9), flag_frac=0.1)
    rng = np.random.default_rng(61)
    vis = rng.normal(size=(prob.n_row, prob.n_chan)) + 1j * rng.normal(size=(prob.n_row, prob.n_chan))
    x = rng.normal(size=(2, 96, 80))
    plan = make_plan(prob, prec)
    inf = plan.info()
    say(f"96x80 {prec}: grid {inf['grid_x']}x{inf['grid_y']}, PSF grid {inf['psf_grid_x']}x{inf['psf_grid_y']}")
    assert (inf["grid_x"], inf["grid_y"]) == (256, 256)
    tol = TOL[prec]
    e = {"dirty": rel(host(plan.grid(to_dev(vis, C))), oracle.grid(prob, vis)),
         "degrid": rel(host(plan.degrid(to_dev(x, R))), oracle.degrid(prob, x)),
         "hessian": rel(host(plan.hessian(to_dev(x, R))), oracle.hessian(prob, x))}
    psf = oracle.psf(prob)
    e["psf"] = rel(host(plan.make_psf()), psf)
    e["psf_conv"] = rel(host(plan.psf_conv(to_dev(x, R))), oracle.psf_conv(psf, x))
    lam = max(oracle.power_iteration(lambda v, b=b: oracle.psf_conv(psf[b:b + 1], v[None])[0],
                                     np.ones((96, 80)), 30)[0] for b in range(2))
    sigma = 0.1 * lam
    g = oracle.psf_conv(psf, np.abs(x))
    e["cg"] = rel(host(plan.precond_solve(to_dev(g, R), sigma, 8)), oracle.precond_solve(psf, g, sigma, 8)[0])
    xg = to_dev(np.abs(x) * 0.5, R)
    plan.fb_step(to_dev(g, R), xg, sigma, 1.0, 1e-3, 8)
    e["fb_step"] = rel(host(xg), oracle.fb_step(psf, g, np.abs(x) * 0.5, sigma, 1.0, 1e-3, 8))
    ws = plan.prox_workspace(7)
    e["wavelets"] = rel(host(plan.wavelet_analysis(to_dev(x, R), ws, 7, 3)), wv.psi_adj(x, 3))
    xp = to_dev(np.zeros_like(x), R)
    z = g / np.abs(g).max()
    plan.prox(to_dev(z, R), xp, ws, 0.05, 1.0, sigma, 1.05 * lam, 10, 7, 3)
    ref, _ = wv.prox_pd(lambda v: oracle.psf_conv(psf, v), z, sigma, 1.0, 0.05, 1.05 * lam, 3, 10)
    e["prox"] = rel(host(xp), ref)
    say(f"96x80 {prec}: " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()))
    for k in ("dirty", "degrid", "hessian", "psf", "psf_conv", "wavelets"):
        assert e[k] < tol, k
    for k in ("cg", "fb_step", "prox"):
        assert e[k] < (1e-4 if prec == "fp32" else 1e-9), k


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_paper_image_1728x1200(prec):
    R, C = _dt(prec)
    nx, ny = 1728, 1200
    prob = synth.tiny_problem(seed=synth.SEED_BASE + 62, nx=nx, ny=ny, n_row=800, cell_arcsec=1.0, n_band=1)
    rng = np.random.default_rng(63)
    vis = rng.normal(size=(prob.n_row, prob.n_chan)) + 1j * rng.normal(size=(prob.n_row, prob.n_chan))
    plan = make_plan(prob, prec)
    inf = plan.info()
    say(f"1728x1200 {prec}: grid {inf['grid_x']}x{inf['grid_y']}, PSF grid {inf['psf_grid_x']}x{inf['psf_grid_y']}, "
        f"{inf['n_wplanes_max']} w-planes")
    P = nx * ny
    fixed = [0, ny - 1, (nx - 1) * ny, P - 1, (nx // 2) * ny + ny // 2]
    pix = np.concatenate([fixed, rng.choice(P, 1024, replace=False)])
    xs = np.zeros((1, nx, ny))
    xs.ravel()[rng.choice(P, 300, replace=False)] = rng.uniform(0.1, 1.0, 300)
    tol = TOL[prec]
    e = {"dirty": rel(host(plan.grid(to_dev(vis, C))).ravel()[pix], oracle.grid(prob, vis, pix=pix)),
         "degrid": rel(host(plan.degrid(to_dev(xs, R))), oracle.degrid(prob, xs)),
         "hessian": rel(host(plan.hessian(to_dev(xs, R))).ravel()[pix], oracle.hessian(prob, xs, pix=pix))}
    say(f"1728x1200 {prec}: oracle PSF (factored direct sum over {2 * nx}x{2 * ny})")
    psf = oracle.psf_factored(prob)
    e["psf"] = rel(host(plan.make_psf()), psf)
    conv = oracle.psf_conv_op(psf)
    x = synth.extended_sky(synth.SEED_BASE + 62, 1, nx, ny).astype(np.float64)
    e["psf_conv"] = rel(host(plan.psf_conv(to_dev(x, R))), conv(x))
    lam = oracle.power_iteration(lambda v: conv.band(0, v), np.ones((nx, ny)), 10)[0]
    g = conv(x)
    y_ref, _ = oracle.precond_solve(psf, g, 1e-2 * lam, 10, conv=conv)
    e["cg"] = rel(host(plan.precond_solve(to_dev(g, R), 1e-2 * lam, 10)), y_ref)
    say(f"1728x1200 {prec}: " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()))
    for k in ("dirty", "degrid", "hessian", "psf", "psf_conv"):
        assert e[k] < tol, k
    assert e["cg"] < (1e-4 if prec == "fp32" else 1e-9)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_partial_last_column_group(prec):
    """64 x 34: the cropped row spectra of the w-plane transforms are stored in
    groups of 8 (FP32) or 4 (FP64) columns, and the convolution's half spectra in
    groups of 4 (FP32) or 2 (FP64): with ny = 34 the last plane group holds 2 of
    its columns, and gx = 2 nx takes the index-shift form of the centring factors
    while gy = 128 > 2 ny does not.  Operators against the FP64 oracle, two bands."""
    R, C = _dt(prec)
    prob = synth.tiny_problem(seed=synth.SEED_BASE + 64, nx=64, ny=34, n_row=900, cell_arcsec=40.0,
                              n_band=2, freqs=(1.0e9, 1.1e9, 1.2e9, 1.3e9), flag_frac=0.1, w_frac=0.5)
    rng = np.random.default_rng(65)
    vis = rng.normal(size=(prob.n_row, prob.n_chan)) + 1j * rng.normal(size=(prob.n_row, prob.n_chan))
    x = rng.normal(size=(2, 64, 34))
    plan = make_plan(prob, prec)
    inf = plan.info()
    assert (inf["grid_x"], inf["grid_y"]) == (128, 128)
    e = {"dirty": rel(host(plan.grid(to_dev(vis, C))), oracle.grid(prob, vis)),
         "degrid": rel(host(plan.degrid(to_dev(x, R))), oracle.degrid(prob, x)),
         "hessian": rel(host(plan.hessian(to_dev(x, R))), oracle.hessian(prob, x))}
    psf = oracle.psf(prob)
    e["psf"] = rel(host(plan.make_psf()), psf)
    e["psf_conv"] = rel(host(plan.psf_conv(to_dev(x, R))), oracle.psf_conv(psf, x))
    say(f"64x34 {prec}: w-planes {inf['n_wplanes_max']}; " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()))
    for k, v in e.items():
        assert v < TOL[prec], k
