"""GPU parity of the backward step (eq. 7 with the regulariser of eq. 9) through the
C ABI: the wavelet dictionary Psi^dagger / Psi and the primal-dual prox against
the FP64 oracle, on a two-band, non-square problem."""
import numpy as np
import pytest

import oracle
import synth
from oracle import wavelets as wv
from gpu_helpers import TOL, host, make_plan, rel, say, to_dev

pytestmark = pytest.mark.gpu

PRECISIONS = ["fp32", "fp64"]


def _real(prec):
    import torch
    return torch.float64 if prec == "fp64" else torch.float32


@pytest.fixture(scope="module")
def mb():
    prob = synth.tiny_problem(seed=91, nx=64, ny=32, n_row=700, freqs=(1.0e9, 1.1e9, 1.3e9, 1.4e9),
                              cell_arcsec=120.0, w_frac=1.5, n_band=2, flag_frac=0.2)
    say("oracle: PSF of the two-band problem")
    psf = oracle.psf(prob)
    unorm, _ = oracle.power_iteration(lambda v: oracle.psf_conv(psf, v), np.ones((2, 64, 32)), 60)
    return dict(prob=prob, psf=psf, unorm=1.05 * unorm)


@pytest.fixture(scope="module", params=PRECISIONS)
def mb_plan(request, mb):
    say(f"plan: two-band 64x32 {request.param}")
    plan = make_plan(mb["prob"], request.param)
    plan.make_psf(want_image=False)
    return request.param, plan


@pytest.mark.parametrize("nbasis,levels", [(7, 3), (3, 1), (1, 2)])
def test_wavelet_analysis_and_synthesis(mb_plan, nbasis, levels):
    prec, plan = mb_plan
    R = _real(prec)
    rng = np.random.default_rng(5 + nbasis + levels)
    x = rng.normal(size=(2, 64, 32))
    c = rng.normal(size=(nbasis, 2, 64, 32))
    ws = plan.prox_workspace(nbasis)
    say(f"wavelets {prec} nbasis {nbasis} levels {levels}")
    a = host(plan.wavelet_analysis(to_dev(x, R), ws, nbasis, levels))
    assert rel(a, wv.psi_adj(x, levels, nbasis)) < TOL[prec]
    s = host(plan.wavelet_synthesis(to_dev(c, R), ws, nbasis, levels))
    assert rel(s, wv.psi(c, levels, nbasis)) < TOL[prec]
    # tight frame on the GPU: Psi Psi^dagger x = x
    back = host(plan.wavelet_synthesis(to_dev(a, R), ws, nbasis, levels))
    assert rel(back, x) < TOL[prec]


def test_prox_matches_oracle_and_warm_start(mb, mb_plan):
    prec, plan = mb_plan
    R = _real(prec)
    rng = np.random.default_rng(17)
    z = rng.normal(size=(2, 64, 32)) + 0.3
    unorm = mb["unorm"]
    sigma, gamma, lam, levels, iters = 0.1 * unorm, 1.0, 0.1, 2, 30
    ws = plan.prox_workspace(7)
    zg = to_dev(z, R)
    say(f"prox {prec}: {iters} primal-dual iterations")
    x = plan.prox(zg, to_dev(np.zeros_like(z), R), ws, lam, gamma, sigma, unorm, iters, 7, levels)
    xh = host(x)
    x_ref, v_ref = wv.prox_pd(lambda v: oracle.psf_conv(mb["psf"], v), z, sigma, gamma, lam, unorm, levels, iters)
    tol = 5e-5 if prec == "fp32" else 1e-9
    assert rel(xh, x_ref) < tol
    assert (xh >= 0).all()
    # the dual variable left in the workspace: |v| <= lam per band vector
    v = host(ws[: 7 * 2 * 64 * 32 * (8 if prec == "fp64" else 4)].view(R)).reshape(7, 2, 64, 32)
    assert rel(v, v_ref) < 10 * tol
    assert (np.sqrt((v.astype(np.float64) ** 2).sum(axis=1)) <= lam * (1 + 1e-5)).all()
    # 15 + 15 warm-started iterations equal 30 in one call, bit for bit
    x2 = plan.prox(zg, to_dev(np.zeros_like(z), R), ws, lam, gamma, sigma, unorm, 15, 7, levels)
    x2 = plan.prox(zg, x2, ws, lam, gamma, sigma, unorm, 15, 7, levels, warm=True)
    assert np.array_equal(host(x2), xh)


def test_prox_zero_iterations_and_bad_arguments(mb_plan):
    prec, plan = mb_plan
    R = _real(prec)
    from paper_2101_08072_amd import _lib
    z = np.random.default_rng(2).normal(size=(2, 64, 32))
    ws = plan.prox_workspace(7)
    x = host(plan.prox(to_dev(z, R), to_dev(np.zeros_like(z), R), ws, 0.1, 1.0, 0.0, 1.0, 0))
    assert np.array_equal(x, np.maximum(z, 0).astype(x.dtype))
    with pytest.raises(_lib.PfbError):
        plan.prox(to_dev(z, R), to_dev(z, R), ws, 0.1, 1.0, 0.0, 1.0, 3, levels=7)   # 32 is not a multiple of 2^7
    with pytest.raises(_lib.PfbError):
        plan.prox(to_dev(z, R), to_dev(z, R), ws[:16], 0.1, 1.0, 0.0, 1.0, 3)        # workspace too small


def test_fb_step_wavelet_two_steps(mb, mb_plan):
    """Two forward-backward steps (eqs. 6-7, prior of eq. 9), the second warm-started
    from the first step's primal and dual variables."""
    prec, plan = mb_plan
    R = _real(prec)
    rng = np.random.default_rng(23)
    dirty = oracle.psf_conv(mb["psf"], np.abs(rng.normal(size=(2, 64, 32))))
    x0 = np.zeros((2, 64, 32))
    unorm = mb["unorm"]
    sigma, gamma, lam, levels, cg_iters, pd_iters = 0.1 * unorm, 1.0, 0.02 * np.abs(dirty).max(), 2, 8, 10
    ws = plan.prox_workspace(7)
    xg = to_dev(x0, R)
    dg = to_dev(dirty, R)
    say(f"fb_step_wavelet {prec}")
    plan.fb_step_wavelet(dg, xg, ws, sigma, gamma, lam, unorm, cg_iters, pd_iters, 7, levels)
    x1 = host(xg).copy()
    plan.fb_step_wavelet(dg, xg, ws, sigma, gamma, lam, unorm, cg_iters, pd_iters, 7, levels, warm=True)
    x2 = host(xg)
    r1, v1 = wv.fb_step_wavelet(mb["psf"], dirty, x0, sigma, gamma, lam, unorm, cg_iters, pd_iters, levels)
    r2, _ = wv.fb_step_wavelet(mb["psf"], dirty, r1, sigma, gamma, lam, unorm, cg_iters, pd_iters, levels,
                               v0=v1, warm=True)
    tol = 1e-4 if prec == "fp32" else 1e-9
    assert rel(x1, r1) < tol
    assert rel(x2, r2) < tol
    assert (x2 >= 0).all() and np.linalg.norm(x2) > 0


def test_clean_exact_gradient_major_cycles(mb, mb_plan):
    """Two pfb-clean steps with the exact gradient (one Hessian each, eq. 3) and the
    wavelet prior, against the oracle's direct-sum Hessian."""
    prec, plan = mb_plan
    R = _real(prec)
    prob = mb["prob"]
    x_true = synth.point_sky(93, 2, 64, 32, n_src=6)
    vis = oracle.degrid(prob, x_true)
    dirty = oracle.grid(prob, vis)
    x0 = np.zeros((2, 64, 32))
    unorm = mb["unorm"]
    sigma, gamma, lam, levels, cg_iters, pd_iters, n_major = 0.1 * unorm, 1.0, 1e-3 * np.abs(dirty).max(), 2, 8, 10, 2
    ws = plan.prox_workspace(7)
    xg = to_dev(x0, R)
    say(f"clean {prec}: {n_major} major steps")
    plan.clean(to_dev(dirty, R), xg, ws, sigma, gamma, lam, unorm, cg_iters, pd_iters, n_major, 7, levels)
    ref, _ = wv.clean(prob, mb["psf"], dirty, x0, sigma, gamma, lam, unorm, cg_iters, pd_iters, n_major, levels)
    tol = 1e-4 if prec == "fp32" else 1e-9
    assert rel(host(xg), ref) < tol


def test_precond_solve_two_bands(mb, mb_plan):
    """CG on U = I^psf * + sigma Id (eq. 8) with two bands: each band's system has
    its own step lengths, as in the oracle."""
    prec, plan = mb_plan
    R = _real(prec)
    g = np.random.default_rng(29).normal(size=(2, 64, 32))
    sigma, iters = 0.1 * mb["unorm"], 8
    say(f"precond_solve two bands {prec}")
    y = host(plan.precond_solve(to_dev(g, R), sigma, iters))
    y_ref, _ = oracle.precond_solve(mb["psf"], g, sigma, iters)
    tol = 1e-4 if prec == "fp32" else 1e-9
    for b in range(2):
        assert rel(y[b], y_ref[b]) < tol


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_wavelets_and_prox_with_interior_tiles(prec):
    """At 256 x 128 most analysis and synthesis tiles of db2-db6 lie inside the image,
    so the kernels' interior (non-wrapping) branch is compared with the oracle too:
    Psi^dagger, Psi, the tight-frame round trip and 10 primal-dual steps of eq. 7 with
    the full dictionary (two bands, 3 levels)."""
    import torch
    R = _real(prec)
    prob = synth.tiny_problem(seed=97, nx=256, ny=128, n_row=1500, n_band=2, freqs=(1.0e9, 1.1e9, 1.2e9, 1.3e9),
                              cell_arcsec=20.0)
    plan = make_plan(prob, prec)
    rng = np.random.default_rng(98)
    x = rng.normal(size=(2, 256, 128))
    ws = plan.prox_workspace(7)
    c = host(plan.wavelet_analysis(to_dev(x, R), ws, 7, 3))
    c_ref = wv.psi_adj(x, 3)
    v = rng.normal(size=c_ref.shape)
    s = host(plan.wavelet_synthesis(to_dev(v, R), ws, 7, 3))
    rt = host(plan.wavelet_synthesis(plan.wavelet_analysis(to_dev(x, R), ws, 7, 3), ws, 7, 3))
    psf = oracle.psf(prob)
    unorm = max(oracle.power_iteration(lambda t, b=b: oracle.psf_conv(psf[b:b + 1], t[None])[0],
                                       np.ones((256, 128)), 30)[0] for b in range(2))
    plan.make_psf(want_image=False)
    z = oracle.psf_conv(psf, np.abs(x)) / unorm
    xp = to_dev(np.zeros_like(x), R)
    plan.prox(to_dev(z, R), xp, ws, 0.05, 1.0, 0.1 * unorm, 1.05 * unorm, 10, 7, 3)
    ref, _ = wv.prox_pd(lambda t: oracle.psf_conv(psf, t), z, 0.1 * unorm, 1.0, 0.05, 1.05 * unorm, 3, 10)
    e = (rel(c, c_ref), rel(s, wv.psi(v, 3)), rel(rt, x), rel(host(xp), ref))
    say(f"wavelets 256x128 {prec}: analysis {e[0]:.2e}, synthesis {e[1]:.2e}, round trip {e[2]:.2e}, prox {e[3]:.2e}")
    tol = TOL[prec]
    assert e[0] < tol and e[1] < tol and e[2] < tol
    assert e[3] < (5e-5 if prec == "fp32" else 1e-9)
