"""Pins of the FP64 backward-step reference (eqs. 7 and 9) against facts that do
not come from its own code: the closed-form Haar and db2 filters, the published
db3 table, the defining
properties of Daubechies filters, perfect reconstruction and Parseval of an
orthonormal transform, a hand-computed Haar level, the tight-frame identity of
the dictionary, the closed-form prox in the Dirac / identity-metric case and
the fixed-point equations of the primal-dual iteration."""
import math

import numpy as np
import pytest

import oracle
from oracle import wavelets as wv


def test_haar_and_db2_closed_forms():
    assert np.allclose(wv.daubechies(1), [1 / math.sqrt(2), 1 / math.sqrt(2)], atol=1e-15)
    r3 = math.sqrt(3.0)
    db2 = np.array([1 + r3, 3 + r3, 3 - r3, 1 - r3]) / (4 * math.sqrt(2.0))
    assert np.allclose(wv.daubechies(2), db2, atol=1e-14)
    # db3 as tabulated in Daubechies' Ten Lectures on Wavelets (Table 6.1, scaled to sum sqrt 2)
    db3 = [0.3326705529500826, 0.8068915093110925, 0.4598775021184915,
           -0.1350110200102545, -0.0854412738820267, 0.0352262918857095]
    assert np.allclose(wv.daubechies(3), db3, atol=1e-13)


@pytest.mark.parametrize("n", range(1, 7))
def test_daubechies_defining_properties(n):
    h = wv.daubechies(n)
    g = wv.highpass(h)
    L = len(h)
    assert L == 2 * n
    assert abs(h.sum() - math.sqrt(2.0)) < 1e-13
    for m in range(0, n):     # orthonormal to its even shifts
        s = sum(h[k] * h[k + 2 * m] for k in range(L - 2 * m))
        assert abs(s - (1.0 if m == 0 else 0.0)) < 1e-12
    for p in range(n):        # n vanishing moments of the wavelet filter
        assert abs(sum(g[k] * k ** p for k in range(L))) < 1e-9 * max(1, (L - 1) ** p)
    assert abs(g.sum()) < 1e-13 and abs(np.dot(h, g)) < 1e-13


def test_haar_level_by_hand():
    x = np.array([[1.0, 2.0], [3.0, 4.0]])
    c = wv.dwt2(x, wv.daubechies(1), 1)
    # rows: (a+b)/sqrt2, (a-b)/sqrt2 ... with the wavelet g = (h1, -h0) = (1, -1)/sqrt2
    ref = np.array([[(1 + 2 + 3 + 4) / 2, (1 - 2 + 3 - 4) / 2],
                    [(1 + 2 - 3 - 4) / 2, (1 - 2 - 3 + 4) / 2]])
    assert np.allclose(c, ref, atol=1e-15)


@pytest.mark.parametrize("n", range(1, 7))
@pytest.mark.parametrize("levels", [1, 3])
def test_perfect_reconstruction_and_parseval(n, levels):
    rng = np.random.default_rng(100 + n)
    x = rng.normal(size=(2, 16, 32))
    h = wv.daubechies(n)
    c = wv.dwt2(x, h, levels)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
    assert np.allclose(wv.idwt2(c, h, levels), x, atol=1e-12)
    # the synthesis is the adjoint of the analysis
    y = rng.normal(size=x.shape)
    assert abs(np.vdot(wv.dwt2(x, h, levels), y) - np.vdot(x, wv.idwt2(y, h, levels))) < 1e-11


def test_dictionary_is_a_tight_frame():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(3, 16, 16))
    c = wv.psi_adj(x, 2)
    assert c.shape == (7, 3, 16, 16)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
    assert np.allclose(wv.psi(c, 2), x, atol=1e-12)


def test_pd_dirac_identity_metric_matches_closed_form():
    """U = Id (a delta PSF and sigma_u = 0) and the Dirac basis alone: the prox of
    gamma (lam ||.||_{2,1} + iota_+) is the group soft threshold of the positive part."""
    rng = np.random.default_rng(3)
    nb, nx, ny = 3, 8, 8
    z = rng.normal(size=(nb, nx, ny))
    delta = np.zeros((nb, 2 * nx, 2 * ny))
    delta[:, nx, ny] = 1.0
    apply_psf = lambda v: oracle.psf_conv(delta, v)
    assert np.allclose(apply_psf(z), z, atol=1e-12)
    gamma, lam = 0.7, 0.4
    x, _ = wv.prox_pd(apply_psf, z, 0.0, gamma, lam, 1.0, 1, 400, nbasis=1)
    zp = np.maximum(z, 0.0)
    nrm = np.sqrt((zp * zp).sum(axis=0, keepdims=True))
    ref = zp * np.maximum(0.0, 1.0 - gamma * lam / np.where(nrm > 0, nrm, 1.0))
    assert np.abs(x - ref).max() < 1e-9


def test_pd_fixed_point_with_psf_metric():
    """With the full dictionary and U = I^psf * + sigma Id the iterates settle on a
    fixed point: x = max(x - tau (grad + Psi v), 0) and v = project(v + sigma_d Psi^dagger x)."""
    rng = np.random.default_rng(9)
    nb, nx, ny = 2, 16, 16
    yy, xx = np.mgrid[-nx:nx, -ny:ny]
    psf = np.exp(-(xx ** 2 + yy ** 2) / 6.0)[None].repeat(nb, axis=0)
    apply_psf = lambda v: oracle.psf_conv(psf, v)
    unorm, _ = oracle.power_iteration(apply_psf, np.ones((nb, nx, ny)), 60)
    z = rng.normal(size=(nb, nx, ny)) + 0.5
    sigma_u, gamma, lam, levels = 0.1 * unorm, 1.0, 0.05, 2
    x, v = wv.prox_pd(apply_psf, z, sigma_u, gamma, lam, 1.05 * unorm, levels, 1500)
    _, sigma_d, tau = wv.pd_steps(1.05 * unorm, sigma_u, gamma)
    d = x - z
    grad = (apply_psf(d) + sigma_u * d) / gamma
    x2 = np.maximum(x - tau * (grad + wv.psi(v, levels)), 0.0)
    v2 = wv.l21_dual_project(v + sigma_d * wv.psi_adj(x, levels), lam)
    assert np.linalg.norm(x2 - x) < 1e-7 * np.linalg.norm(x)
    assert np.linalg.norm(v2 - v) < 1e-7 * max(np.linalg.norm(v), 1e-30)
    # the dual is feasible (l2 over bands <= lam) and the primal non-negative
    assert (np.sqrt((v * v).sum(axis=1)) <= lam * (1 + 1e-12)).all() and (x >= 0).all()


def test_dual_projection_is_the_moreau_complement_of_the_group_soft_threshold():
    """prox of sigma H^* for H = lam ||.||_{2,1} (over the band axis) equals
    t - sigma prox_{H / sigma}(t / sigma) (Moreau's identity), where the prox of the
    group norm is the group soft threshold."""
    rng = np.random.default_rng(31)
    t = rng.normal(size=(3, 4, 5, 6)) * 2.0
    lam, sigma = 0.7, 2.5
    u = t / sigma
    nrm = np.sqrt((u * u).sum(axis=1, keepdims=True))
    soft = u * np.maximum(0.0, 1.0 - (lam / sigma) / np.where(nrm > 0, nrm, 1.0))
    ref = t - sigma * soft
    assert np.allclose(wv.l21_dual_project(t, lam), ref, atol=1e-12)


def test_condat_step_rule_satisfies_the_convergence_condition():
    """Condat (2013), Theorem 3.1: the iteration converges when
    1 / tau - sigma_d ||L||^2 > beta / 2 for L = Psi^dagger.  ||L||^2 is measured here by
    power iteration on Psi Psi^dagger (a tight frame gives 1), not taken from the code."""
    rng = np.random.default_rng(5)
    v = rng.normal(size=(2, 16, 16))
    for _ in range(30):
        w = wv.psi(wv.psi_adj(v, 2), 2)
        nrm2 = float(np.vdot(v, w) / np.vdot(v, v))
        v = w / np.linalg.norm(w)
    assert abs(nrm2 - 1.0) < 1e-12
    for unorm, sigma_u, gamma in [(3.0, 0.0, 1.0), (120.0, 0.12, 0.5), (1.0, 1e-3, 1.9)]:
        beta, sigma_d, tau = wv.pd_steps(unorm, sigma_u, gamma)
        assert beta == pytest.approx((unorm + sigma_u) / gamma)   # Lipschitz constant of grad F
        assert 1.0 / tau - sigma_d * nrm2 > 0.5 * beta


def _delta_psf(nb, nx, ny, c):
    D = np.zeros((nb, 2 * nx, 2 * ny))
    D[:, nx, ny] = c
    return D


def test_fb_step_wavelet_scaled_delta_psf_closed_form():
    """I^psf = c delta and U = (c + sigma) Id: the forward step (eq. 6) is
    z = x - gamma (c x - I^d) / (c + sigma), and the U-metric prox of eq. 7 with the Dirac
    basis alone is the prox of gamma / (c + sigma) (lam ||.||_{2,1} + iota_+), the group
    soft threshold of z_+ with threshold gamma lam / (c + sigma)."""
    rng = np.random.default_rng(13)
    nb, nx, ny = 3, 8, 8
    c, sigma, gamma, lam = 2.0, 0.5, 0.6, 0.3
    D = _delta_psf(nb, nx, ny, c)
    x = rng.uniform(0.0, 1.0, (nb, nx, ny))
    dirty = rng.normal(0.0, 1.5, (nb, nx, ny)) + 1.0
    xo, v = wv.fb_step_wavelet(D, dirty, x, sigma, gamma, lam, c, 3, 3000, 1, nbasis=1)
    z = x - gamma * (c * x - dirty) / (c + sigma)
    zp = np.maximum(z, 0.0)
    nrm = np.sqrt((zp * zp).sum(axis=0, keepdims=True))
    ref = zp * np.maximum(0.0, 1.0 - (gamma * lam / (c + sigma)) / np.where(nrm > 0, nrm, 1.0))
    assert (ref == 0).any() and (ref > 0).any()
    assert np.abs(xo - ref).max() < 1e-9
    # zero primal-dual iterations: a cold start returns max(z, 0), a warm one its start x
    xc, _ = wv.fb_step_wavelet(D, dirty, x, sigma, gamma, lam, c, 3, 0, 1, nbasis=1)
    assert np.abs(xc - zp).max() < 1e-13
    xw, _ = wv.fb_step_wavelet(D, dirty, x, sigma, gamma, lam, c, 3, 0, 1, nbasis=1,
                               v0=np.zeros((1,) + x.shape), warm=True)
    assert np.array_equal(xw, x)


def _clean_problem():
    import synth
    p = synth.tiny_problem(seed=61, nx=16, ny=16, n_row=80, w_frac=0.5, cell_arcsec=60.0)
    x_true = synth.point_sky(61, 1, 16, 16, n_src=5, flux=(0.2, 1.0))
    return p, x_true


def test_clean_fixed_point_with_exact_gradient():
    """lam = 0, I^d = R^dagger Sigma^-1 R x_true (eq. 3, w term included) and x_true >= 0:
    the exact gradient vanishes at x_true, so the pfb-clean iterations started there
    return x_true unchanged."""
    p, x_true = _clean_problem()
    psf = oracle.psf(p)
    dirty = oracle.hessian(p, x_true)
    lam_max, _ = oracle.power_iteration(lambda t: oracle.psf_conv(psf, t), np.ones((1, 16, 16)), 40)
    x, _ = wv.clean(p, psf, dirty, x_true, 1e-2 * lam_max, 1.0, 0.0, 1.05 * lam_max, 10, 20, 3, 2)
    assert np.abs(x - x_true).max() < 1e-10 * np.abs(x_true).max()


def test_clean_decreases_the_data_fidelity():
    """From x = 0 with lam = 0, each exact-gradient step (eq. 3) preconditioned by
    U = I^psf * + sigma Id (eq. 8), gamma = 1 < 2 / L_U, followed by the U-metric
    projection onto x >= 0 (eq. 7 with lam = 0) lowers f(x) of eq. 2."""
    p, x_true = _clean_problem()
    vis = oracle.degrid(p, x_true)
    psf = oracle.psf(p)
    dirty = oracle.grid(p, vis)
    lam_max, _ = oracle.power_iteration(lambda t: oracle.psf_conv(psf, t), np.ones((1, 16, 16)), 40)
    sigma = 1e-1 * lam_max
    x = np.zeros_like(x_true)
    f = [oracle.fidelity(p, x, vis)]
    for n in range(1, 5):
        x, _ = wv.clean(p, psf, dirty, np.zeros_like(x_true), sigma, 1.0, 0.0, 1.05 * lam_max, 40, 300, n, 2)
        f.append(oracle.fidelity(p, x, vis))
    assert np.all(np.diff(f) < 0), f
    assert f[-1] < 0.5 * f[0]
    assert (x >= 0).all()


def test_clean_warm_starts_from_the_previous_step():
    """With zero primal-dual iterations the prox returns its start point: the first
    (cold) step gives max(z, 0), and every later step is warm-started from the previous
    iterate, so it returns that iterate unchanged."""
    p, x_true = _clean_problem()
    psf = oracle.psf(p)
    dirty = oracle.hessian(p, x_true)
    x0 = np.full_like(x_true, 0.05)
    args = (p, psf, dirty, x0, 0.5, 1.0, 0.1, 100.0, 10, 0)
    x1, _ = wv.clean(*args, 1, 2)
    x3, _ = wv.clean(*args, 3, 2)
    assert np.array_equal(x1, x3)
    y, _ = oracle.precond_solve(psf, oracle.hessian(p, x0) - dirty, 0.5, 10)
    assert not np.array_equal(x1, x0)
    assert np.abs(x1 - np.maximum(x0 - y, 0.0)).max() < 1e-13
