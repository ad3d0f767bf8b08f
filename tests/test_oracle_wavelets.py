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
