"""FP64 reference for the paper's backward step (eq. 7 with the regulariser of eq. 9).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the product package
never imports or runs it.

The regulariser is r(x) = lambda ||Psi^dagger x||_{2,1} + iota_+(x) (eq. 9):
Psi holds the Dirac basis and the first six Daubechies wavelet bases, the l2
norm runs over imaging bands and the l1 sum over bases and coefficients.  The
backward step prox^U_{gamma r}(z) (eq. 7) is solved with the primal-dual
algorithm of Condat (2013) that the text after eq. 8 names.

* ``daubechies(n)``   orthonormal Daubechies low-pass filter with n vanishing
                      moments (length 2n), from its defining polynomial
* ``dwt2``/``idwt2``  multi-level periodic 2-D wavelet analysis / synthesis
* ``psi_adj``/``psi`` Psi^dagger and Psi of the normalised dictionary
* ``prox_pd``         the primal-dual iteration for eq. 7

Readings (the paper gives none of these): periodic boundaries; the dictionary
is scaled by 1/sqrt(number of bases) so that Psi Psi^dagger = Id (a tight
frame with ||Psi^dagger|| = 1); Condat's algorithm without relaxation with
F(x) = (x - z)^T U (x - z) / (2 gamma), G = iota_+, H = lambda ||.||_{2,1},
L = Psi^dagger, dual step sigma_d = beta = ||U|| / gamma and primal step
tau = 0.99 / (beta / 2 + sigma_d); the iteration starts from x = max(z, 0),
v = 0 unless given.
"""
from __future__ import annotations

import math

import numpy as np


def daubechies(n):
    """Low-pass filter h of the Daubechies wavelet with n vanishing moments.

    |m0|^2 = cos^(2n)(xi/2) P(sin^2(xi/2)) with P(y) = sum_{k<n} C(n-1+k, k) y^k;
    each root y of P gives the z-plane pair z + 1/z = 2 - 4y, of which the root
    inside the unit circle is kept (minimum phase).  h is the coefficient list of
    (z + 1)^n prod (z - z_i) in descending powers, scaled to sum sqrt(2)."""
    if n < 1:
        raise ValueError("n >= 1")
    coeffs = [math.comb(n - 1 + k, k) for k in range(n)]          # ascending powers of y
    yroots = np.roots(coeffs[::-1]) if n > 1 else np.array([])
    zroots = []
    for y in yroots:
        b = 1.0 - 2.0 * y                                          # z^2 - 2 b z + 1 = 0
        s = np.sqrt(b * b - 1.0 + 0j)
        z1, z2 = b + s, b - s
        zroots.append(z1 if abs(z1) < 1.0 else z2)
    h = np.real(np.poly(np.array([-1.0] * n + zroots, dtype=complex)))
    return h * (math.sqrt(2.0) / h.sum())


def highpass(h):
    """g_k = (-1)^k h_{L-1-k}: the orthonormal wavelet filter of h."""
    L = len(h)
    return np.array([(-1.0) ** k * h[L - 1 - k] for k in range(L)])


def _idx(n, L):
    # input positions (2k + j) mod n read by output k for tap j
    return (2 * np.arange(n // 2)[:, None] + np.arange(L)[None, :]) % n


def dwt1(x, h, axis):
    """One periodic analysis level along ``axis``: [low | high], each n/2 long:
    low[k] = sum_j h[j] x[(2k + j) mod n], high[k] = sum_j g[j] x[(2k + j) mod n]."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    n = x.shape[-1]
    idx = _idx(n, len(h))
    xs = x[..., idx]                                               # (..., n/2, L)
    out = np.concatenate([xs @ h, xs @ highpass(h)], axis=-1)
    return np.moveaxis(out, -1, axis)


def idwt1(c, h, axis):
    """Adjoint of ``dwt1`` (its inverse for an orthonormal filter): each
    coefficient is added back, times its tap, at every position it read."""
    c = np.moveaxis(np.asarray(c, dtype=np.float64), axis, -1)
    n = c.shape[-1]
    idx = _idx(n, len(h))
    lo, hi = c[..., : n // 2], c[..., n // 2:]
    contrib = lo[..., :, None] * h[None, :] + hi[..., :, None] * highpass(h)[None, :]   # (..., n/2, L)
    x = np.zeros(c.shape)
    flat_x = x.reshape(-1, n)
    flat_c = contrib.reshape(-1, idx.size)
    for r in range(flat_x.shape[0]):
        np.add.at(flat_x[r], idx.ravel(), flat_c[r])
    return np.moveaxis(x, -1, axis)


def dwt2(x, h, levels):
    """Multi-level 2-D analysis of the last two axes (Mallat layout): each level
    transforms the rows, then the columns, of the current top-left low-pass block."""
    c = np.array(x, dtype=np.float64)
    nx, ny = c.shape[-2:]
    for _ in range(levels):
        blk = c[..., :nx, :ny]
        blk = dwt1(blk, h, axis=-1)
        blk = dwt1(blk, h, axis=-2)
        c[..., :nx, :ny] = blk
        nx //= 2
        ny //= 2
    return c


def idwt2(c, h, levels):
    """Inverse (= adjoint) of ``dwt2``: levels from the coarsest, columns then rows."""
    x = np.array(c, dtype=np.float64)
    nx, ny = x.shape[-2:]
    sizes = []
    for _ in range(levels):
        sizes.append((nx, ny))
        nx //= 2
        ny //= 2
    for nx, ny in reversed(sizes):
        blk = x[..., :nx, :ny]
        blk = idwt1(blk, h, axis=-2)
        blk = idwt1(blk, h, axis=-1)
        x[..., :nx, :ny] = blk
    return x


def filters(nbasis=7):
    """Wavelet filters of the dictionary: bases 1 .. nbasis - 1 are db1, db2, ..."""
    return [daubechies(k) for k in range(1, nbasis)]


def psi_adj(x, levels, nbasis=7):
    """Psi^dagger x for images x[..., nx, ny]: shape (nbasis, ..., nx, ny);
    basis 0 is the Dirac basis, basis k >= 1 the db_k analysis."""
    s = 1.0 / math.sqrt(nbasis)
    x = np.asarray(x, dtype=np.float64)
    out = [x * s] + [dwt2(x, h, levels) * s for h in filters(nbasis)]
    return np.stack(out)


def psi(v, levels, nbasis=7):
    """Psi v = (v_0 + sum_k idwt_k(v_k)) / sqrt(nbasis) (the adjoint of psi_adj)."""
    s = 1.0 / math.sqrt(nbasis)
    v = np.asarray(v, dtype=np.float64)
    x = v[0].copy()
    for k, h in enumerate(filters(nbasis), start=1):
        x += idwt2(v[k], h, levels)
    return x * s


def l21_dual_project(t, lam):
    """prox of sigma H^* for H = lam ||.||_{2,1}: every group (the bands of one
    basis and coefficient, axis 1) is scaled onto the l2 ball of radius lam."""
    nrm = np.sqrt(np.sum(t * t, axis=1, keepdims=True))
    scale = np.minimum(1.0, lam / np.where(nrm > 0, nrm, 1.0))
    return t * scale


def pd_steps(unorm, sigma_u, gamma):
    """(beta, sigma_d, tau) for F with gradient U (x - z) / gamma, ||U|| = unorm + sigma_u."""
    beta = (unorm + sigma_u) / gamma
    sigma_d = beta
    tau = 0.99 / (0.5 * beta + sigma_d)
    return beta, sigma_d, tau


def prox_pd(apply_psf, z, sigma_u, gamma, lam, unorm, levels, iters, nbasis=7, x0=None, v0=None):
    """Condat primal-dual iterations for eq. 7 with U = I^psf * + sigma_u Id:

        x~ = max(x - tau (U (x - z) / gamma + Psi v), 0)
        v  = project_lam(v + sigma_d Psi^dagger (2 x~ - x))
        x  = x~

    ``apply_psf`` is the PSF convolution (eq. 4); ``unorm`` bounds its norm.
    Returns (x, v)."""
    z = np.asarray(z, dtype=np.float64)
    _, sigma_d, tau = pd_steps(unorm, sigma_u, gamma)
    x = np.maximum(z, 0.0) if x0 is None else np.array(x0, dtype=np.float64)
    v = np.zeros((nbasis,) + z.shape) if v0 is None else np.array(v0, dtype=np.float64)
    for _ in range(iters):
        d = x - z
        grad = (apply_psf(d) + sigma_u * d) / gamma
        xt = np.maximum(x - tau * (grad + psi(v, levels, nbasis)), 0.0)
        v = l21_dual_project(v + sigma_d * psi_adj(2.0 * xt - x, levels, nbasis), lam)
        x = xt
    return x, v


def fb_step_wavelet(psf_img, dirty, x, sigma, gamma, lam, unorm, cg_iters, pd_iters, levels, nbasis=7,
                    v0=None, warm=False):
    """One forward-backward step of eqs. 6-7 with the regulariser of eq. 9:
    z = x - gamma U^-1 (I^psf * x - I^d) by CG, then x = prox^U_{gamma r}(z) by
    ``prox_pd`` (warm: from the given x and dual v0).  Returns (x, v)."""
    import oracle
    grad = oracle.psf_conv(psf_img, x) - dirty
    y, _ = oracle.precond_solve(psf_img, grad, sigma, cg_iters)
    z = np.asarray(x, dtype=np.float64) - gamma * y
    return prox_pd(lambda v: oracle.psf_conv(psf_img, v), z, sigma, gamma, lam, unorm, levels, pd_iters, nbasis,
                   x0=x if warm else None, v0=v0 if warm else None)


def clean(prob, psf_img, dirty, x0, sigma, gamma, lam, unorm, cg_iters, pd_iters, n_major, levels, nbasis=7):
    """``n_major`` forward-backward steps of eqs. 6-7 with the exact gradient
    R^dagger Sigma^-1 R x - I^d (eq. 3, the FP64 direct-sum Hessian) and the prior of
    eq. 9; the prox is warm-started from the previous step after the first."""
    import oracle
    x = np.array(x0, dtype=np.float64)
    v = None
    for k in range(n_major):
        grad = oracle.hessian(prob, x) - dirty
        y, _ = oracle.precond_solve(psf_img, grad, sigma, cg_iters)
        z = x - gamma * y
        x, v = prox_pd(lambda t: oracle.psf_conv(psf_img, t), z, sigma, gamma, lam, unorm, levels, pd_iters, nbasis,
                       x0=x if k > 0 else None, v0=v if k > 0 else None)
    return x, v
