"""Pins for the FP64 oracle: closed forms, identities, library special cases and
brute force, chosen so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.

Each test names the passage of the paper (Bester et al. 2021, Section 2) whose
definition it pins.
"""
import math

import numpy as np
import pytest

import synth

C0 = 299792458.0


def _small(seed=7, nx=16, ny=16, n_row=60, **kw):
    return synth.tiny_problem(seed=seed, nx=nx, ny=ny, n_row=n_row, **kw)


# --------------------------------------------------------------------------
# R  (eq. 1: V = R x + eps; R maps n_b real images to n_nu x n_d complex data)
# --------------------------------------------------------------------------

def test_degrid_point_source_at_phase_centre_is_unity(oracle_mod):
    """A unit source at l = m = 0 has n = 1 and zero phase: every unflagged V is 1."""
    p = _small(flag_frac=0.2)
    x = np.zeros((1, p.nx, p.ny))
    x[0, p.nx // 2, p.ny // 2] = 1.0
    V = oracle_mod.degrid(p, x)
    on = p.effective_weight() != 0
    assert np.abs(V[on] - 1.0).max() < 1e-14
    assert np.all(V[~on] == 0)          # flagged entries are zero by convention


def _grid_frequency_problem(nx, ny, cell, f=1.4e9, w_m=0.0):
    """Visibilities at every DFT frequency u = k/(nx cell), v = k'/(ny cell), w = w_m."""
    k, kp = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    lam = C0 / f
    uvw = np.stack([k.ravel() / (nx * cell) * lam, kp.ravel() / (ny * cell) * lam,
                    np.full(k.size, w_m)], axis=1)
    return synth.Problem(uvw=uvw, freq=np.array([f]), weight=np.ones((k.size, 1)), flag=None,
                         chan_band=np.zeros(1, np.int32), n_band=1, nx=nx, ny=ny,
                         cellx=cell, celly=cell)


@pytest.mark.parametrize("flat", [True, False])
def test_degrid_equals_numpy_fft_on_grid_frequencies(oracle_mod, flat):
    """With w = 0 and (u, v) on the DFT grid, R x is numpy's FFT of x / n, after moving
    pixel (nx/2, ny/2) to index 0.  Pins the Fourier sign, the pixel origin and the
    axis order (axis 0 pairs with u).  n is computed here as cos(asin(r)), not from
    the oracle's formula."""
    nx, ny, cell = 12, 10, 2e-3
    p = _grid_frequency_problem(nx, ny, cell)
    x = np.random.default_rng(1).normal(size=(1, nx, ny))
    V = oracle_mod.degrid(p, x, flat=flat).reshape(nx, ny)
    li = (np.arange(nx) - nx // 2) * cell
    mj = (np.arange(ny) - ny // 2) * cell
    rho = np.hypot(li[:, None], mj[None, :])
    n = np.cos(np.arcsin(rho))
    img = x[0] if flat else x[0] / n
    ref = np.fft.fft2(np.fft.ifftshift(img))
    assert np.abs(V - ref).max() / np.abs(ref).max() < 1e-12


def test_degrid_w_term_phase_slope_and_amplitude(oracle_mod):
    """At u = v = 0 a unit source at angle theta from the centre gives |V| = 1/cos(theta)
    and a phase that advances by 2 pi * 2 sin^2(theta/2) per wavelength of w.
    Pins the sign and size of the w (n - 1) term and the 1/n factor."""
    nx = ny = 32
    cell = 4e-3
    f = 1e9
    lam = C0 / f
    ws = np.array([0.0, 0.37, 0.81, 1.3]) * lam      # w in metres -> w/lam wavelengths
    uvw = np.stack([np.zeros(4), np.zeros(4), ws], axis=1)
    p = synth.Problem(uvw=uvw, freq=np.array([f]), weight=np.ones((4, 1)), flag=None,
                      chan_band=np.zeros(1, np.int32), n_band=1, nx=nx, ny=ny,
                      cellx=cell, celly=cell)
    for (i, j) in [(3, 5), (30, 17), (16, 0), (25, 25)]:
        x = np.zeros((1, nx, ny))
        x[0, i, j] = 1.0
        V = oracle_mod.degrid(p, x)[:, 0]
        theta = math.asin(math.hypot((i - nx // 2) * cell, (j - ny // 2) * cell))
        assert np.allclose(np.abs(V) * math.cos(theta), 1.0, rtol=0, atol=1e-13)
        slope = 2.0 * math.sin(theta / 2) ** 2          # = 1 - n
        expect = np.exp(2j * math.pi * slope * ws / lam)
        assert np.abs(V * math.cos(theta) - expect).max() < 1e-12


def test_conjugate_symmetry_of_real_sky(oracle_mod):
    """For a real image, V(-u, -v, -w) = conj V(u, v, w)."""
    p = _small()
    q = synth.Problem(**{**p.__dict__, "uvw": -p.uvw})
    x = np.random.default_rng(2).normal(size=(1, p.nx, p.ny))
    assert np.abs(oracle_mod.degrid(q, x) - np.conj(oracle_mod.degrid(p, x))).max() < 1e-12


def test_bands_only_see_their_own_channels(oracle_mod):
    """R maps band b's image only to band b's channels (Section 2, n_b << n_nu)."""
    p = synth.tiny_problem(seed=3, nx=8, ny=8, n_row=20, freqs=(1.0e9, 1.05e9, 1.1e9, 1.15e9),
                           n_band=2)
    x = np.zeros((2, 8, 8))
    x[1] = np.random.default_rng(4).normal(size=(8, 8))
    V = oracle_mod.degrid(p, x)
    assert np.all(V[:, :2] == 0)
    assert np.abs(V[:, 2:]).min() > 0
    I = oracle_mod.grid(p, V)
    assert np.all(I[0] == 0)


def test_c_oracle_matches_dense_numpy_twin(oracle_mod):
    """Two independent codes (C loops, NumPy matrix) for R and R^dagger Sigma^-1."""
    p = synth.tiny_problem(seed=5, nx=16, ny=12, n_row=80, freqs=(1.0e9, 1.1e9, 1.2e9, 1.3e9),
                           n_band=2, flag_frac=0.15)
    A, W, idx = oracle_mod.dense_operator(p)
    rng = np.random.default_rng(6)
    x = rng.normal(size=(2, 16, 12))
    V = oracle_mod.degrid(p, x).ravel()
    Vd = A @ x.ravel()
    assert np.abs(V[idx] - Vd).max() / np.abs(Vd).max() < 1e-13
    vis = rng.normal(size=V.shape) + 1j * rng.normal(size=V.shape)
    I = oracle_mod.grid(p, vis)
    Id = (A.conj().T @ (W * vis[idx])).real
    assert np.abs(I.ravel() - Id).max() / np.abs(Id).max() < 1e-13


# --------------------------------------------------------------------------
# R^dagger, dirty image, Hessian  (eqs. 2-3 and the definition of I^d)
# --------------------------------------------------------------------------

def test_adjoint_identity(oracle_mod):
    """Re <R x, Sigma^-1 V> = <x, R^dagger Sigma^-1 V> for real x."""
    p = _small(flag_frac=0.1)
    rng = np.random.default_rng(8)
    x = rng.normal(size=(1, p.nx, p.ny))
    vis = rng.normal(size=(p.n_row, p.n_chan)) + 1j * rng.normal(size=(p.n_row, p.n_chan))
    lhs = np.sum(p.effective_weight() * (np.conj(oracle_mod.degrid(p, x)) * vis)).real
    rhs = np.sum(x * oracle_mod.grid(p, vis))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs))


def test_dirty_image_peak_of_point_source(oracle_mod):
    """Noise-free V = R delta_p: I^d[p] = sum(weights) / n_p^2 exactly."""
    p = synth.tiny_problem(seed=9, nx=32, ny=32, n_row=100, cell_arcsec=600.0)
    for (i, j) in [(16, 16), (2, 29), (31, 5)]:
        x = np.zeros((1, 32, 32))
        x[0, i, j] = 1.0
        I = oracle_mod.grid(p, oracle_mod.degrid(p, x))
        rho2 = ((i - 16) * p.cellx) ** 2 + ((j - 16) * p.celly) ** 2
        expect = p.effective_weight().sum() / (1.0 - rho2)
        assert abs(I[0, i, j] - expect) < 1e-12 * expect
        assert I[0].max() == I[0, i, j]


def test_hessian_symmetric_psd_with_closed_form_diagonal(oracle_mod):
    """H = R^dagger Sigma^-1 R is symmetric, <x, Hx> = sum w |Rx|^2 >= 0 and its
    diagonal is sum(w) / n_p^2."""
    p = synth.tiny_problem(seed=10, nx=8, ny=8, n_row=40, cell_arcsec=900.0)
    P = 64
    H = np.empty((P, P))
    for k in range(P):
        e = np.zeros(P)
        e[k] = 1.0
        H[:, k] = oracle_mod.hessian(p, e.reshape(1, 8, 8)).ravel()
    assert np.abs(H - H.T).max() < 1e-11 * np.abs(H).max()
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > -1e-9 * np.abs(H).max()
    li = (np.arange(8) - 4) * p.cellx
    rho2 = (li[:, None] ** 2 + li[None, :] ** 2).ravel()
    assert np.allclose(np.diag(H), p.effective_weight().sum() / (1.0 - rho2), rtol=1e-12)
    x = np.random.default_rng(11).normal(size=(1, 8, 8))
    quad = float(np.sum(x * oracle_mod.hessian(p, x)))
    V = oracle_mod.degrid(p, x)
    assert abs(quad - np.sum(p.effective_weight() * np.abs(V) ** 2)) < 1e-11 * quad


def test_gradient_matches_finite_difference_of_fidelity(oracle_mod):
    """eq. (3) is the gradient of eq. (2): f is quadratic so a central difference
    along any direction d equals <grad f, d> up to rounding."""
    p = _small(seed=12, nx=8, ny=8, n_row=30)
    rng = np.random.default_rng(13)
    x = rng.normal(size=(1, 8, 8))
    vis = rng.normal(size=(p.n_row, p.n_chan)) + 1j * rng.normal(size=(p.n_row, p.n_chan))
    g = oracle_mod.gradient(p, x, vis)
    for _ in range(3):
        d = rng.normal(size=x.shape)
        h = 1e-3
        fd = (oracle_mod.fidelity(p, x + h * d, vis) - oracle_mod.fidelity(p, x - h * d, vis)) / (2 * h)
        assert abs(fd - np.sum(g * d)) < 1e-8 * max(1.0, abs(fd))


# --------------------------------------------------------------------------
# PSF and the PSF-approximate gradient (eq. 4)
# --------------------------------------------------------------------------

def test_psf_symmetric_with_peak_sum_of_weights(oracle_mod):
    p = _small(seed=14, flag_frac=0.1)
    P = oracle_mod.psf(p)[0]
    nx, ny = p.nx, p.ny
    sw = p.effective_weight().sum()
    assert abs(P[nx, ny] - sw) < 1e-12 * sw
    assert np.all(np.abs(P) <= sw * (1 + 1e-14))
    assert np.all(P[0, :] == 0) and np.all(P[:, 0] == 0)
    core = P[1:, 1:]
    assert np.abs(core - core[::-1, ::-1]).max() < 1e-12 * sw   # PSF(d) = PSF(-d)
    # spectrum of the centred PSF is real once the -N row/column is zero
    Pc = np.roll(P, (-nx, -ny), axis=(0, 1))
    assert np.abs(np.fft.fft2(Pc).imag).max() < 1e-10 * sw


def test_flat_hessian_equals_psf_convolution(oracle_mod):
    """Without the w term and with n = 1 the Hessian is exactly the convolution with
    the PSF (the approximation of eq. 4 becomes an identity)."""
    p0 = _small(seed=15, nx=12, ny=10, n_row=50)
    p = synth.Problem(**{**p0.__dict__, "celly": 1.3 * p0.cellx})   # non-square cells
    x = np.random.default_rng(16).normal(size=(1, 12, 10))
    H = oracle_mod.hessian(p, x, flat=True)
    C = oracle_mod.psf_conv(oracle_mod.psf(p), x)
    assert np.abs(H - C).max() < 1e-11 * np.abs(H).max()
    # ... and with the w term and 1/n it differs (the caveat after eq. 4)
    Hw = oracle_mod.hessian(synth.Problem(**{**p.__dict__, "cellx": 0.02, "celly": 0.02}), x)
    Cw = oracle_mod.psf_conv(oracle_mod.psf(synth.Problem(**{**p.__dict__, "cellx": 0.02,
                                                             "celly": 0.02})), x)
    assert np.abs(Hw - Cw).max() > 1e-3 * np.abs(Hw).max()


def test_psf_conv_direct_sum_vs_library_and_delta(oracle_mod):
    rng = np.random.default_rng(17)
    nx, ny = 9 * 2, 7 * 2
    psf_img = rng.normal(size=(1, 2 * nx, 2 * ny))
    x = rng.normal(size=(1, nx, ny))
    y = oracle_mod.psf_conv(psf_img, x)
    yd = oracle_mod.psf_conv_direct(psf_img[0], x[0])
    assert np.abs(y[0] - yd).max() < 1e-11 * np.abs(yd).max()
    d = np.zeros((1, nx, ny))
    d[0, nx // 2, ny // 2] = 1.0
    yc = oracle_mod.psf_conv(psf_img, d)[0]
    assert np.allclose(yc, psf_img[0, nx - nx // 2:2 * nx - nx // 2, ny - ny // 2:2 * ny - ny // 2],
                       atol=1e-12)


def _dense_psf_matrix(oracle_mod, psf_img):
    nb, NX, NY = psf_img.shape
    nx, ny = NX // 2, NY // 2
    M = np.empty((nx * ny, nx * ny))
    for k in range(nx * ny):
        e = np.zeros((1, nx, ny))
        e.flat[k] = 1.0
        M[:, k] = oracle_mod.psf_conv(psf_img, e).ravel()
    return M


def test_cg_against_dense_solve_and_scaled_delta(oracle_mod):
    """CG on U = I^psf * + sigma Id (eq. 8) converges to numpy's dense solve; with
    I^psf = c delta one step gives g / (c + sigma)."""
    p = _small(seed=18, nx=8, ny=8, n_row=40)
    P = oracle_mod.psf(p)
    M = _dense_psf_matrix(oracle_mod, P)
    lam_max = np.linalg.eigvalsh(0.5 * (M + M.T)).max()
    sigma = 0.1 * lam_max
    g = np.random.default_rng(19).normal(size=(1, 8, 8))
    y, trace = oracle_mod.precond_solve(P, g, sigma, 64)
    ref = np.linalg.solve(M + sigma * np.eye(64), g.ravel())
    assert np.abs(y.ravel() - ref).max() < 1e-9 * np.abs(ref).max()
    assert trace[0][-1] < 1e-16 * trace[0][0]
    D = np.zeros((1, 16, 16))
    D[0, 8, 8] = 3.0
    y1, _ = oracle_mod.precond_solve(D, g, 0.5, 1)
    assert np.allclose(y1, g / 3.5, rtol=1e-14)
    # bands are independent systems: with PSFs 3 delta and 5 delta one step gives
    # g_b / (c_b + sigma) in each band (one step length shared by both bands would not)
    D2 = np.zeros((2, 16, 16))
    D2[0, 8, 8], D2[1, 8, 8] = 3.0, 5.0
    g2 = np.random.default_rng(20).normal(size=(2, 8, 8))
    y2, _ = oracle_mod.precond_solve(D2, g2, 0.5, 1)
    assert np.allclose(y2[0], g2[0] / 3.5, rtol=1e-14) and np.allclose(y2[1], g2[1] / 5.5, rtol=1e-14)


def test_power_iteration_matches_eigvalsh(oracle_mod):
    """Power iteration (used for the Lipschitz constant behind the step size after
    eq. 8): on a symmetric matrix with a clear spectral gap it reaches numpy's
    eigvalsh; on the PSF operator (nearly degenerate top pair) it approaches the top
    eigenvalue from below."""
    rng = np.random.default_rng(21)
    Q, _ = np.linalg.qr(rng.normal(size=(40, 40)))
    ev = np.linspace(1.0, 5.0, 40)
    ev[-1] = 9.0
    S = (Q * ev) @ Q.T
    lam, v = oracle_mod.power_iteration(lambda z: S @ z, rng.normal(size=40), 200)
    assert abs(lam - 9.0) < 1e-12 * 9.0
    assert abs(abs(np.dot(v, Q[:, -1])) - 1.0) < 1e-10
    p = _small(seed=20, nx=8, ny=8, n_row=40)
    P = oracle_mod.psf(p)
    M = _dense_psf_matrix(oracle_mod, P)
    ref = np.linalg.eigvalsh(0.5 * (M + M.T)).max()
    lam, _ = oracle_mod.power_iteration(lambda v: oracle_mod.psf_conv(P, v),
                                        rng.normal(size=(1, 8, 8)), 300)
    assert ref * (1 - 1e-2) < lam <= ref * (1 + 1e-12)


def test_fb_steps_decrease_the_objective(oracle_mod):
    """With gamma <= 1 < 2 / L_U the preconditioned forward-backward iteration
    (eqs. 6-7) decreases 1/2 x^T (I^psf * x) - x^T I^d + lam ||x||_1 monotonically,
    and a fixed point of the step is returned unchanged."""
    p = _small(seed=22, nx=16, ny=16, n_row=60)
    P = oracle_mod.psf(p)
    x_true = synth.point_sky(22, 1, 16, 16, n_src=4)
    dirty = oracle_mod.hessian(p, x_true, flat=True)
    lam_max, _ = oracle_mod.power_iteration(lambda v: oracle_mod.psf_conv(P, v),
                                            np.ones((1, 16, 16)), 50)
    sigma, gamma, lam = 1e-3 * lam_max, 1.0, 1e-3

    def obj(x):
        return 0.5 * np.sum(x * oracle_mod.psf_conv(P, x)) - np.sum(x * dirty) + lam * np.abs(x).sum()

    x = np.zeros((1, 16, 16))
    vals = [obj(x)]
    for _ in range(6):
        x = oracle_mod.fb_step(P, dirty, x, sigma, gamma, lam, 60)
        vals.append(obj(x))
    assert np.all(np.diff(vals) < 1e-9 * abs(vals[0] - vals[-1]))
    assert vals[-1] < vals[0]
    # zero image, zero dirty image: x = 0 is a fixed point
    z = oracle_mod.fb_step(P, np.zeros_like(dirty), np.zeros_like(dirty), sigma, gamma, lam, 10)
    assert np.all(z == 0)


@pytest.mark.parametrize("gamma", [0.5, 1.7])
def test_fb_step_scaled_delta_psf_closed_form(oracle_mod, gamma):
    """I^psf = c_b delta in band b makes U = (c_b + sigma) Id (eq. 8), so the CG solve is
    exact after one step and the forward-backward step (eq. 6, then the l1 + positivity
    prox standing in for eq. 7) has the closed form
    max(x - gamma (c_b x - I^d) / (c_b + sigma) - gamma lam, 0).  gamma != 1 separates the
    threshold gamma lam from lam; the bands have different c_b, so one step length
    shared by both bands would fail."""
    rng = np.random.default_rng(41)
    nb, nx, ny = 2, 8, 6
    c = np.array([2.5, 4.0])
    sigma, lam = 0.3, 0.2
    D = np.zeros((nb, 2 * nx, 2 * ny))
    D[:, nx, ny] = c
    x = rng.uniform(0.0, 1.0, (nb, nx, ny))
    dirty = rng.normal(0.0, 2.0, (nb, nx, ny))
    out = oracle_mod.fb_step(D, dirty, x, sigma, gamma, lam, 3)
    cb = c[:, None, None]
    ref = np.maximum(x - gamma * (cb * x - dirty) / (cb + sigma) - gamma * lam, 0.0)
    assert np.abs(out - ref).max() < 1e-12
    # positivity is enforced and active; the threshold leaves some pixels positive
    assert (out >= 0).all() and (out == 0).any() and (out > 0).any()


def test_factored_psf_equals_the_direct_sum(oracle_mod):
    """The matrix-product form of the PSF sum (each phase split over the two axes)
    agrees with the C direct sum, including the zeroed offset -n row and column, in
    several bands with flags and a non-square image."""
    p = synth.tiny_problem(seed=51, nx=24, ny=16, n_row=90, n_band=2, freqs=(1.0e9, 1.2e9, 1.3e9, 1.4e9),
                           flag_frac=0.2)
    ref = oracle_mod.psf(p)
    got = oracle_mod.psf_factored(p)
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


def test_fft_convolution_operator_equals_direct_sum_and_library(oracle_mod):
    """psf_conv_op (period-2n FFT, spectrum computed once) equals the plain O(N^4)
    sum and scipy's full linear convolution, for several bands and a non-square
    image; the CG and FB step give the same result with either convolution."""
    p = synth.tiny_problem(seed=52, nx=12, ny=10, n_row=50, n_band=2, freqs=(1.0e9, 1.2e9))
    P = oracle_mod.psf(p)
    x = np.random.default_rng(53).normal(size=(2, 12, 10))
    op = oracle_mod.psf_conv_op(P)
    y = op(x)
    for b in range(2):
        d = oracle_mod.psf_conv_direct(P[b], x[b])
        assert np.abs(y[b] - d).max() < 1e-12 * np.abs(d).max()
    assert np.abs(y - oracle_mod.psf_conv(P, x)).max() < 1e-12 * np.abs(y).max()
    g = np.random.default_rng(54).normal(size=(2, 12, 10))
    y1, t1 = oracle_mod.precond_solve(P, g, 0.3, 7)
    y2, t2 = oracle_mod.precond_solve(P, g, 0.3, 7, conv=op)
    assert np.abs(y1 - y2).max() < 1e-10 * np.abs(y1).max()
    x0 = np.abs(x)
    f1 = oracle_mod.fb_step(P, g, x0, 0.3, 0.8, 0.01, 5)
    f2 = oracle_mod.fb_step(P, g, x0, 0.3, 0.8, 0.01, 5, conv=op)
    assert np.abs(f1 - f2).max() < 1e-10 * np.abs(f1).max()
