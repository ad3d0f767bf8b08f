"""GPU parity of every C-ABI operator against the FP64 oracle, element by element,
on seeded inputs (rel-l2 <= 1e-5 for the FP32 path, <= 1e-10 for FP64 mode).

Operators (Bester et al. 2021, Section 2): dirty image R^dagger Sigma^-1 V,
degridding R x (eq. 1), Hessian R^dagger Sigma^-1 R x (eq. 3), PSF and PSF
convolution (eq. 4), the CG solve of U y = g with U = I^psf * + sigma Id (eq. 8),
power iteration, and one forward-backward step (eqs. 6-7).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, host, make_plan, rel, say, to_dev

pytestmark = pytest.mark.gpu

PRECISIONS = ["fp64", "fp32"]


def _dtypes(prec):
    import torch
    return (torch.float64, torch.complex128) if prec == "fp64" else (torch.float32, torch.complex64)


# --------------------------------------------------------------------------
# the tiny workload: 128 x 128, cell 10", 2 channels x 4096 rows, w ~ N(0, 0.1 |u|max)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def tiny():
    prob = synth.workload("tiny-128")
    seed = synth.SEED_BASE
    x = synth.point_sky(seed, 1, 128, 128, n_src=10)
    vis = oracle.degrid(prob, x) + synth.complex_noise(seed, (prob.n_row, prob.n_chan), 0.01)
    rng = np.random.default_rng(11)
    xd = rng.normal(size=(1, 128, 128))
    say("oracle: tiny workload references")
    ref = dict(prob=prob, x=x, vis=vis, xd=xd,
               dirty=oracle.grid(prob, vis),
               degrid=oracle.degrid(prob, xd),
               hess=oracle.hessian(prob, xd),
               psf=oracle.psf(prob))
    ref["conv"] = oracle.psf_conv(ref["psf"], xd)
    return ref


@pytest.fixture(scope="module", params=PRECISIONS)
def tiny_plan(request, tiny):
    say(f"plan: tiny-128 {request.param}")
    plan = make_plan(tiny["prob"], request.param)
    plan.make_psf(want_image=False)
    return request.param, plan


def test_dirty_image(tiny, tiny_plan):
    prec, plan = tiny_plan
    R, C = _dtypes(prec)
    say(f"grid {prec}")
    img = host(plan.grid(to_dev(tiny["vis"], C)))
    assert rel(img, tiny["dirty"]) < TOL[prec]


def test_degrid(tiny, tiny_plan):
    prec, plan = tiny_plan
    R, C = _dtypes(prec)
    say(f"degrid {prec}")
    v = host(plan.degrid(to_dev(tiny["xd"], R)))
    assert rel(v, tiny["degrid"]) < TOL[prec]


def test_hessian(tiny, tiny_plan):
    prec, plan = tiny_plan
    R, C = _dtypes(prec)
    say(f"hessian {prec}")
    y = host(plan.hessian(to_dev(tiny["xd"], R)))
    assert rel(y, tiny["hess"]) < TOL[prec]


def test_psf(tiny, tiny_plan):
    prec, plan = tiny_plan
    say(f"psf {prec}")
    p = host(plan.make_psf())
    assert rel(p, tiny["psf"]) < TOL[prec]
    sw = tiny["prob"].effective_weight().sum()
    assert abs(p[0, 128, 128] - sw) < TOL[prec] * sw * 10
    assert np.all(p[0, 0, :] == 0) and np.all(p[0, :, 0] == 0)


def test_psf_conv(tiny, tiny_plan):
    prec, plan = tiny_plan
    R, C = _dtypes(prec)
    say(f"psf_conv {prec}")
    y = host(plan.psf_conv(to_dev(tiny["xd"], R)))
    assert rel(y, tiny["conv"]) < TOL[prec]


def test_precond_solve_and_fb_step(tiny, tiny_plan):
    prec, plan = tiny_plan
    R, C = _dtypes(prec)
    psf = tiny["psf"]
    lam_max, _ = oracle.power_iteration(lambda v: oracle.psf_conv(psf, v), np.ones((1, 128, 128)), 40)
    sigma, iters = 1e-1 * lam_max, 10
    g = tiny["xd"]
    say(f"precond_solve {prec}")
    import torch
    resid = torch.empty(1, dtype=torch.float64, device="cuda")
    y = host(plan.precond_solve(to_dev(g, R), sigma, iters, resid=resid))
    y_ref, trace = oracle.precond_solve(psf, g, sigma, iters)
    assert rel(y, y_ref) < 10 * TOL[prec]
    assert abs(host(resid)[0] - trace[0][-1]) < 1e-3 * trace[0][0]
    say(f"fb_step {prec}")
    dirty = tiny["dirty"]
    x0 = np.abs(tiny["xd"]) * 1e-3
    xg = to_dev(x0, R)
    plan.fb_step(to_dev(dirty, R), xg, sigma, 1.0, 1e-4, iters)
    x_ref = oracle.fb_step(psf, dirty, x0, sigma, 1.0, 1e-4, iters)
    assert rel(host(xg), x_ref) < 10 * TOL[prec]


def test_power_iteration(tiny, tiny_plan):
    prec, plan = tiny_plan
    R, C = _dtypes(prec)
    say(f"power_iteration {prec}")
    v0 = np.random.default_rng(5).normal(size=(1, 128, 128))
    lam = host(plan.power_iteration(to_dev(v0, R), 15))
    ref, _ = oracle.power_iteration(lambda v: oracle.psf_conv(tiny["psf"], v), v0, 15)
    assert abs(lam[0] - ref) < 10 * TOL[prec] * ref


def test_gpu_grid_degrid_are_adjoint(tiny, tiny_plan):
    """The GPU operators are exact mutual adjoints (same kernel, same correction)."""
    prec, plan = tiny_plan
    R, C = _dtypes(prec)
    rng = np.random.default_rng(12)
    x = rng.normal(size=(1, 128, 128))
    v = rng.normal(size=tiny["vis"].shape) + 1j * rng.normal(size=tiny["vis"].shape)
    Rx = host(plan.degrid(to_dev(x, R)))
    RtV = host(plan.grid(to_dev(v, C)))
    w = tiny["prob"].effective_weight()
    lhs = np.sum(w * np.conj(Rx) * v).real
    rhs = np.sum(x * RtV)
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert abs(lhs - rhs) < tol * (abs(lhs) + abs(rhs))


def test_fused_hessian_matches_grid_of_degrid(tiny, tiny_plan):
    prec, plan = tiny_plan
    R, C = _dtypes(prec)
    xg = to_dev(tiny["xd"], R)
    h = host(plan.hessian(xg))
    gd = host(plan.grid(plan.degrid(xg)))
    assert rel(h, gd) < (1e-13 if prec == "fp64" else 1e-6)


def test_fp32_tile16(tiny):
    """FP32 path with 16-cell tiles (the kernels' runtime tile side, not the
    specialised default of 32): dirty image, degrid and Hessian against the oracle."""
    import torch
    plan = make_plan(tiny["prob"], "fp32", tile=16)
    assert plan.info()["tile"] == 16
    assert rel(host(plan.grid(to_dev(tiny["vis"], torch.complex64))), tiny["dirty"]) < TOL["fp32"]
    assert rel(host(plan.degrid(to_dev(tiny["xd"], torch.float32))), tiny["degrid"]) < TOL["fp32"]
    assert rel(host(plan.hessian(to_dev(tiny["xd"], torch.float32))), tiny["hess"]) < TOL["fp32"]


@pytest.mark.parametrize("support,tol", [(5, 5e-4), (8, 1e-5)])
def test_fp32_other_supports(tiny, support, tol):
    """FP32 path at kernel supports other than the default 7: the interpolation's
    zero-weight columns (W = 5) and a full eight-column footprint (W = 8).  The
    tolerance is the ES kernel's own error at that support (about 3x the 1-D
    figure for the 3-D product), not a kernel error."""
    import torch
    plan = make_plan(tiny["prob"], "fp32", support=support)
    assert plan.info()["support"] == support
    assert rel(host(plan.degrid(to_dev(tiny["xd"], torch.float32))), tiny["degrid"]) < tol
    assert rel(host(plan.grid(to_dev(tiny["vis"], torch.complex64))), tiny["dirty"]) < tol
    assert rel(host(plan.hessian(to_dev(tiny["xd"], torch.float32))), tiny["hess"]) < tol


def test_independent_plans_are_bitwise_identical(tiny):
    """The plan-time entry order depends on the inputs only (radix sort on a
    total key), so two plans of one problem grid, degrid and apply the Hessian
    identically, bit for bit."""
    import torch
    outs = []
    for _ in range(2):
        plan = make_plan(tiny["prob"], "fp32")
        v = to_dev(tiny["vis"], torch.complex64)
        xg = to_dev(tiny["xd"], torch.float32)
        outs.append((host(plan.grid(v)), host(plan.degrid(xg)), host(plan.hessian(xg))))
        del plan
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


# --------------------------------------------------------------------------
# wider field, two bands, flags, non-square image, split work items
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def multi():
    prob = synth.tiny_problem(seed=77, nx=64, ny=32, n_row=700, freqs=(1.0e9, 1.1e9, 1.3e9, 1.4e9),
                              cell_arcsec=120.0, w_frac=1.5, n_band=2, flag_frac=0.2)
    rng = np.random.default_rng(78)
    x = rng.normal(size=(2, 64, 32))
    vis = rng.normal(size=(prob.n_row, prob.n_chan)) + 1j * rng.normal(size=(prob.n_row, prob.n_chan))
    say("oracle: multi-band references")
    psf = oracle.psf(prob)
    return dict(prob=prob, x=x, vis=vis, dirty=oracle.grid(prob, vis), degrid=oracle.degrid(prob, x),
                hess=oracle.hessian(prob, x), psf=psf, conv=oracle.psf_conv(psf, x))


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("chunk", [0, 64])
def test_multiband_all_operators(multi, prec, chunk):
    R, C = _dtypes(prec)
    say(f"plan: multi {prec} chunk={chunk}")
    plan = make_plan(multi["prob"], prec, chunk=chunk)
    info = plan.info()
    assert info["n_wplanes_max"] > 8          # several w-planes per band
    say("  grid / degrid / hessian / psf / conv")
    assert rel(host(plan.grid(to_dev(multi["vis"], C))), multi["dirty"]) < TOL[prec]
    v = host(plan.degrid(to_dev(multi["x"], R)))
    assert rel(v, multi["degrid"]) < TOL[prec]
    flagged = multi["prob"].effective_weight() == 0
    assert np.all(v[flagged] == 0)
    assert rel(host(plan.hessian(to_dev(multi["x"], R))), multi["hess"]) < TOL[prec]
    assert rel(host(plan.make_psf()), multi["psf"]) < TOL[prec]
    assert rel(host(plan.psf_conv(to_dev(multi["x"], R))), multi["conv"]) < TOL[prec]


@pytest.fixture(scope="module")
def three():
    prob = synth.tiny_problem(seed=79, nx=48, ny=40, n_row=500, freqs=(1.0e9, 1.05e9, 1.2e9, 1.25e9, 1.4e9, 1.45e9),
                              cell_arcsec=90.0, w_frac=1.0, n_band=3, flag_frac=0.15)
    rng = np.random.default_rng(80)
    x = rng.normal(size=(3, 48, 40))
    vis = rng.normal(size=(prob.n_row, prob.n_chan)) + 1j * rng.normal(size=(prob.n_row, prob.n_chan))
    say("oracle: three-band references")
    return dict(prob=prob, x=x, vis=vis, dirty=oracle.grid(prob, vis), degrid=oracle.degrid(prob, x),
                hess=oracle.hessian(prob, x))


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("band_batch", [1, 2])
def test_partial_band_batches(three, prec, band_batch):
    """Three bands with one or two bands' w-planes resident at a time: the batches
    start at bands 0, 1, 2 or 0, 2, so every per-band table (work lists, tile-row
    lists, flags) is read from a band offset and the last batch is short."""
    R, C = _dtypes(prec)
    plan = make_plan(three["prob"], prec, band_batch=band_batch)
    assert plan.info()["band_batch"] == band_batch
    assert rel(host(plan.grid(to_dev(three["vis"], C))), three["dirty"]) < TOL[prec]
    assert rel(host(plan.degrid(to_dev(three["x"], R))), three["degrid"]) < TOL[prec]
    assert rel(host(plan.hessian(to_dev(three["x"], R))), three["hess"]) < TOL[prec]


@pytest.mark.parametrize("prec", PRECISIONS)
def test_flat_mode_hessian_equals_psf_convolution(multi, prec):
    """Without w and 1/n the Hessian is exactly the PSF convolution (eq. 4 becomes exact)."""
    R, C = _dtypes(prec)
    plan = make_plan(multi["prob"], prec, flat=True)
    plan.make_psf(want_image=False)
    xg = to_dev(multi["x"], R)
    assert rel(host(plan.hessian(xg)), host(plan.psf_conv(xg))) < TOL[prec]
    ref = oracle.hessian(multi["prob"], multi["x"], flat=True)
    assert rel(host(plan.hessian(xg)), ref) < TOL[prec]


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", PRECISIONS)
def test_empty_band_and_wrapped_uv(prec):
    """Band 1 fully flagged (no visibilities); u, v beyond the grid's Nyquist extent
    wrap periodically, exactly as the pixel-grid direct sum does."""
    R, C = _dtypes(prec)
    prob = synth.tiny_problem(seed=90, nx=32, ny=32, n_row=300, freqs=(1.0e9, 1.2e9, 1.3e9, 1.5e9),
                              cell_arcsec=60.0, uv_frac=1.3, n_band=2)
    flag = np.zeros((prob.n_row, prob.n_chan), np.uint8)
    flag[:, 2:] = 1
    prob.flag = flag
    rng = np.random.default_rng(91)
    vis = rng.normal(size=flag.shape) + 1j * rng.normal(size=flag.shape)
    x = rng.normal(size=(2, 32, 32))
    plan = make_plan(prob, prec)
    d = host(plan.grid(to_dev(vis, C)))
    assert np.all(d[1] == 0)
    assert rel(d, oracle.grid(prob, vis)) < TOL[prec]
    v = host(plan.degrid(to_dev(x, R)))
    assert np.all(v[:, 2:] == 0)
    assert rel(v, oracle.degrid(prob, x)) < TOL[prec]
    p = host(plan.make_psf())
    assert np.all(p[1] == 0)


@pytest.mark.parametrize("prec", PRECISIONS)
def test_single_visibility(prec):
    R, C = _dtypes(prec)
    prob = synth.tiny_problem(seed=92, nx=16, ny=16, n_row=1, freqs=(1.4e9,), cell_arcsec=100.0)
    vis = np.array([[0.3 - 0.7j]])
    plan = make_plan(prob, prec)
    assert rel(host(plan.grid(to_dev(vis, C))), oracle.grid(prob, vis)) < TOL[prec]
    x = np.random.default_rng(93).normal(size=(1, 16, 16))
    assert rel(host(plan.degrid(to_dev(x, R))), oracle.degrid(prob, x)) < TOL[prec]


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("nx", [64, 512])
def test_sparse_tiles_at_corners_and_wrap(prec, nx):
    """Visibilities clustered on a tile corner and across the periodic edge, with
    w spread over several planes: most tiles and tile rows are empty (no spread
    items; the row transforms read them as zero or skip them; the column passes
    skip empty rows) while footprints straddle tiles next to empty ones and the
    interpolation halo wraps.  nx = 512 gives 1024-row columns (two-pass)."""
    R, C = _dtypes(prec)
    ny = 64
    prob = synth.tiny_problem(seed=97, nx=nx, ny=ny, n_row=240, freqs=(1.3e9,), cell_arcsec=20.0)
    rng = np.random.default_rng(98)
    gx, gy = 2 * nx, 2 * ny
    # grid coordinates (cells): half the rows near the corner (32, 96), half
    # near (0, gy - 1), i.e. across the wrap of both axes
    tu = np.where(np.arange(prob.n_row) < prob.n_row // 2, 32.0, 0.5) + rng.normal(0, 2.0, prob.n_row)
    tv = np.where(np.arange(prob.n_row) < prob.n_row // 2, 96.0, gy - 0.5) + rng.normal(0, 2.0, prob.n_row)
    lam = synth.C_LIGHT / prob.freq[0]
    u = tu / (prob.cellx * gx)
    v = tv / (prob.celly * gy)
    w = rng.normal(0.0, 6.0e4 * (64.0 / nx) ** 2, prob.n_row)   # a few w-planes at either size
    prob.uvw = np.stack([u, v, w], axis=1) * lam
    vis = rng.normal(size=(prob.n_row, 1)) + 1j * rng.normal(size=(prob.n_row, 1))
    x = rng.normal(size=(1, nx, ny))
    plan = make_plan(prob, prec)
    inf = plan.info()
    say(f"sparse tiles {prec} {nx}x{ny}: {inf['n_wplanes_max']} planes, occupied tiles "
        f"{inf['occ_tiles']} in {inf['occ_tile_rows']} tile rows, needed {inf['need_tiles']}")
    assert inf["n_wplanes_max"] >= 3
    assert inf["occ_tiles"] < inf["n_wplanes_total"] * (gx // inf["tile"]) * (gy // inf["tile"])
    if nx == 512:   # >= half of the tile rows empty: the column passes skip rows
        assert inf["occ_tile_rows"] * 2 <= inf["n_wplanes_total"] * (gx // inf["tile"])
    assert rel(host(plan.degrid(to_dev(x, R))), oracle.degrid(prob, x)) < TOL[prec]
    assert rel(host(plan.grid(to_dev(vis, C))), oracle.grid(prob, vis)) < TOL[prec]
    assert rel(host(plan.hessian(to_dev(x, R))), oracle.hessian(prob, x)) < TOL[prec]


def test_error_paths():
    from paper_2101_08072_amd import PfbError
    prob = synth.tiny_problem(seed=94, nx=16, ny=16, n_row=10)
    plan = make_plan(prob, "fp32")
    import torch
    x = torch.zeros((1, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(PfbError, match="PFB_ESTATE"):
        plan.psf_conv(x)
    bad = synth.Problem(**{**prob.__dict__, "nx": 23})      # odd side
    with pytest.raises(PfbError, match="PFB_EINVAL"):
        make_plan(bad, "fp32")
    with pytest.raises(PfbError, match="PFB_EINVAL"):
        make_plan(prob, "fp32", support=7, tile=4)
    wide = synth.Problem(**{**prob.__dict__, "cellx": 0.2, "celly": 0.2})
    with pytest.raises(PfbError, match="PFB_EINVAL"):
        make_plan(wide, "fp32")


# --------------------------------------------------------------------------
# rectangular image with long columns (operator grid 1024 x 512)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", PRECISIONS)
def test_long_columns_sampled(prec):
    """512 x 256 image: operator grid 1024 x 512 (1024-point columns as two
    512-point halves, more rows than columns) and PSF-convolution columns of
    1024; outputs checked on samples."""
    R, C = _dtypes(prec)
    prob = synth.tiny_problem(seed=95, nx=512, ny=256, n_row=1500, freqs=(1.0e9, 1.2e9),
                              cell_arcsec=8.0, w_frac=0.3, flag_frac=0.05)
    rng = np.random.default_rng(96)
    vis = rng.normal(size=(prob.n_row, prob.n_chan)) + 1j * rng.normal(size=(prob.n_row, prob.n_chan))
    x = np.zeros((1, 512, 256))
    x[0, rng.integers(0, 512, 30), rng.integers(0, 256, 30)] = rng.uniform(0.1, 1, 30)
    x[0, 200:260, 100:150] += rng.normal(size=(60, 50))
    plan = make_plan(prob, prec)
    say(f"long columns {prec}: info {plan.info()}")
    pix = rng.integers(0, 512 * 256, 300)
    d = host(plan.grid(to_dev(vis, C))).ravel()[pix]
    assert rel(d, oracle.grid(prob, vis, pix=pix)) < TOL[prec]
    active = np.flatnonzero(prob.effective_weight().ravel())
    sel = rng.choice(active, 300, replace=False)
    v = host(plan.degrid(to_dev(x, R))).ravel()[sel]
    assert rel(v, oracle.degrid(prob, x, sel=sel)) < TOL[prec]
    h = host(plan.hessian(to_dev(x, R))).ravel()[pix]
    assert rel(h, oracle.hessian(prob, x, pix=pix)) < TOL[prec]
    psf = host(plan.make_psf())
    ppix = rng.integers(0, 4 * 512 * 256, 300)
    assert rel(psf.ravel()[ppix], oracle.psf(prob, pix=ppix)) < TOL[prec]
    # convolution with the GPU's own PSF against the library convolution in FP64
    xr = rng.normal(size=(1, 512, 256))
    y = host(plan.psf_conv(to_dev(xr, R)))
    assert rel(y, oracle.psf_conv(psf.astype(np.float64), xr)) < TOL[prec]
