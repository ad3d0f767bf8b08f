"""Seeded synthetic inputs for the imaging operators.

This module only draws inputs: antenna layouts, uvw tracks, frequencies,
weights, flags, sky images and noise.  It contains none of the measurement
operator's arithmetic (no Fourier phases, no gridding), so both the FP64
oracle and the HIP library can consume what it produces without sharing any
of the method's code.

Shapes follow the paper's statement of the measurement operator
(Section 2, the map from n_b imaging bands of n_p pixels to n_nu channels of
n_d rows): visibilities are laid out ``[n_row][n_chan]``, images
``[n_band][nx][ny]`` with axis 0 along l.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_LIGHT = 299792458.0
ARCSEC = math.pi / (180.0 * 3600.0)
SEED_BASE = 210108072


@dataclasses.dataclass
class Problem:
    """Everything that defines R for one imaging job (inputs only)."""

    uvw: np.ndarray          # float64 [n_row][3], metres
    freq: np.ndarray         # float64 [n_chan], Hz
    weight: np.ndarray       # float32/float64 [n_row][n_chan] = diag(Sigma^-1)
    flag: np.ndarray | None  # uint8 [n_row][n_chan] or None
    chan_band: np.ndarray    # int32 [n_chan]
    n_band: int
    nx: int
    ny: int
    cellx: float             # radians
    celly: float             # radians

    @property
    def n_row(self) -> int:
        return int(self.uvw.shape[0])

    @property
    def n_chan(self) -> int:
        return int(self.freq.shape[0])

    def effective_weight(self) -> np.ndarray:
        """Weights with flagged entries set to zero (float64)."""
        w = self.weight.astype(np.float64, copy=True)
        if self.flag is not None:
            w[self.flag != 0] = 0.0
        return w


def contiguous_bands(n_chan: int, n_band: int) -> np.ndarray:
    """Channel -> band map with equal contiguous blocks (one band per spectral window)."""
    if n_chan % n_band:
        raise ValueError("n_chan must be a multiple of n_band")
    return (np.arange(n_chan) // (n_chan // n_band)).astype(np.int32)


# ---------------------------------------------------------------------------
# tiny configuration: uv uniform in a disk, w Gaussian
# ---------------------------------------------------------------------------

def tiny_problem(seed: int = SEED_BASE, nx: int = 128, ny: int = 128,
                 n_row: int = 4096, freqs=(1.0e9, 1.1e9), cell_arcsec: float = 10.0,
                 uv_frac: float = 0.4, w_frac: float = 0.1, n_band: int = 1,
                 flag_frac: float = 0.0) -> Problem:
    """u, v uniform in a disk of radius ``uv_frac/cell`` wavelengths at the highest
    frequency; w ~ N(0, w_frac * that radius); weights U[0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    freq = np.asarray(freqs, dtype=np.float64)
    cell = cell_arcsec * ARCSEC
    fmax = float(freq.max())
    rmax = uv_frac / cell                       # wavelengths at fmax
    r = rmax * np.sqrt(rng.uniform(0.0, 1.0, n_row))
    th = rng.uniform(0.0, 2.0 * math.pi, n_row)
    w = rng.normal(0.0, w_frac * rmax, n_row)
    uvw_lambda = np.stack([r * np.cos(th), r * np.sin(th), w], axis=1)
    uvw = uvw_lambda * (C_LIGHT / fmax)
    weight = rng.uniform(0.5, 1.5, (n_row, freq.size))
    flag = None
    if flag_frac > 0:
        flag = (rng.uniform(0.0, 1.0, (n_row, freq.size)) < flag_frac).astype(np.uint8)
    return Problem(uvw=uvw, freq=freq, weight=weight, flag=flag,
                   chan_band=contiguous_bands(freq.size, n_band), n_band=n_band,
                   nx=nx, ny=ny, cellx=cell, celly=cell)


def point_sky(seed: int, n_band: int, nx: int, ny: int, n_src: int = 10,
              flux=(0.1, 1.0), margin: int = 0, dtype=np.float64) -> np.ndarray:
    """``n_src`` point sources at random pixels with U(flux) amplitudes (same in every band)."""
    rng = np.random.default_rng(seed + 1000)
    x = np.zeros((n_band, nx, ny), dtype=dtype)
    ii = rng.integers(margin, nx - margin, n_src)
    jj = rng.integers(margin, ny - margin, n_src)
    a = rng.uniform(flux[0], flux[1], n_src)
    for i, j, f in zip(ii, jj, a):
        x[:, i, j] += f
    return x


def complex_noise(seed: int, shape, sigma: float) -> np.ndarray:
    """Circular complex Gaussian: Re and Im each N(0, sigma^2/2)."""
    rng = np.random.default_rng(seed + 2000)
    s = sigma / math.sqrt(2.0)
    return rng.normal(0.0, s, shape) + 1j * rng.normal(0.0, s, shape)


# ---------------------------------------------------------------------------
# earth-rotation generator (VLA-like array of 64 antennas)
# ---------------------------------------------------------------------------

def antenna_enu(seed: int, n_ant: int = 64, radius_m: float = 4000.0) -> np.ndarray:
    rng = np.random.default_rng(seed + 3000)
    r = radius_m * np.sqrt(rng.uniform(0.0, 1.0, n_ant))
    th = rng.uniform(0.0, 2.0 * math.pi, n_ant)
    return np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n_ant)], axis=1)


def earth_rotation_uvw(enu: np.ndarray, n_row: int, lat_deg: float = 34.0,
                       dec_deg: float = 40.0, ha_span_h: float = 4.0) -> np.ndarray:
    """Baseline uvw tracks in metres, time-major, truncated to ``n_row`` rows.

    Textbook ENU -> equatorial XYZ -> (u, v, w) rotation for hour angle H and
    declination delta (Thompson, Moran & Swenson, ch. 4)."""
    n_ant = enu.shape[0]
    a1, a2 = np.triu_indices(n_ant, 1)
    b = enu[a2] - enu[a1]                     # [n_bl][3] E, N, U
    lat = math.radians(lat_deg)
    X = -b[:, 1] * math.sin(lat) + b[:, 2] * math.cos(lat)
    Y = b[:, 0]
    Z = b[:, 1] * math.cos(lat) + b[:, 2] * math.sin(lat)
    n_bl = b.shape[0]
    n_t = -(-n_row // n_bl)
    H = np.linspace(-ha_span_h, ha_span_h, n_t) * (math.pi / 12.0)
    dec = math.radians(dec_deg)
    sH, cH = np.sin(H)[:, None], np.cos(H)[:, None]
    u = sH * X + cH * Y
    v = -math.sin(dec) * cH * X + math.sin(dec) * sH * Y + math.cos(dec) * Z
    w = math.cos(dec) * cH * X - math.cos(dec) * sH * Y + math.sin(dec) * Z
    uvw = np.stack([u.ravel(), v.ravel(), w.ravel()], axis=1)[:n_row]
    return np.ascontiguousarray(uvw)


def pareto_flux(rng, n, smin=1e-3, smax=1.0):
    """dN/dS ~ S^-2 on [smin, smax] by inverse CDF."""
    u = rng.uniform(0.0, 1.0, n)
    return 1.0 / (1.0 / smin - u * (1.0 / smin - 1.0 / smax))


def extended_sky(seed: int, n_band: int, nx: int, ny: int, n_pts: int = 500,
                 n_blobs: int = 20, margin: int = 16) -> np.ndarray:
    """500 point sources plus 20 circular Gaussian blobs with power-law fluxes (float32)."""
    rng = np.random.default_rng(seed + 4000)
    img = np.zeros((nx, ny), dtype=np.float64)
    ii = rng.integers(margin, nx - margin, n_pts)
    jj = rng.integers(margin, ny - margin, n_pts)
    np.add.at(img, (ii, jj), pareto_flux(rng, n_pts))
    for _ in range(n_blobs):
        ci = rng.integers(margin, nx - margin)
        cj = rng.integers(margin, ny - margin)
        sig = rng.uniform(2.0, 20.0)
        flux = pareto_flux(rng, 1)[0]
        h = int(min(4 * sig, nx // 2))
        i0, i1 = max(ci - h, 0), min(ci + h + 1, nx)
        j0, j1 = max(cj - h, 0), min(cj + h + 1, ny)
        gi = np.arange(i0, i1)[:, None] - ci
        gj = np.arange(j0, j1)[None, :] - cj
        g = np.exp(-(gi * gi + gj * gj) / (2.0 * sig * sig))
        img[i0:i1, j0:j1] += flux * g / g.sum()
    return np.broadcast_to(img.astype(np.float32), (n_band, nx, ny)).copy()


def rotation_problem(seed: int, nx: int, n_row: int, n_chan: int, n_band: int = 1,
                     fov_deg: float = 1.0, f_lo: float = 0.9e9, f_hi: float = 1.7e9,
                     flag_frac=0.10, per_band_flag=None, weight_dtype=np.float32) -> Problem:
    """Synthetic VLA-like problem; ``per_band_flag`` = (lo, hi) draws a flag fraction
    per band from U(lo, hi) so visibility counts per band are uneven."""
    rng = np.random.default_rng(seed)
    uvw = earth_rotation_uvw(antenna_enu(seed), n_row)
    freq = np.linspace(f_lo, f_hi, n_chan)
    cell = math.radians(fov_deg) / nx
    weight = rng.uniform(0.5, 1.5, (n_row, n_chan)).astype(weight_dtype)
    chan_band = contiguous_bands(n_chan, n_band)
    if per_band_flag is not None:
        frac = rng.uniform(per_band_flag[0], per_band_flag[1], n_band)
        p = frac[chan_band][None, :]
    else:
        p = flag_frac
    flag = (rng.uniform(0.0, 1.0, (n_row, n_chan)) < p).astype(np.uint8)
    return Problem(uvw=uvw, freq=freq, weight=weight, flag=flag, chan_band=chan_band,
                   n_band=n_band, nx=nx, ny=nx, cellx=cell, celly=cell)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

WORKLOADS = {
    # name: (builder, kwargs)
    "tiny-128": dict(kind="tiny"),
    "single-band-2048": dict(kind="rotation", nx=2048, n_row=1_000_000, n_chan=64, n_band=1),
    "precision-4096": dict(kind="rotation", nx=4096, n_row=2_000_000, n_chan=128, n_band=1),
    "batched-8x4096": dict(kind="rotation", nx=4096, n_row=1_000_000, n_chan=256, n_band=8,
                           per_band_flag=(0.0, 0.6)),
}


def workload(name: str, seed: int | None = None, **over) -> Problem:
    spec = dict(WORKLOADS[name])
    spec.update(over)
    kind = spec.pop("kind")
    idx = list(WORKLOADS).index(name)
    seed = SEED_BASE + idx if seed is None else seed
    if kind == "tiny":
        return tiny_problem(seed=seed, **spec)
    return rotation_problem(seed=seed, **spec)
