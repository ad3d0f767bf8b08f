"""FP64 reference ("oracle") for the pfb-clean hot path.

TEST INFRASTRUCTURE ONLY: the product package never imports, links or runs
anything under ``oracle/``.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

Everything here follows Bester et al., "A practical preconditioner for
wide-field continuum imaging of radio interferometric data", Section 2:

* ``degrid``      R x                       (eq. 1, the measurement operator)
* ``grid``        R^dagger Sigma^-1 V       (the dirty image I^d, after eq. 3)
* ``hessian``     R^dagger Sigma^-1 R x     (eq. 3)
* ``fidelity``    f(x)                      (eq. 2)
* ``gradient``    exact gradient            (eq. 3)
* ``psf``         I^psf, flat, 2nx x 2ny    (eq. 4)
* ``psf_factored`` the same sum with each phase factor split over the two axes
                  (a matrix product; for large images with few visibilities)
* ``psf_conv``    I^psf * x, linear         (eq. 4)
* ``psf_conv_op`` the same convolution by FFT with the PSF spectrum computed once
* ``cg``          conjugate gradient on U = I^psf * + sigma Id    (eq. 8 and the text after it)
* ``power_iteration``  largest eigenvalue of a symmetric operator (step-size rationale after eq. 8)
* ``fb_step``     one forward (eq. 6) and Euclidean l1+positivity backward step

R itself is the plain direct sum that the paper's w-corrected 2-D NUFFT
approximates (C file ``pfb_oracle.c``), evaluated in FP64 with compensated
summation.  A dense-matrix twin (``dense_operator``) written separately in
NumPy serves as brute force at tiny sizes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

C0 = 299792458.0


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc + OpenMP (plain C, -O2, no fast-math)."""
    src = os.path.join(_HERE, "pfb_oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        os.makedirs(os.path.dirname(_SO), exist_ok=True)
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        i64, i32p, dp, i64p = ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), \
            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
        ci, cd = ctypes.c_int, ctypes.c_double
        lib.oracle_degrid.argtypes = [i64, i64, i32p, dp, dp, dp, ci, ci, cd, cd, ci,
                                      i64, i64p, dp, i64, i64p, dp]
        lib.oracle_grid.argtypes = [i64, i64, i32p, dp, dp, dp, ci, ci, cd, cd, ci,
                                    dp, i64, i64p, dp]
        lib.oracle_psf.argtypes = [i64, i64, i32p, dp, dp, dp, ci, ci, cd, cd, i64, i64p, dp]
        lib.oracle_threads.restype = ci
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().oracle_threads())


def _p(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _common(prob):
    cb = np.ascontiguousarray(prob.chan_band, dtype=np.int32)
    fr = np.ascontiguousarray(prob.freq, dtype=np.float64)
    uvw = np.ascontiguousarray(prob.uvw, dtype=np.float64)
    wt = np.ascontiguousarray(prob.effective_weight(), dtype=np.float64)
    return cb, fr, uvw, wt


def degrid(prob, x, sel=None, flat=False):
    """V = R x at the selected visibilities (sel = flat indices r*n_chan+c; None = all).

    ``x`` is a dense image [n_band][nx][ny]; only its nonzero pixels enter the sum.
    Flagged / zero-weight entries return 0."""
    lib = _load()
    cb, fr, uvw, wt = _common(prob)
    x = np.asarray(x, dtype=np.float64).reshape(prob.n_band, prob.nx, prob.ny)
    pix = np.flatnonzero(x).astype(np.int64)
    val = np.ascontiguousarray(x.ravel()[pix])
    full = sel is None
    if full:
        sel = np.arange(prob.n_row * prob.n_chan, dtype=np.int64)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    out = np.zeros(2 * sel.size)
    lib.oracle_degrid(prob.n_row, prob.n_chan, _p(cb, ctypes.c_int32), _p(fr), _p(uvw), _p(wt),
                      prob.nx, prob.ny, prob.cellx, prob.celly, int(flat),
                      pix.size, _p(pix, ctypes.c_int64), _p(val),
                      sel.size, _p(sel, ctypes.c_int64), _p(out))
    v = out[0::2] + 1j * out[1::2]
    return v.reshape(prob.n_row, prob.n_chan) if full else v


def grid(prob, vis, pix=None, flat=False):
    """I^d = Re R^dagger Sigma^-1 V at the selected pixels (flat b*nx*ny+i*ny+j; None = all)."""
    lib = _load()
    cb, fr, uvw, wt = _common(prob)
    v = np.asarray(vis, dtype=np.complex128).reshape(prob.n_row, prob.n_chan)
    vv = np.ascontiguousarray(np.stack([v.real, v.imag], axis=-1))
    full = pix is None
    if full:
        pix = np.arange(prob.n_band * prob.nx * prob.ny, dtype=np.int64)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    out = np.zeros(pix.size)
    lib.oracle_grid(prob.n_row, prob.n_chan, _p(cb, ctypes.c_int32), _p(fr), _p(uvw), _p(wt),
                    prob.nx, prob.ny, prob.cellx, prob.celly, int(flat),
                    _p(vv), pix.size, _p(pix, ctypes.c_int64), _p(out))
    return out.reshape(prob.n_band, prob.nx, prob.ny) if full else out


def hessian(prob, x, pix=None, flat=False):
    """R^dagger Sigma^-1 R x (eq. 3): the dirty image of the noise-free visibilities of x."""
    return grid(prob, degrid(prob, x, flat=flat), pix=pix, flat=flat)


def psf(prob, pix=None):
    """Flat PSF of every band on the 2nx x 2ny grid (peak sum of weights at (nx, ny))."""
    lib = _load()
    cb, fr, uvw, wt = _common(prob)
    NX, NY = 2 * prob.nx, 2 * prob.ny
    full = pix is None
    if full:
        pix = np.arange(prob.n_band * NX * NY, dtype=np.int64)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    out = np.zeros(pix.size)
    lib.oracle_psf(prob.n_row, prob.n_chan, _p(cb, ctypes.c_int32), _p(fr), _p(uvw), _p(wt),
                   prob.nx, prob.ny, prob.cellx, prob.celly, pix.size, _p(pix, ctypes.c_int64),
                   _p(out))
    return out.reshape(prob.n_band, NX, NY) if full else out


def psf_factored(prob):
    """The flat PSF of ``psf`` evaluated as a matrix product (eq. 4).

    The phase of the PSF sum is u dl + v dm, so each term
    w cos(2 pi (u dl + v dm)) is the real part of w e^{2 pi i u dl} e^{2 pi i v dm}:
    PSF_b = Re(E_l^T diag(w) E_m) over the visibilities of band b, with
    E_l[k, i'] = e^{2 pi i u_k dl_i'} and E_m[k, j'] = e^{2 pi i v_k dm_j'}.  Phases are
    reduced by their nearest integer in FP64 before the exponential; row 0 and
    column 0 (offset -nx, -ny) are zero.  Exact in exact arithmetic; the cost is a
    (2nx x K) by (K x 2ny) product, so it serves images too large for the
    per-pixel direct sum when the visibility count K is small."""
    wt = prob.effective_weight()
    NX, NY = 2 * prob.nx, 2 * prob.ny
    dl = (np.arange(NX) - prob.nx) * prob.cellx
    dm = (np.arange(NY) - prob.ny) * prob.celly
    out = np.zeros((prob.n_band, NX, NY))
    for b in range(prob.n_band):
        rr, cc = np.nonzero(wt * (prob.chan_band[None, :] == b))
        if rr.size == 0:
            continue
        s = prob.freq[cc] / C0
        u = prob.uvw[rr, 0] * s
        v = prob.uvw[rr, 1] * s
        tl = np.outer(u, dl)
        tm = np.outer(v, dm)
        El = np.exp(2j * np.pi * (tl - np.rint(tl))) * wt[rr, cc][:, None]
        Em = np.exp(2j * np.pi * (tm - np.rint(tm)))
        out[b] = (El.T @ Em).real
    out[:, 0, :] = 0.0
    out[:, :, 0] = 0.0
    return out


def fidelity(prob, x, vis):
    """f(x) = 1/2 (V - Rx)^H Sigma^-1 (V - Rx)   (eq. 2)."""
    r = np.asarray(vis).reshape(prob.n_row, prob.n_chan) - degrid(prob, x)
    return 0.5 * float(np.sum(prob.effective_weight() * (r.real ** 2 + r.imag ** 2)))


def gradient(prob, x, vis):
    """Exact gradient R^dagger Sigma^-1 R x - I^d   (eq. 3)."""
    return hessian(prob, x) - grid(prob, vis)


# ---------------------------------------------------------------------------
# dense twin (brute force, tiny sizes only)
# ---------------------------------------------------------------------------

def dense_operator(prob, flat=False):
    """Return (A, W, rows, bands): A[k, b*P + p] for active visibility k; W its weights.

    Built with NumPy broadcasting, independently of the C loops."""
    wt = prob.effective_weight()
    rr, cc = np.nonzero(wt)
    lam = C0 / prob.freq[cc]
    u = prob.uvw[rr, 0] / lam
    v = prob.uvw[rr, 1] / lam
    w = prob.uvw[rr, 2] / lam
    li = (np.arange(prob.nx) - prob.nx // 2) * prob.cellx
    mj = (np.arange(prob.ny) - prob.ny // 2) * prob.celly
    L, M = np.meshgrid(li, mj, indexing="ij")
    N = np.sqrt(1.0 - L * L - M * M)
    S = -(L * L + M * M) / (1.0 + N)      # n - 1 without cancellation
    L, M, N, S = L.ravel(), M.ravel(), N.ravel(), S.ravel()
    ph = np.outer(u, L) + np.outer(v, M)
    if not flat:
        ph = ph + np.outer(w, S)
    blk = np.exp(-2j * np.pi * ph)
    if not flat:
        blk = blk / N[None, :]
    P = prob.nx * prob.ny
    A = np.zeros((rr.size, prob.n_band * P), dtype=np.complex128)
    b = prob.chan_band[cc]
    for band in range(prob.n_band):
        k = b == band
        A[k, band * P:(band + 1) * P] = blk[k]
    return A, wt[rr, cc], rr * prob.n_chan + cc


# ---------------------------------------------------------------------------
# PSF convolution and the preconditioned solve
# ---------------------------------------------------------------------------

def psf_conv_direct(psf_b, x_b):
    """y[i,j] = sum_{i2,j2} PSF[i-i2+nx, j-j2+ny] x[i2,j2]  (plain O(N^4) sum, one band)."""
    nx, ny = x_b.shape
    y = np.zeros((nx, ny))
    for i2 in range(nx):
        for j2 in range(ny):
            a = x_b[i2, j2]
            if a != 0.0:
                y += a * psf_b[nx - i2:2 * nx - i2, ny - j2:2 * ny - j2]
    return y


def psf_conv(psf_img, x):
    """Linear convolution with the PSF, cropped to the image (eq. 4), FP64, every band.

    Uses ``scipy.signal.fftconvolve`` in 'full' mode as the library convolution."""
    from scipy.signal import fftconvolve
    psf_img = np.asarray(psf_img, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    nb, nx, ny = x.shape
    out = np.empty_like(x)
    for b in range(nb):
        full = fftconvolve(psf_img[b], x[b], mode="full")
        out[b] = full[nx:2 * nx, ny:2 * ny]
    return out


def psf_conv_op(psf_img):
    """I^psf * (eq. 4) as a function of x, by FFT with the PSF spectrum computed once.

    For output pixels i in [n, 2n) and inputs i2 in [0, n) the offset i - i2 lies in
    [1, 2n - 1], so the circular convolution of period 2n (per axis) of the 2n x 2n
    PSF with the zero-padded image, cropped to [n, 2n), is the linear convolution of
    ``psf_conv`` exactly: no offset wraps.  scipy.fft (all cores) is the library FFT."""
    import scipy.fft as sfft
    psf_img = np.asarray(psf_img, dtype=np.float64)
    nb, NX, NY = psf_img.shape
    nx, ny = NX // 2, NY // 2
    spec = [sfft.rfft2(psf_img[b], workers=-1) for b in range(nb)]

    def band(b, v):
        xs = sfft.rfft2(np.asarray(v, dtype=np.float64), s=(NX, NY), workers=-1)
        xs *= spec[b]
        return sfft.irfft2(xs, s=(NX, NY), workers=-1)[nx:, ny:].copy()

    def apply(x):
        x = np.asarray(x, dtype=np.float64).reshape(nb, nx, ny)
        return np.stack([band(b, x[b]) for b in range(nb)])
    apply.band = band
    return apply


def cg(apply_A, g, iters, y0=None):
    """Conjugate gradient for A y = g from y0 = 0, a fixed number of iterations.

    Returns (y, residual norms^2 per iteration).  Scalars and vectors in FP64."""
    g = np.asarray(g, dtype=np.float64)
    y = np.zeros_like(g) if y0 is None else np.array(y0, dtype=np.float64)
    r = g - apply_A(y) if y0 is not None else g.copy()
    p = r.copy()
    rr = float(np.vdot(r, r))
    trace = [rr]
    for _ in range(iters):
        if rr == 0.0:
            break
        Ap = apply_A(p)
        alpha = rr / float(np.vdot(p, Ap))
        y = y + alpha * p
        r = r - alpha * Ap
        rr_new = float(np.vdot(r, r))
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        trace.append(rr)
    return y, np.array(trace)


def precond_solve(psf_img, g, sigma, iters, conv=None):
    """y ~= (I^psf * + sigma Id)^-1 g by ``iters`` CG steps (eq. 8 and the text after it).

    U acts on every band with that band's PSF (eq. 4), so the system is
    block-diagonal over bands; each band's system gets its own CG (its own step
    lengths).  ``conv``: the PSF convolution of all bands as a function (default
    ``psf_conv`` of ``psf_img``; e.g. ``psf_conv_op(psf_img)`` for large images).
    Returns (y, residual norms^2 with shape (n_band, iterations + 1))."""
    g = np.asarray(g, dtype=np.float64)
    psf_img = np.asarray(psf_img, dtype=np.float64)
    nb = g.shape[0]
    ys, traces = [], []
    for b in range(nb):
        if conv is None:
            pb = psf_img[b:b + 1]
            conv_b = lambda v, pb=pb: psf_conv(pb, v[None])[0]  # noqa: E731
        elif hasattr(conv, "band"):
            conv_b = lambda v, b=b: conv.band(b, v)  # noqa: E731
        else:
            def conv_b(v, b=b):
                full = np.zeros((nb,) + v.shape)
                full[b] = v
                return conv(full)[b]
        yb, tb = cg(lambda v: conv_b(v) + sigma * v, g[b], iters)
        ys.append(yb)
        traces.append(tb)
    n = max(len(t) for t in traces)
    trace = np.array([np.pad(t, (0, n - len(t)), mode="edge") for t in traces])
    return np.stack(ys), trace


def power_iteration(apply_A, v0, iters):
    """v <- A v / ||A v||; returns (lambda = v^T A v, v)."""
    v = np.asarray(v0, dtype=np.float64)
    v = v / math.sqrt(float(np.vdot(v, v)))
    for _ in range(iters):
        Av = apply_A(v)
        v = Av / math.sqrt(float(np.vdot(Av, Av)))
    return float(np.vdot(v, apply_A(v))), v


def fb_step(psf_img, dirty, x, sigma, gamma, lam, cg_iters, conv=None):
    """One preconditioned forward-backward step with the PSF-approximate gradient.

    forward  (eq. 6): x_half = x - gamma U^-1 (I^psf * x - I^d), U = I^psf * + sigma Id
    backward (eq. 7 with U replaced by the identity): prox of gamma(lam ||.||_1 + positivity)
             = max(x_half - gamma lam, 0).
    ``conv`` as for ``precond_solve``."""
    conv = conv or (lambda v: psf_conv(psf_img, v))
    grad = conv(x) - dirty
    y, _ = precond_solve(psf_img, grad, sigma, cg_iters, conv=conv)
    x_half = x - gamma * y
    return np.maximum(x_half - gamma * lam, 0.0)


def rel_l2(a, b):
    """||a - b||_2 / ||b||_2 over all entries (complex counts Re and Im)."""
    a = np.asarray(a)
    b = np.asarray(b)
    num = np.linalg.norm((a - b).ravel())
    den = np.linalg.norm(b.ravel())
    return float(num / den) if den > 0 else float(num)
