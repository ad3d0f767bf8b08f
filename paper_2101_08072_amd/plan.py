"""Python binding of the pfb C ABI: one ``Plan`` per imaging problem.

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of every operator runs in the library's own kernels.
The names follow ``include/pfb.h`` (and through it the paper's Section 2).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib


@dataclass
class Options:
    precision: str = "fp32"     # "fp32" or "fp64"
    support: int = 0            # ES kernel support W (0 = default: 7 fp32, 13 fp64)
    tile: int = 0               # uv tile side (0 = default: 32 fp32, 8 fp64)
    flat: bool = False          # drop the w term and 1/n (w = 0, n = 1)
    band_batch: int = 0         # bands whose w-planes are resident together (0 = all that fit)
    chunk: int = 0              # bucket entries per work item (0 = entries / compute units)
    epsilon: float = 0.0        # requested grid/degrid accuracy: picks the support when support = 0

    def to_c(self) -> _lib.PfbOptions:
        o = _lib.PfbOptions()
        o.precision = _lib.PFB_FP64 if self.precision == "fp64" else _lib.PFB_FP32
        o.support = int(self.support)
        o.oversample = 2.0
        o.tile = int(self.tile)
        o.flat = int(bool(self.flat))
        o.band_batch = int(self.band_batch)
        o.chunk = int(self.chunk)
        o.epsilon = float(self.epsilon)
        return o


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Plan:
    """Holds one problem's plan and its device workspace (a torch uint8 tensor).

    Inputs (device tensors): uvw float64 [n_row, 3] metres; weight float32/float64
    [n_row, n_chan]; flag uint8 [n_row, n_chan] or None.  Host arrays: freq
    float64 [n_chan] Hz, chan_band int32 [n_chan].  The plan keeps references to
    the device tensors (the library borrows them)."""

    def __init__(self, uvw, freq, weight, flag, chan_band, n_band, nx, ny, cellx, celly,
                 options: Options | None = None, count_scratch: torch.Tensor | str | None = None,
                 offset: tuple[int, int] = (0, 0)):
        self.lib = _lib.load()
        self.opt = options or Options()
        self.real = torch.float64 if self.opt.precision == "fp64" else torch.float32
        self.cplx = torch.complex128 if self.opt.precision == "fp64" else torch.complex64
        if not (uvw.is_cuda and weight.is_cuda and (flag is None or flag.is_cuda)):
            raise ValueError("uvw, weight and flag must be device tensors")
        self.uvw = uvw.contiguous()
        self.weight = weight.contiguous()
        if self.weight.dtype != self.real:
            raise ValueError(f"weight must be {self.real} for precision {self.opt.precision}")
        self.flag = None if flag is None else flag.contiguous()
        self.freq = np.ascontiguousarray(freq, dtype=np.float64)
        self.chan_band = np.ascontiguousarray(chan_band, dtype=np.int32)
        self.n_row, self.n_chan = int(self.uvw.shape[0]), int(self.freq.size)
        self.n_band, self.nx, self.ny = int(n_band), int(nx), int(ny)
        if tuple(self.weight.shape) != (self.n_row, self.n_chan):
            raise ValueError("weight shape must be [n_row, n_chan]")
        prob = _lib.PfbProblem()
        prob.n_row, prob.n_chan, prob.n_band = self.n_row, self.n_chan, self.n_band
        prob.chan_band = self.chan_band.ctypes.data
        prob.freq = self.freq.ctypes.data
        prob.uvw = self.uvw.data_ptr()
        prob.weight = self.weight.data_ptr()
        prob.flag = 0 if self.flag is None else self.flag.data_ptr()
        prob.nx, prob.ny = self.nx, self.ny
        prob.cellx, prob.celly = float(cellx), float(celly)
        prob.offx, prob.offy = int(offset[0]), int(offset[1])   # facet: centre pixel's offset
        self._prob = prob
        copt = self.opt.to_c()
        handle = ctypes.c_void_p()
        _lib.check(self.lib.pfb_plan_create(ctypes.byref(handle), ctypes.byref(prob),
                                            ctypes.byref(copt), _stream()))
        self.handle = handle
        # counting pass in a scratch buffer the caller may provide (it is free again on
        # return), or with count_scratch="static" in the library's fixed device buffer
        if isinstance(count_scratch, str):
            if count_scratch != "static":
                raise ValueError("count_scratch must be a device tensor, None or 'static'")
            _lib.check(self.lib.pfb_plan_count_static(self.handle, _stream()))
        else:
            cbytes = ctypes.c_size_t()
            _lib.check(self.lib.pfb_plan_count_scratch_size(self.handle, ctypes.byref(cbytes)))
            if count_scratch is None or count_scratch.numel() < cbytes.value:
                count_scratch = torch.empty(max(int(cbytes.value), 256), dtype=torch.uint8, device=self.uvw.device)
            _lib.check(self.lib.pfb_plan_count(self.handle, _ptr(count_scratch), count_scratch.numel(), _stream()))
            del count_scratch
        nbytes = ctypes.c_size_t()
        _lib.check(self.lib.pfb_plan_workspace_size(self.handle, ctypes.byref(nbytes)))
        self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8,
                                     device=self.uvw.device)
        _lib.check(self.lib.pfb_plan_set_workspace(self.handle, _ptr(self.workspace),
                                                   self.workspace.numel(), _stream()))

    @classmethod
    def from_problem(cls, prob, device="cuda", options: Options | None = None, count_scratch=None):
        """Build from a ``synth.Problem`` (host numpy arrays)."""
        options = options or Options()
        real = torch.float64 if options.precision == "fp64" else torch.float32
        uvw = torch.as_tensor(prob.uvw, dtype=torch.float64, device=device)
        weight = torch.as_tensor(np.asarray(prob.weight), device=device).to(real)
        flag = None if prob.flag is None else torch.as_tensor(prob.flag, dtype=torch.uint8, device=device)
        return cls(uvw, prob.freq, weight, flag, prob.chan_band, prob.n_band, prob.nx, prob.ny,
                   prob.cellx, prob.celly, options, count_scratch)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.pfb_plan_destroy(h)
            self.handle = None

    # -- description ------------------------------------------------------------------
    def info(self) -> dict:
        inf = _lib.PfbPlanInfo()
        _lib.check(self.lib.pfb_plan_get_info(self.handle, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def fb_graph(self, dirty: torch.Tensor, x: torch.Tensor, sigma: float, gamma: float, lam: float,
                 cg_iters: int, n_steps: int = 1) -> "FbGraph":
        """Capture `n_steps` FB iterations (eqs. 4, 6, 8 + prox) into a HIP graph; x updated in place."""
        self._chk(dirty, (self.n_band, self.nx, self.ny), self.real)
        self._chk(x, (self.n_band, self.nx, self.ny), self.real)
        cap = torch.cuda.Stream(device=x.device)
        cap.wait_stream(torch.cuda.current_stream())
        g = ctypes.c_void_p()
        _lib.check(self.lib.pfb_fb_graph_create(self.handle, _ptr(dirty), _ptr(x), float(sigma), float(gamma),
                                                float(lam), int(cg_iters), int(n_steps),
                                                ctypes.c_void_p(cap.cuda_stream), ctypes.byref(g)))
        torch.cuda.current_stream().wait_stream(cap)
        return FbGraph(self, g, (dirty, x))

    # -- diagnostics -------------------------------------------------------------------
    def profile(self, on: bool):
        """Record HIP events around every kernel launched by this plan's operator calls."""
        _lib.check(self.lib.pfb_profile_enable(self.handle, int(bool(on))))

    def profile_report(self) -> dict:
        """{kernel name: (launches, total ms)} for the recorded launches (synchronises)."""
        buf = ctypes.create_string_buffer(1 << 16)
        _lib.check(self.lib.pfb_profile_report(self.handle, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, n, ms = line.split()
            out[name] = (int(n), float(ms))
        return out

    # -- tensors ----------------------------------------------------------------------
    def image(self, side_factor: int = 1) -> torch.Tensor:
        return torch.empty((self.n_band, side_factor * self.nx, side_factor * self.ny),
                           dtype=self.real, device=self.uvw.device)

    def vis(self) -> torch.Tensor:
        return torch.empty((self.n_row, self.n_chan), dtype=self.cplx, device=self.uvw.device)

    def _chk(self, t: torch.Tensor, shape, dtype):
        if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"expected contiguous device tensor {dtype} {tuple(shape)}, "
                             f"got {t.dtype} {tuple(t.shape)}")

    # -- operators (eqs. 1-8 of the paper, see include/pfb.h) ----------------------------
    def grid(self, vis: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Dirty image I^d = R^dagger Sigma^-1 V."""
        self._chk(vis, (self.n_row, self.n_chan), self.cplx)
        out = self.image() if out is None else out
        self._chk(out, (self.n_band, self.nx, self.ny), self.real)
        _lib.check(self.lib.pfb_grid(self.handle, _ptr(vis), _ptr(out), _lib.PFB_GRID_DIRTY, _stream()))
        return out

    def make_psf(self, out: torch.Tensor | None = None, want_image: bool = True):
        """PSF on the 2nx x 2ny grid; also makes the resident PSF spectrum."""
        if want_image:
            out = self.image(2) if out is None else out
            self._chk(out, (self.n_band, 2 * self.nx, 2 * self.ny), self.real)
        _lib.check(self.lib.pfb_grid(self.handle, None, _ptr(out if want_image else None),
                                     _lib.PFB_GRID_PSF, _stream()))
        return out

    def degrid(self, image: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Model visibilities V = R x."""
        self._chk(image, (self.n_band, self.nx, self.ny), self.real)
        out = self.vis() if out is None else out
        self._chk(out, (self.n_row, self.n_chan), self.cplx)
        _lib.check(self.lib.pfb_degrid(self.handle, _ptr(image), _ptr(out), _stream()))
        return out

    def degrid_add(self, image: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """V += R x (flagged entries of V untouched)."""
        self._chk(image, (self.n_band, self.nx, self.ny), self.real)
        self._chk(out, (self.n_row, self.n_chan), self.cplx)
        _lib.check(self.lib.pfb_degrid_add(self.handle, _ptr(image), _ptr(out), _stream()))
        return out

    def hessian(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """R^dagger Sigma^-1 R x (eq. 3)."""
        self._chk(x, (self.n_band, self.nx, self.ny), self.real)
        out = self.image() if out is None else out
        self._chk(out, (self.n_band, self.nx, self.ny), self.real)
        _lib.check(self.lib.pfb_hessian(self.handle, _ptr(x), _ptr(out), _stream()))
        return out

    def psf_conv(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """I^psf * x (eq. 4)."""
        self._chk(x, (self.n_band, self.nx, self.ny), self.real)
        out = self.image() if out is None else out
        self._chk(out, (self.n_band, self.nx, self.ny), self.real)
        _lib.check(self.lib.pfb_psf_conv(self.handle, _ptr(x), _ptr(out), _stream()))
        return out

    def precond_solve(self, g: torch.Tensor, sigma: float, iters: int,
                      out: torch.Tensor | None = None, resid: torch.Tensor | None = None, tol: float = 0.0):
        """(I^psf * + sigma Id) y = g by `iters` CG steps (eq. 8); tol > 0 stops once every
        band has ||r|| <= tol ||g|| (host-synchronising)."""
        self._chk(g, (self.n_band, self.nx, self.ny), self.real)
        out = self.image() if out is None else out
        self._chk(out, (self.n_band, self.nx, self.ny), self.real)
        if resid is not None:
            self._chk(resid, (self.n_band,), torch.float64)
        _lib.check(self.lib.pfb_precond_solve(self.handle, _ptr(g), _ptr(out), float(sigma), int(iters),
                                              float(tol), _ptr(resid), _stream()))
        return out

    def power_iteration(self, v0: torch.Tensor, iters: int, op: str = "psf") -> torch.Tensor:
        """Largest eigenvalue per band of I^psf * (op='psf') or the Hessian (op='hessian')."""
        self._chk(v0, (self.n_band, self.nx, self.ny), self.real)
        lam = torch.empty(self.n_band, dtype=torch.float64, device=v0.device)
        _lib.check(self.lib.pfb_power_iteration(self.handle, 0 if op == "psf" else 1, _ptr(v0), int(iters),
                                                _ptr(lam), _stream()))
        return lam

    def fb_step(self, dirty: torch.Tensor, x: torch.Tensor, sigma: float, gamma: float, lam: float,
                cg_iters: int) -> torch.Tensor:
        """One preconditioned forward-backward step (eqs. 4, 6, 8; l1 + positivity prox); x in place."""
        self._chk(dirty, (self.n_band, self.nx, self.ny), self.real)
        self._chk(x, (self.n_band, self.nx, self.ny), self.real)
        _lib.check(self.lib.pfb_fb_step(self.handle, _ptr(dirty), _ptr(x), float(sigma), float(gamma),
                                        float(lam), int(cg_iters), _stream()))
        return x

    # -- backward step: eq. (7) with the regulariser of eq. (9) -------------------------
    def prox_workspace(self, nbasis: int = 7) -> torch.Tensor:
        """Device workspace of the wavelet and prox calls (holds the dual variable)."""
        n = ctypes.c_size_t(0)
        _lib.check(self.lib.pfb_prox_workspace_size(self.handle, int(nbasis), ctypes.byref(n)))
        return torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=self.uvw.device)

    def coeffs(self, nbasis: int = 7) -> torch.Tensor:
        return torch.empty((nbasis, self.n_band, self.nx, self.ny), dtype=self.real, device=self.uvw.device)

    def wavelet_analysis(self, x: torch.Tensor, ws: torch.Tensor, nbasis: int = 7, levels: int = 3,
                         out: torch.Tensor | None = None) -> torch.Tensor:
        """Psi^dagger x: Dirac + db1 .. db(nbasis-1), periodic, ``levels`` levels."""
        self._chk(x, (self.n_band, self.nx, self.ny), self.real)
        out = self.coeffs(nbasis) if out is None else out
        self._chk(out, (nbasis, self.n_band, self.nx, self.ny), self.real)
        _lib.check(self.lib.pfb_wavelet_analysis(self.handle, _ptr(x), _ptr(out), _ptr(ws), ws.numel(),
                                                 int(nbasis), int(levels), _stream()))
        return out

    def wavelet_synthesis(self, c: torch.Tensor, ws: torch.Tensor, nbasis: int = 7, levels: int = 3,
                          out: torch.Tensor | None = None) -> torch.Tensor:
        """Psi c (the adjoint of wavelet_analysis)."""
        self._chk(c, (nbasis, self.n_band, self.nx, self.ny), self.real)
        out = self.image() if out is None else out
        self._chk(out, (self.n_band, self.nx, self.ny), self.real)
        _lib.check(self.lib.pfb_wavelet_synthesis(self.handle, _ptr(c), _ptr(out), _ptr(ws), ws.numel(),
                                                  int(nbasis), int(levels), _stream()))
        return out

    def prox(self, z: torch.Tensor, x: torch.Tensor, ws: torch.Tensor, lam: float, gamma: float, sigma: float,
             unorm: float, iters: int, nbasis: int = 7, levels: int = 3, warm: bool = False) -> torch.Tensor:
        """x = prox^U_{gamma r}(z), U = I^psf * + sigma Id, by ``iters`` primal-dual steps; x in place."""
        self._chk(z, (self.n_band, self.nx, self.ny), self.real)
        self._chk(x, (self.n_band, self.nx, self.ny), self.real)
        _lib.check(self.lib.pfb_prox_solve(self.handle, _ptr(z), _ptr(x), _ptr(ws), ws.numel(), int(nbasis),
                                           int(levels), float(lam), float(gamma), float(sigma), float(unorm),
                                           int(iters), 1 if warm else 0, _stream()))
        return x

    def fb_step_wavelet(self, dirty: torch.Tensor, x: torch.Tensor, ws: torch.Tensor, sigma: float, gamma: float,
                        lam: float, unorm: float, cg_iters: int, pd_iters: int, nbasis: int = 7, levels: int = 3,
                        warm: bool = False) -> torch.Tensor:
        """One forward-backward step of eqs. 6-7 with the l2,1 wavelet prior of eq. 9; x in place."""
        self._chk(dirty, (self.n_band, self.nx, self.ny), self.real)
        self._chk(x, (self.n_band, self.nx, self.ny), self.real)
        _lib.check(self.lib.pfb_fb_step_wavelet(self.handle, _ptr(dirty), _ptr(x), _ptr(ws), ws.numel(),
                                                int(nbasis), int(levels), float(sigma), float(gamma), float(lam),
                                                float(unorm), int(cg_iters), int(pd_iters), 1 if warm else 0,
                                                _stream()))
        return x

    def clean(self, dirty: torch.Tensor, x: torch.Tensor, ws: torch.Tensor, sigma: float, gamma: float, lam: float,
              unorm: float, cg_iters: int, pd_iters: int, n_major: int, nbasis: int = 7,
              levels: int = 3) -> torch.Tensor:
        """``n_major`` forward-backward steps with the exact gradient (one Hessian each); x in place."""
        self._chk(dirty, (self.n_band, self.nx, self.ny), self.real)
        self._chk(x, (self.n_band, self.nx, self.ny), self.real)
        _lib.check(self.lib.pfb_clean(self.handle, _ptr(dirty), _ptr(x), _ptr(ws), ws.numel(), int(nbasis),
                                      int(levels), float(sigma), float(gamma), float(lam), float(unorm),
                                      int(cg_iters), int(pd_iters), int(n_major), _stream()))
        return x


class FbGraph:
    """An instantiated HIP graph of FB iterations (keeps its plan and buffers alive)."""

    def __init__(self, plan: Plan, handle, keep):
        self.plan, self.handle, self._keep = plan, handle, keep

    def launch(self):
        _lib.check(self.plan.lib.pfb_graph_launch(self.handle, _stream()))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.plan.lib.pfb_graph_destroy(h)
            self.handle = None
