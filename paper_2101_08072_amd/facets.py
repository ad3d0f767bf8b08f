"""Faceted imaging: one image as a grid of facets, each with its own plan.

The image is cut into fx x fy facets of equal size; facet (a, b) is an image of
nx/fx x ny/fy pixels whose centre pixel sits at a whole-pixel offset from the
phase centre (pfb_problem offx, offy), so it has its own w-range of n - 1 and
so its own (smaller) number of w-planes, and its own, smaller FFTs.  All facet
plans borrow the same visibilities, weights and flags.  The operators of the
whole image follow from R being a sum over pixels (Section 2, eq. 1):

    R x        = sum over facets f of R_f x_f                 (pfb_degrid_add per facet)
    R^+ S^-1 V = the facets' dirty images R_f^+ S^-1 V, side by side
    H x        = R^+ S^-1 (sum_f R_f x_f), facet by facet     (eq. 3)

Copies between the whole image and the facets are memory plumbing; every
operator step runs in the library's kernels.
"""
from __future__ import annotations

import torch

from .plan import Options, Plan


class FacetedPlan:
    """fx x fy facets of an nx x ny image (nx / fx and ny / fy powers of two >= 16)."""

    def __init__(self, uvw, freq, weight, flag, chan_band, n_band, nx, ny, cellx, celly, fx, fy,
                 options: Options | None = None):
        if nx % fx or ny % fy:
            raise ValueError("the image sides must be multiples of the facet counts")
        self.nx, self.ny, self.fx, self.fy, self.n_band = int(nx), int(ny), int(fx), int(fy), int(n_band)
        self.sx, self.sy = self.nx // self.fx, self.ny // self.fy
        self.facets = []
        for a in range(self.fx):
            for b in range(self.fy):
                # centre pixel of facet (a, b) in whole-image pixels, relative to (nx/2, ny/2)
                off = (a * self.sx + self.sx // 2 - self.nx // 2, b * self.sy + self.sy // 2 - self.ny // 2)
                plan = Plan(uvw, freq, weight, flag, chan_band, n_band, self.sx, self.sy, cellx, celly,
                            options, offset=off)
                self.facets.append(((a, b), plan))
        self.real, self.cplx = self.facets[0][1].real, self.facets[0][1].cplx
        self.n_row, self.n_chan = self.facets[0][1].n_row, self.facets[0][1].n_chan

    @classmethod
    def from_problem(cls, prob, fx, fy, device="cuda", options: Options | None = None):
        import numpy as np
        options = options or Options()
        real = torch.float64 if options.precision == "fp64" else torch.float32
        uvw = torch.as_tensor(prob.uvw, dtype=torch.float64, device=device)
        weight = torch.as_tensor(np.asarray(prob.weight), device=device).to(real)
        flag = None if prob.flag is None else torch.as_tensor(prob.flag, dtype=torch.uint8, device=device)
        return cls(uvw, prob.freq, weight, flag, prob.chan_band, prob.n_band, prob.nx, prob.ny, prob.cellx,
                   prob.celly, fx, fy, options)

    def _region(self, a, b):
        return (slice(None), slice(a * self.sx, (a + 1) * self.sx), slice(b * self.sy, (b + 1) * self.sy))

    def info(self) -> list[dict]:
        return [dict(facet=ab, **p.info()) for ab, p in self.facets]

    def image(self) -> torch.Tensor:
        return torch.empty((self.n_band, self.nx, self.ny), dtype=self.real, device=self.facets[0][1].uvw.device)

    def grid(self, vis: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Dirty image R^+ S^-1 V of the whole image, facet by facet."""
        out = self.image() if out is None else out
        for (a, b), p in self.facets:
            out[self._region(a, b)] = p.grid(vis)
        return out

    def degrid(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """V = sum over facets of R_f x_f (flagged entries 0)."""
        p0 = self.facets[0][1]
        out = p0.vis() if out is None else out
        out.zero_()
        for (a, b), p in self.facets:
            p.degrid_add(x[self._region(a, b)].contiguous(), out)
        return out

    def hessian(self, x: torch.Tensor, out: torch.Tensor | None = None, vis_tmp: torch.Tensor | None = None):
        """H x = R^+ S^-1 R x (eq. 3) of the whole image: the model visibilities of all
        facets, then every facet's dirty image of them."""
        v = self.degrid(x, out=vis_tmp)
        return self.grid(v, out=out)
