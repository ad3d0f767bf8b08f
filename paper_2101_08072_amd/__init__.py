"""MI355X (gfx950) library for the hot path of preconditioned forward-backward
radio-interferometric imaging (Bester et al., ADASS XXX): the w-corrected NUFFT
measurement operator, its Hessian, the PSF convolution and the CG-preconditioned
forward-backward step.  The compute lives in ``_build/libpfb.so`` (C ABI in
``include/pfb.h``); this package is its ctypes binding.
"""
from ._lib import EXPORTS, PfbError, load  # noqa: F401
from .plan import Options, Plan  # noqa: F401

__all__ = ["Plan", "Options", "PfbError", "load", "EXPORTS"]
