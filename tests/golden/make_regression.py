"""Writes tiny16_regression.npz from the FP64 oracle only (no HIP path)."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def make():
    p = synth.tiny_problem(seed=4242, nx=16, ny=16, n_row=60, cell_arcsec=60.0, flag_frac=0.1)
    rng = np.random.default_rng(4243)
    x = rng.normal(size=(1, 16, 16))
    vis = rng.normal(size=(60, 2)) + 1j * rng.normal(size=(60, 2))
    out = dict(x=x, vis=vis, degrid=oracle.degrid(p, x), dirty=oracle.grid(p, vis),
               psf=oracle.psf(p), hessian=oracle.hessian(p, x))
    np.savez(os.path.join(HERE, "tiny16_regression.npz"), **out)


if __name__ == "__main__":
    make()
