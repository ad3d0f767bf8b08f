"""Writes tiny16_regression.json from the FP64 oracle only (no HIP path)."""
import json
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
    V = oracle.degrid(p, x)
    out = {"problem": "synth.tiny_problem(seed=4242, nx=16, ny=16, n_row=60, cell_arcsec=60, flag_frac=0.1)",
           "x": x.ravel().tolist(), "vis_re": vis.real.ravel().tolist(), "vis_im": vis.imag.ravel().tolist(),
           "degrid_re": V.real.ravel().tolist(), "degrid_im": V.imag.ravel().tolist(),
           "dirty": oracle.grid(p, vis).ravel().tolist(), "psf": oracle.psf(p).ravel().tolist(),
           "hessian": oracle.hessian(p, x).ravel().tolist()}
    with open(os.path.join(HERE, "tiny16_regression.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    make()
