"""The oracle reproduces its own committed regression fixture (tests/golden)."""
import json
import os

import numpy as np

import oracle
import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_regression_fixture():
    with open(os.path.join(HERE, "tiny16_regression.json")) as f:
        g = json.load(f)
    p = synth.tiny_problem(seed=4242, nx=16, ny=16, n_row=60, cell_arcsec=60.0, flag_frac=0.1)
    x = np.array(g["x"]).reshape(1, 16, 16)
    vis = (np.array(g["vis_re"]) + 1j * np.array(g["vis_im"])).reshape(60, 2)
    V = oracle.degrid(p, x)
    assert np.allclose(V.real.ravel(), g["degrid_re"], rtol=0, atol=1e-12)
    assert np.allclose(V.imag.ravel(), g["degrid_im"], rtol=0, atol=1e-12)
    assert np.allclose(oracle.grid(p, vis).ravel(), g["dirty"], rtol=0, atol=1e-11)
    assert np.allclose(oracle.psf(p).ravel(), g["psf"], rtol=0, atol=1e-11)
    assert np.allclose(oracle.hessian(p, x).ravel(), g["hessian"], rtol=0, atol=1e-10)
