"""The oracle reproduces its own committed regression fixture (tests/golden)."""
import os

import numpy as np

import oracle
import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_regression_fixture():
    g = np.load(os.path.join(HERE, "tiny16_regression.npz"))
    p = synth.tiny_problem(seed=4242, nx=16, ny=16, n_row=60, cell_arcsec=60.0, flag_frac=0.1)
    assert np.allclose(oracle.degrid(p, g["x"]), g["degrid"], rtol=0, atol=1e-12)
    assert np.allclose(oracle.grid(p, g["vis"]), g["dirty"], rtol=0, atol=1e-11)
    assert np.allclose(oracle.psf(p), g["psf"], rtol=0, atol=1e-11)
    assert np.allclose(oracle.hessian(p, g["x"]), g["hessian"], rtol=0, atol=1e-10)
