"""The autotuner returns a configuration within the error budget (FP64 reference on the GPU)."""
import pytest

import synth
from gpu_helpers import say

pytestmark = pytest.mark.gpu


def test_autotune_small_problem():
    from paper_2101_08072_amd.tune import autotune
    prob = synth.tiny_problem(seed=41, nx=128, ny=128, n_row=3000, cell_arcsec=10.0, flag_frac=0.1)
    best, table = autotune(prob, err_budget=3e-6, supports=(6, 7, 8), tiles=(16, 32), reps=2)
    for r in table:
        say(r)
    assert best.support in (7, 8)
    ok = [r for r in table if r.get("ok")]
    assert all(r["support"] != 6 for r in ok)     # W = 6 misses a 3e-6 budget
