"""The C-ABI library loads and exports every symbol that include/pfb.h declares;
argument validation that needs no GPU returns the documented status codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfb.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:pfb_status|const char \*)\s*(pfb_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2101_08072_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_and_binding_agree():
    from paper_2101_08072_amd import _lib
    assert _declared() == sorted(_lib.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_version_and_last_error(lib):
    assert b"gfx950" in lib.pfb_version()
    assert isinstance(lib.pfb_last_error(), bytes)


def test_null_arguments_rejected_without_gpu(lib):
    from paper_2101_08072_amd import _lib
    assert lib.pfb_plan_create(None, None, None, None) == -1
    h = ctypes.c_void_p()
    assert lib.pfb_plan_create(ctypes.byref(h), None, None, None) == -1
    assert b"NULL" in lib.pfb_last_error()
    assert lib.pfb_plan_workspace_size(None, None) == -1
    assert lib.pfb_grid(None, None, None, 0, None) == -1
    assert lib.pfb_psf_conv(None, None, None, None) == -1
    n = ctypes.c_size_t(0)
    assert lib.pfb_prox_workspace_size(None, 7, ctypes.byref(n)) == -1
    assert lib.pfb_wavelet_analysis(None, None, None, None, 0, 7, 3, None) == -1
    assert lib.pfb_wavelet_synthesis(None, None, None, None, 0, 7, 3, None) == -1
    assert lib.pfb_prox_solve(None, None, None, None, 0, 7, 3, 1.0, 1.0, 1.0, 1.0, 1, 0, None) == -1
    assert lib.pfb_fb_step_wavelet(None, None, None, None, 0, 7, 3, 1.0, 1.0, 1.0, 1.0, 1, 1, 0, None) == -1
    assert lib.pfb_clean(None, None, None, None, 0, 7, 3, 1.0, 1.0, 1.0, 1.0, 1, 1, 1, None) == -1
    assert lib.pfb_plan_destroy(None) == 0


def test_shape_validation_without_gpu(lib):
    """Checks that run before any device access: odd or too small sides, bad bands,
    bad options."""
    import numpy as np
    from paper_2101_08072_amd import _lib
    freq = np.array([1e9, 1.1e9])
    cb = np.array([0, 0], np.int32)
    prob = _lib.PfbProblem()
    prob.n_row, prob.n_chan, prob.n_band = 10, 2, 1
    prob.chan_band, prob.freq = cb.ctypes.data, freq.ctypes.data
    prob.uvw, prob.weight = 16, 16            # never dereferenced: validation fails first
    prob.nx, prob.ny, prob.cellx, prob.celly = 25, 32, 1e-4, 1e-4
    h = ctypes.c_void_p()
    opt = _lib.PfbOptions()
    assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -1
    assert b"even" in lib.pfb_last_error()
    prob.nx = 14
    assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -1
    prob.nx = 32
    opt.support = 3
    assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -1
    opt.support = 0
    opt.oversample = 1.5
    assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -4
    opt.oversample = 0
    prob.nx, prob.ny = 256, 256
    opt.tile = 64                             # 7 w-planes of a 64 x 64 tile exceed the 160 KiB of LDS
    assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -1
    assert b"LDS" in lib.pfb_last_error()
    opt.tile = 0
    # FP64 mode: the operator's rows (2n points) must fit LDS in FP64, so 4096 is its largest side
    prob.nx, prob.ny, prob.cellx, prob.celly = 8192, 8192, 1e-7, 1e-7
    opt.precision = 1
    assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -4
    assert b"FFT rows" in lib.pfb_last_error()
    opt.precision = 0
    prob.nx, prob.ny, prob.cellx, prob.celly = 256, 256, 1e-4, 1e-4
    cb[1] = 3
    assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -1
    assert b"chan_band" in lib.pfb_last_error()


def test_count_and_solve_arguments_without_gpu(lib):
    """The counting pass and its scratch-size query need a plan; the solve's tol is
    validated like its other scalars."""
    n = ctypes.c_size_t(0)
    assert lib.pfb_plan_count_scratch_size(None, ctypes.byref(n)) == -1
    assert lib.pfb_plan_count(None, None, 0, None) == -1
    assert lib.pfb_precond_solve(None, None, None, 1.0, 1, 0.0, None, None) == -1


def test_epsilon_option_validation_without_gpu(lib):
    """epsilon picks the support; a negative or non-finite value, or one below what the
    precision reaches, is rejected before any device access."""
    import numpy as np
    from paper_2101_08072_amd import _lib
    freq = np.array([1e9, 1.1e9])
    cb = np.array([0, 0], np.int32)
    prob = _lib.PfbProblem()
    prob.n_row, prob.n_chan, prob.n_band = 10, 2, 1
    prob.chan_band, prob.freq = cb.ctypes.data, freq.ctypes.data
    prob.uvw, prob.weight = 16, 16            # never dereferenced: validation fails first
    prob.nx, prob.ny, prob.cellx, prob.celly = 64, 64, 1e-4, 1e-4
    h = ctypes.c_void_p()
    opt = _lib.PfbOptions()
    for bad in (-1e-3, float("nan"), float("inf")):
        opt.epsilon = bad
        assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -1
        assert b"epsilon" in lib.pfb_last_error()
    opt.epsilon = 1e-9                        # beyond the FP32 path (W <= 8)
    assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -1
    assert b"FP32" in lib.pfb_last_error()
    opt.precision, opt.epsilon = 1, 1e-16     # beyond the FP64 path (W <= 16)
    assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -1
    assert b"FP64" in lib.pfb_last_error()


def test_facet_offsets_need_the_fp32_w_stacked_path(lib):
    """A facet offset is refused in FP64 mode and in flat mode before any device access."""
    import numpy as np
    from paper_2101_08072_amd import _lib
    freq = np.array([1e9, 1.1e9])
    cb = np.array([0, 0], np.int32)
    prob = _lib.PfbProblem()
    prob.n_row, prob.n_chan, prob.n_band = 10, 2, 1
    prob.chan_band, prob.freq = cb.ctypes.data, freq.ctypes.data
    prob.uvw, prob.weight = 16, 16            # never dereferenced: validation fails first
    prob.nx, prob.ny, prob.cellx, prob.celly = 64, 64, 1e-4, 1e-4
    prob.offx, prob.offy = 32, -32
    h = ctypes.c_void_p()
    opt = _lib.PfbOptions()
    opt.precision = 1
    assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -4
    opt.precision, opt.flat = 0, 1
    assert lib.pfb_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), None) == -4
    assert b"facet" in lib.pfb_last_error()
