"""ctypes declarations of the C ABI in ``include/pfb.h`` (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libpfb.so")

PFB_OK = 0
PFB_FP32, PFB_FP64 = 0, 1
PFB_GRID_DIRTY, PFB_GRID_PSF = 0, 1

STATUS_NAMES = {0: "PFB_OK", -1: "PFB_EINVAL", -2: "PFB_ENOMEM", -3: "PFB_EHIP",
                -4: "PFB_EUNSUPPORTED", -5: "PFB_ESTATE"}

# every symbol include/pfb.h declares
EXPORTS = ["pfb_plan_create", "pfb_plan_count_scratch_size", "pfb_plan_count", "pfb_plan_count_static",
           "pfb_plan_workspace_size", "pfb_plan_set_workspace",
           "pfb_plan_get_info", "pfb_plan_destroy", "pfb_grid", "pfb_degrid", "pfb_degrid_add", "pfb_hessian",
           "pfb_psf_conv", "pfb_precond_solve", "pfb_power_iteration", "pfb_fb_step",
           "pfb_fb_graph_create", "pfb_graph_launch", "pfb_graph_destroy",
           "pfb_profile_enable", "pfb_profile_report", "pfb_last_error", "pfb_version",
           "pfb_prox_workspace_size", "pfb_wavelet_analysis", "pfb_wavelet_synthesis", "pfb_prox_solve",
           "pfb_fb_step_wavelet", "pfb_clean"]


class PfbProblem(ctypes.Structure):
    _fields_ = [("n_row", ctypes.c_int64), ("n_chan", ctypes.c_int64), ("n_band", ctypes.c_int32),
                ("chan_band", ctypes.c_void_p), ("freq", ctypes.c_void_p), ("uvw", ctypes.c_void_p),
                ("weight", ctypes.c_void_p), ("flag", ctypes.c_void_p), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("cellx", ctypes.c_double), ("celly", ctypes.c_double),
                ("offx", ctypes.c_int32), ("offy", ctypes.c_int32)]


class PfbOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("support", ctypes.c_int32),
                ("oversample", ctypes.c_double), ("tile", ctypes.c_int32), ("flat", ctypes.c_int32),
                ("band_batch", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("epsilon", ctypes.c_double), ("reserved", ctypes.c_int32 * 6)]


class PfbPlanInfo(ctypes.Structure):
    _fields_ = [("grid_x", ctypes.c_int32), ("grid_y", ctypes.c_int32),
                ("psf_grid_x", ctypes.c_int32), ("psf_grid_y", ctypes.c_int32),
                ("support", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("n_wplanes_max", ctypes.c_int32), ("band_batch", ctypes.c_int32),
                ("n_vis_active", ctypes.c_int64), ("n_entries", ctypes.c_int64),
                ("n_psf_entries", ctypes.c_int64), ("s_min", ctypes.c_double),
                ("es_beta", ctypes.c_double), ("workspace_bytes", ctypes.c_int64),
                ("n_wplanes_total", ctypes.c_int64), ("occ_tiles", ctypes.c_int64),
                ("occ_tile_rows", ctypes.c_int64), ("need_tiles", ctypes.c_int64),
                ("need_tile_rows", ctypes.c_int64), ("s_max", ctypes.c_double)]


_lib = None


def load():
    """Load the HIP library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} missing "
                           "(run paper_2101_08072_amd.build.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, f64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    plan_pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "pfb_plan_create": [plan_pp, ctypes.POINTER(PfbProblem), ctypes.POINTER(PfbOptions), vp],
        "pfb_plan_count_scratch_size": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "pfb_plan_count": [vp, vp, sz, vp],
        "pfb_plan_count_static": [vp, vp],
        "pfb_plan_workspace_size": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "pfb_plan_set_workspace": [vp, vp, sz, vp],
        "pfb_plan_get_info": [vp, ctypes.POINTER(PfbPlanInfo)],
        "pfb_plan_destroy": [vp],
        "pfb_grid": [vp, vp, vp, i32, vp],
        "pfb_degrid": [vp, vp, vp, vp],
        "pfb_degrid_add": [vp, vp, vp, vp],
        "pfb_hessian": [vp, vp, vp, vp],
        "pfb_psf_conv": [vp, vp, vp, vp],
        "pfb_precond_solve": [vp, vp, vp, f64, i32, f64, vp, vp],
        "pfb_power_iteration": [vp, i32, vp, i32, vp, vp],
        "pfb_fb_step": [vp, vp, vp, f64, f64, f64, i32, vp],
        "pfb_fb_graph_create": [vp, vp, vp, f64, f64, f64, i32, i32, vp, ctypes.POINTER(ctypes.c_void_p)],
        "pfb_graph_launch": [vp, vp],
        "pfb_graph_destroy": [vp],
        "pfb_profile_enable": [vp, i32],
        "pfb_profile_report": [vp, ctypes.c_char_p, sz],
        "pfb_prox_workspace_size": [vp, i32, ctypes.POINTER(ctypes.c_size_t)],
        "pfb_wavelet_analysis": [vp, vp, vp, vp, sz, i32, i32, vp],
        "pfb_wavelet_synthesis": [vp, vp, vp, vp, sz, i32, i32, vp],
        "pfb_prox_solve": [vp, vp, vp, vp, sz, i32, i32, f64, f64, f64, f64, i32, i32, vp],
        "pfb_fb_step_wavelet": [vp, vp, vp, vp, sz, i32, i32, f64, f64, f64, f64, i32, i32, i32, vp],
        "pfb_clean": [vp, vp, vp, vp, sz, i32, i32, f64, f64, f64, f64, i32, i32, i32, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.pfb_last_error.restype = ctypes.c_char_p
    lib.pfb_last_error.argtypes = []
    lib.pfb_version.restype = ctypes.c_char_p
    lib.pfb_version.argtypes = []
    _lib = lib
    return lib


class PfbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def check(status: int):
    if status != PFB_OK:
        raise PfbError(status, load().pfb_last_error().decode())
