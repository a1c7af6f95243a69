"""ctypes loader for libmi.so (the HIP library).  There is no fallback implementation:
if the library is missing or fails to load, every call raises."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmi.so")

MI_OK, MI_ERR_ARG, MI_ERR_SHAPE, MI_ERR_UNSUPPORTED, MI_ERR_NOMEM, MI_ERR_DEVICE, MI_ERR_INSTANCE = range(7)
MI_INST_EMPTY, MI_INST_LOBE_CLIPPED, MI_INST_RESTORE_CLIPPED, MI_INST_TEST_FAILED, MI_INST_ABORTED = 1, 2, 4, 8, 16
MI_NATURAL, MI_UNIFORM = 0, 1
MI_LAYOUT_FULL, MI_LAYOUT_HALF = 0, 1
MI_PROF_CLEAN, MI_PROF_GRID, MI_PROF_IFFT, MI_PROF_GRID_FFT = 1, 2, 4, 8

# every entry point declared in include/mi.h
EXPORTS = ("mi_ctx_create", "mi_ctx_destroy", "mi_last_error", "mi_version", "mi_grid", "mi_ifft2",
           "mi_dirty_image", "mi_dirty_beam", "mi_hogbom_clean", "mi_degrid", "mi_gmm_levels", "mi_disk_offsets", "mi_phase_shift", "mi_profile_begin",
           "mi_profile_end", "mi_dirty_image_w", "mi_profile_begin_kinds", "mi_profile_end_kinds",
           "mi_predict_transpose", "mi_steer_clean", "mi_hogbom_clean_noalloc", "mi_set_tuning", "mi_get_tuning")


class MiBatch(ctypes.Structure):
    _fields_ = [("n_inst", c_int32), ("vis_offset", c_void_p), ("n_img", c_void_p), ("cell_rad", c_void_p),
                ("weight_mode", c_void_p), ("status", c_void_p)]


class MiCleanParams(ctypes.Structure):
    _fields_ = [("gain", c_float), ("niter", c_void_p), ("threshold", c_void_p), ("positive_only", c_int32),
                ("team_size", c_int32), ("threshold_dev", c_void_p),
                ("window", c_void_p)]


class MiTuning(ctypes.Structure):
    _fields_ = [("grid_chunk", c_int32), ("fft_elems", c_int32)]


class MiSteerParams(ctypes.Structure):
    _fields_ = [("gain", c_float), ("trim", c_float), ("ncycle", c_void_p), ("threshold", c_void_p),
                ("threshold_dev", c_void_p), ("positive_only", c_int32)]


class MiWprojParams(ctypes.Structure):
    _fields_ = [("w_max", c_void_p), ("phase_tol", c_double)]


class MiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mi error {code}: {msg}")
        self.code = code


_lib = None


def loaded() -> bool:
    return _lib is not None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1712_06913_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    L.mi_ctx_create.argtypes = [POINTER(c_void_p), c_int]
    L.mi_ctx_destroy.argtypes = [vp]
    L.mi_last_error.argtypes = [vp]
    L.mi_last_error.restype = c_char_p
    L.mi_version.restype = c_char_p
    L.mi_grid.argtypes = [vp, POINTER(MiBatch), vp, vp, vp, c_int, c_int, vp, vp, vp, vp]
    L.mi_ifft2.argtypes = [vp, vp, vp, vp, c_int32, vp]
    L.mi_dirty_image.argtypes = [vp, POINTER(MiBatch), vp, vp, vp, vp, vp, vp, vp]
    L.mi_dirty_beam.argtypes = [vp, POINTER(MiBatch), vp, vp, vp, vp]
    L.mi_hogbom_clean.argtypes = [vp, POINTER(MiBatch), vp, vp, POINTER(MiCleanParams), vp, vp, vp, vp, vp, vp,
                                  vp, vp]
    L.mi_hogbom_clean_noalloc.argtypes = L.mi_hogbom_clean.argtypes
    L.mi_set_tuning.argtypes = [vp, POINTER(MiTuning)]
    L.mi_get_tuning.argtypes = [vp, POINTER(MiTuning)]
    L.mi_dirty_image_w.argtypes = [vp, POINTER(MiBatch), vp, vp, vp, vp, POINTER(MiWprojParams), vp, vp, vp, vp]
    L.mi_degrid.argtypes = [vp, POINTER(MiBatch), vp, vp, vp, c_int, vp, vp]
    L.mi_predict_transpose.argtypes = [vp, POINTER(MiBatch), vp, vp, vp, vp, vp]
    L.mi_steer_clean.argtypes = [vp, POINTER(MiBatch), vp, vp, POINTER(MiSteerParams), vp, vp, vp, vp, vp, vp, vp,
                                 vp]
    L.mi_profile_begin_kinds.argtypes = [vp, ctypes.c_uint32]
    L.mi_profile_end_kinds.argtypes = [vp, vp, vp, c_int32, vp]
    for name in EXPORTS:
        if name not in ("mi_last_error", "mi_version"):
            getattr(L, name).restype = c_int
    _lib = L
    return L


def check(ctx, code: int):
    if code != MI_OK:
        msg = lib().mi_last_error(ctx).decode() if ctx else ""
        raise MiError(code, msg)
