"""ctypes view of libepic.so (the C ABI in include/epic.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libepic.so")

EPIC_OK, EPIC_E_INVALID, EPIC_E_DEVICE, EPIC_E_NOMEM, EPIC_E_OFFGRID, EPIC_E_STATE, \
    EPIC_E_LAUNCH, EPIC_E_UNSUPPORTED = range(8)
STATUS_NAMES = {0: "EPIC_OK", 1: "EPIC_E_INVALID", 2: "EPIC_E_DEVICE", 3: "EPIC_E_NOMEM",
                4: "EPIC_E_OFFGRID", 5: "EPIC_E_STATE", 6: "EPIC_E_LAUNCH",
                7: "EPIC_E_UNSUPPORTED"}
EPIC_FP32, EPIC_SPLIT_FP16, EPIC_SPLIT_BF16 = 0, 1, 2
EPIC_FLAG_STAGED, EPIC_FLAG_TIMING, EPIC_FLAG_REMOVE_AUTOS = 1, 2, 4

# Every function declared in include/epic.h, with its ctypes signature.
EXPORTS = ("epic_init", "epic_set_stream", "epic_set_antennas", "epic_set_antennas_kernels",
           "epic_gridding_program",
           "epic_image_accumulate", "epic_image_accumulate_noalloc",
           "epic_image_backward", "epic_last_timing", "epic_timing_history", "epic_last_autos_timing",
           "epic_last_kernel_name",
           "epic_destroy", "epic_last_error",
           "epic_batch_create", "epic_batch_set_antennas", "epic_batch_accumulate",
           "epic_batch_capture", "epic_batch_replay", "epic_batch_tune", "epic_batch_plan",
           "epic_batch_launch_plan", "epic_batch_set_launch",
           "epic_batch_serial", "epic_batch_set_serial",
           "epic_batch_destroy", "epic_batch_last_error",
           "epic_postprocess", "epic_kernel_taper",
           "epic_frontend", "epic_pipeline_create", "epic_pipeline_push", "epic_pipeline_report",
           "epic_pipeline_destroy", "epic_pipeline_last_error")


class EpicConfig(ctypes.Structure):
    _fields_ = [("grid_n", ctypes.c_int32), ("n_chan", ctypes.c_int32),
                ("n_pol", ctypes.c_int32), ("n_ant", ctypes.c_int32),
                ("kernel_support", ctypes.c_int32), ("kernel_sigma_cells", ctypes.c_double),
                ("cell_wavelengths", ctypes.c_double), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class PipelineStats(ctypes.Structure):
    _fields_ = [("gulps", ctypes.c_int64), ("over_budget", ctypes.c_int64),
                ("gulp_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("mean_copy_ms", ctypes.c_double),
                ("mean_compute_ms", ctypes.c_double)]


class EpicError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the built library (it must exist: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1904_11422_amd.build`")
    L = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    L.epic_init.argtypes = [ctypes.POINTER(EpicConfig), ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.epic_init.restype = ctypes.c_int
    L.epic_set_stream.argtypes = [vp, vp]
    L.epic_set_stream.restype = ctypes.c_int
    L.epic_set_antennas.argtypes = [vp, dp, dp]
    L.epic_set_antennas.restype = ctypes.c_int
    L.epic_set_antennas_kernels.argtypes = [vp, dp, dp, vp]
    L.epic_set_antennas_kernels.restype = ctypes.c_int
    L.epic_gridding_program.argtypes = [ctypes.POINTER(EpicConfig), dp, dp,
                                        ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(i64),
                                        ctypes.POINTER(i32)]
    L.epic_gridding_program.restype = ctypes.c_int
    L.epic_image_accumulate.argtypes = [vp, vp, i64, vp, vp, i32]
    L.epic_image_accumulate.restype = ctypes.c_int
    L.epic_image_accumulate_noalloc.argtypes = [vp, vp, i64, vp, vp, i32]
    L.epic_image_accumulate_noalloc.restype = ctypes.c_int
    L.epic_image_backward.argtypes = [vp, vp, i64, vp, vp, vp]
    L.epic_image_backward.restype = ctypes.c_int
    L.epic_last_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
    L.epic_last_timing.restype = ctypes.c_int
    L.epic_timing_history.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]
    L.epic_timing_history.restype = ctypes.c_int
    L.epic_last_autos_timing.argtypes = L.epic_last_timing.argtypes
    L.epic_last_autos_timing.restype = ctypes.c_int
    L.epic_last_kernel_name.argtypes = [vp]
    L.epic_last_kernel_name.restype = ctypes.c_char_p
    L.epic_destroy.argtypes = [vp]
    L.epic_destroy.restype = None
    L.epic_last_error.argtypes = [vp]
    L.epic_last_error.restype = ctypes.c_char_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.epic_batch_create.argtypes = [ctypes.POINTER(EpicConfig), i32, ctypes.c_int, vp,
                                    ctypes.POINTER(vp)]
    L.epic_batch_create.restype = ctypes.c_int
    L.epic_batch_set_antennas.argtypes = [vp, i32, dp, dp]
    L.epic_batch_set_antennas.restype = ctypes.c_int
    for name in ("epic_batch_accumulate", "epic_batch_capture"):
        getattr(L, name).argtypes = [vp, pp, i64, pp, pp, i32]
        getattr(L, name).restype = ctypes.c_int
    L.epic_batch_replay.argtypes = [vp]
    L.epic_batch_replay.restype = ctypes.c_int
    L.epic_batch_tune.argtypes = [vp, pp, i64, pp, pp, ctypes.c_char_p, ctypes.POINTER(i32)]
    L.epic_batch_tune.restype = ctypes.c_int
    L.epic_batch_plan.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.epic_batch_plan.restype = ctypes.c_int
    L.epic_batch_launch_plan.argtypes = [vp, i32] + [ctypes.POINTER(i32)] * 5
    L.epic_batch_launch_plan.restype = ctypes.c_int
    L.epic_batch_set_launch.argtypes = [vp, i32, i32, i32, i32, i32]
    L.epic_batch_set_launch.restype = ctypes.c_int
    L.epic_batch_serial.argtypes = [vp]
    L.epic_batch_serial.restype = i32
    L.epic_batch_set_serial.argtypes = [vp, i32]
    L.epic_batch_set_serial.restype = ctypes.c_int
    L.epic_batch_destroy.argtypes = [vp]
    L.epic_batch_destroy.restype = None
    L.epic_batch_last_error.argtypes = [vp]
    L.epic_batch_last_error.restype = ctypes.c_char_p
    L.epic_postprocess.argtypes = [vp, vp, ctypes.c_double, vp]
    L.epic_postprocess.restype = ctypes.c_int
    L.epic_kernel_taper.argtypes = [vp, vp]
    L.epic_kernel_taper.restype = ctypes.c_int
    L.epic_frontend.argtypes = [vp, vp, i64, i32, i32, i32, vp]
    L.epic_frontend.restype = ctypes.c_int
    L.epic_pipeline_create.argtypes = [vp, i64, i32, i32, i32, ctypes.c_double, ctypes.POINTER(vp)]
    L.epic_pipeline_create.restype = ctypes.c_int
    L.epic_pipeline_push.argtypes = [vp, vp, vp, vp, i32]
    L.epic_pipeline_push.restype = ctypes.c_int
    L.epic_pipeline_report.argtypes = [vp, ctypes.POINTER(PipelineStats)]
    L.epic_pipeline_report.restype = ctypes.c_int
    L.epic_pipeline_destroy.argtypes = [vp]
    L.epic_pipeline_destroy.restype = None
    L.epic_pipeline_last_error.argtypes = [vp]
    L.epic_pipeline_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(L, ctx, status: int):
    if status != EPIC_OK:
        msg = L.epic_last_error(ctx)
        raise EpicError(status, msg.decode() if msg else "")


def check_pipeline(L, p, status: int):
    if status != EPIC_OK:
        msg = L.epic_pipeline_last_error(p)
        raise EpicError(status, msg.decode() if msg else "")


def check_batch(L, b, status: int):
    if status != EPIC_OK:
        msg = L.epic_batch_last_error(b)
        raise EpicError(status, msg.decode() if msg else "")
