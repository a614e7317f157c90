"""ctypes declarations of the C ABI in include/fcc.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfcc.so")

FCC_OK = 0
NOALLOC_SCRATCH_BYTES = 64 << 20      # FCC_NOALLOC_SCRATCH_BYTES
STATUS_NAMES = {0: "FCC_OK", -1: "FCC_ERR_INVALID_ARG", -2: "FCC_ERR_UNSUPPORTED",
                -3: "FCC_ERR_BASIS_AMBIGUOUS", -4: "FCC_ERR_HIP", -5: "FCC_ERR_INTERNAL"}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2, "fp8": 3, "fp8_e4m3": 3}
METHODS = {"fcc": 0, "gcc": 1}
OPERANDS = {"fp16": 0, "storage": 1}

# every symbol include/fcc.h declares
EXPORTS = ("fcc_plan_create", "fcc_plan_destroy", "fcc_plan_query", "fcc_plan_upload",
           "fcc_num_frames", "fcc_workspace_bytes", "fcc_spectra", "fcc_tdoa", "fcc_tdoa_noalloc",
           "fcc_tdoa_from_spectra", "fcc_correlation", "fcc_coefficients", "fcc_tdoa_parabolic",
           "fcc_basis_export", "fcc_mlp_num_params", "fcc_mlp_workspace_bytes", "fcc_mlp_forward",
           "fcc_mlp_backward", "fcc_mlp_adam", "fcc_learned_workspace_bytes", "fcc_tdoa_learned",
           "fcc_smooth_workspace_bytes", "fcc_tdoa_smoothed", "fcc_doa_table", "fcc_doa",
           "fcc_batch_create", "fcc_batch_destroy", "fcc_batch_query", "fcc_batch_layout", "fcc_batch_upload",
           "fcc_batch_tdoa", "fcc_batch_tune", "fcc_batch_tuning",
           "fcc_status_string", "fcc_last_error")


class FccError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


class FccConfig(ctypes.Structure):
    _fields_ = [("num_mics", ctypes.c_int32), ("mic_xyz", ctypes.POINTER(ctypes.c_double)),
                ("fs", ctypes.c_double), ("c", ctypes.c_double),
                ("frame_size", ctypes.c_int32), ("hop", ctypes.c_int32),
                ("tau_max", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("interp", ctypes.c_int32), ("alpha", ctypes.c_float),
                ("precision", ctypes.c_int32), ("method", ctypes.c_int32),
                ("operands", ctypes.c_int32)]


class FccBatchInfo(ctypes.Structure):
    _fields_ = [("num_arrays", ctypes.c_int32), ("num_classes", ctypes.c_int32),
                ("image_bytes", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
                ("audio_floats", ctypes.c_int64), ("tdoa_count", ctypes.c_int64)]


class FccPlanInfo(ctypes.Structure):
    _fields_ = [("num_mics", ctypes.c_int32), ("num_pairs", ctypes.c_int32),
                ("frame_size", ctypes.c_int32), ("hop", ctypes.c_int32),
                ("num_bins", ctypes.c_int32), ("tau_max", ctypes.c_int32),
                ("num_lags", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("rank_sym", ctypes.c_int32), ("rank_anti", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("method", ctypes.c_int32),
                ("basis_bytes", ctypes.c_size_t), ("spectrum_bytes_per_frame", ctypes.c_size_t),
                ("spectrum_elem_bytes", ctypes.c_int32),
                ("interp", ctypes.c_int32),
                ("alpha", ctypes.c_float),
                ("operands", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Loads libfcc.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2204_13622_amd.build`")
    # PyTorch ships its own HIP runtime with the same soname; loading torch
    # first lets libfcc.so bind to that copy, so one process holds one runtime
    # (and torch's device memory and streams are valid in the library).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32p = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "fcc_plan_create": [ctypes.POINTER(FccConfig), ctypes.POINTER(vp)],
        "fcc_plan_query": [vp, ctypes.POINTER(FccPlanInfo)],
        "fcc_plan_upload": [vp, vp, vp],
        "fcc_num_frames": [vp, i64, ctypes.POINTER(i64)],
        "fcc_workspace_bytes": [vp, i64, ctypes.POINTER(ctypes.c_size_t)],
        "fcc_spectra": [vp, vp, vp, i64, i64, vp, vp],
        "fcc_tdoa": [vp, vp, vp, i64, i64, vp, vp, vp],
        "fcc_tdoa_noalloc": [vp, vp, vp, i64, i64, vp, vp],
        "fcc_tdoa_from_spectra": [vp, vp, vp, i64, vp, vp],
        "fcc_correlation": [vp, vp, vp, i64, vp, vp],
        "fcc_coefficients": [vp, vp, vp, i64, vp, vp],
        "fcc_tdoa_parabolic": [vp, vp, vp, i64, vp, vp],
        "fcc_basis_export": [vp, dp, i32p, dp, dp, dp],
        "fcc_mlp_workspace_bytes": [ctypes.c_int32, ctypes.c_int32, i64, ctypes.POINTER(ctypes.c_size_t)],
        "fcc_mlp_forward": [vp, ctypes.c_int32, ctypes.c_int32, vp, i64, vp, vp, vp],
        "fcc_mlp_backward": [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, i64, vp, vp, vp, vp, vp],
        "fcc_batch_create": [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(i64), ctypes.POINTER(vp)],
        "fcc_batch_query": [vp, ctypes.POINTER(FccBatchInfo)],
        "fcc_batch_layout": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "fcc_batch_upload": [vp, vp, vp],
        "fcc_batch_tdoa": [vp, vp, vp, vp, vp, ctypes.c_int32, vp],
        "fcc_batch_tune": [vp, vp, vp, vp, vp, vp],
        "fcc_batch_tuning": [vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32],
        "fcc_doa_table": [vp, dp, ctypes.c_int32, vp],
        "fcc_doa": [vp, vp, i64, vp, ctypes.c_int32, vp, vp, vp],
        "fcc_smooth_workspace_bytes": [vp, i64, ctypes.POINTER(ctypes.c_size_t)],
        "fcc_tdoa_smoothed": [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp],
        "fcc_learned_workspace_bytes": [vp, ctypes.c_int32, i64, ctypes.POINTER(ctypes.c_size_t)],
        "fcc_tdoa_learned": [vp, vp, vp, i64, vp, ctypes.c_int32, ctypes.c_float, vp, vp, vp, vp],
        "fcc_mlp_adam": [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                         ctypes.c_float, ctypes.c_int32, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.fcc_mlp_num_params.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.fcc_mlp_num_params.restype = ctypes.c_size_t
    lib.fcc_batch_destroy.argtypes = [vp]
    lib.fcc_batch_destroy.restype = None
    lib.fcc_plan_destroy.argtypes = [vp]
    lib.fcc_plan_destroy.restype = None
    lib.fcc_status_string.argtypes = [ctypes.c_int]
    lib.fcc_status_string.restype = ctypes.c_char_p
    lib.fcc_last_error.argtypes = []
    lib.fcc_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != FCC_OK:
        msg = _lib.fcc_last_error().decode() if _lib is not None else ""
        raise FccError(status, msg)
