"""ctypes view of libmhfd (include/mhfd.h): structures, signatures, loading.

Argument marshalling only.  The shared library must have been built in-tree
(``paper_2108_12050_amd/libmhfd.so``); if it is missing or cannot be loaded
every call raises ``MHFDLibraryError`` -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhfd.so")

MHFD_MAX_SCALES = 32
MHFD_MAX_RADIUS = 64
MHFD_F32, MHFD_U8 = 0, 1
MHFD_BRIGHT, MHFD_DARK = 0, 1
MHFD_CRITERION_LOG, MHFD_CRITERION_DOG = 0, 1
MHFD_BLUR_DIRECT, MHFD_BLUR_FFT = 0, 1
MHFD_MAX_FFT_SIZE = 4096
MHFD_MAX_FFT_RADIUS = 2048
MHFD_FLAG_BLOB_OVERFLOW = 1
MHFD_FLAG_CAND_OVERFLOW = 2
MHFD_FLAG_INVALID_TILE = 4
MHFD_MAX_BATCH = 4096

STATUS = {0: "MHFD_OK", 1: "MHFD_ERR_INVALID_ARG", 2: "MHFD_ERR_UNSUPPORTED",
          3: "MHFD_ERR_WORKSPACE", 4: "MHFD_ERR_HIP", 5: "MHFD_ERR_OOM"}

# Every symbol include/mhfd.h declares.
EXPORTS = ("mhfd_create_plan", "mhfd_destroy_plan", "mhfd_plan_scales",
           "mhfd_detect_workspace_size", "mhfd_detect", "mhfd_log_stack_workspace_size",
           "mhfd_log_stack", "mhfd_log_stack_static", "mhfd_detect_stack", "mhfd_stretch_levels",
           "mhfd_activity_bytes", "mhfd_log_stack_sparse", "mhfd_detect_stack_sparse",
           "mhfd_batch_workspace_size", "mhfd_detect_batched", "mhfd_focus_workspace_size",
           "mhfd_focus_score", "mhfd_focus_score_backward", "mhfd_status_string",
           "mhfd_last_error")


class MHFDLibraryError(RuntimeError):
    """libmhfd.so is missing or failed to load."""


class MHFDError(RuntimeError):
    """A libmhfd call returned a non-OK status."""

    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")


class Config(C.Structure):
    _fields_ = [("n_scales", C.c_int32), ("sigma_min", C.c_float), ("sigma_max", C.c_float),
                ("sigmas", C.POINTER(C.c_float)), ("truncate", C.c_float),
                ("threshold", C.c_float), ("overlap", C.c_float), ("polarity", C.c_int32),
                ("in_dtype", C.c_int32), ("max_h", C.c_int32), ("max_w", C.c_int32),
                ("max_candidates", C.c_int64), ("stretch", C.c_int32), ("criterion", C.c_int32),
                ("sigma_cap", C.c_float), ("blur", C.c_int32)]


class Blob(C.Structure):
    _fields_ = [("y", C.c_int32), ("x", C.c_int32), ("k", C.c_int32), ("sigma", C.c_float),
                ("response", C.c_float)]


class Tile(C.Structure):
    _fields_ = [("img", C.c_void_p), ("h", C.c_int32), ("w", C.c_int32), ("pitch", C.c_int64),
                ("blobs", C.c_void_p), ("result", C.c_void_p), ("capacity", C.c_int32),
                ("seg_rows", C.c_int32)]


class BatchOpts(C.Structure):
    _fields_ = [("log_groups_per_cu", C.c_int32), ("nms_groups_per_cu", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("n_blobs", C.c_int64), ("n_candidates", C.c_int64), ("flags", C.c_int32),
                ("reserved", C.c_int32), ("density", C.c_double)]


# mhfd_result as int64 words: n_blobs, n_candidates, flags (low 32 bits),
# density (the bits of a double)
RESULT_WORDS = 4
MHFD_FOCUS_BAD_SIGMA = 1

assert C.sizeof(Blob) == 20 and C.sizeof(Result) == 8 * RESULT_WORDS and C.sizeof(Tile) == 48

_lib = None


def load(path: str | None = None):
    """Load libmhfd.so and declare its signatures (cached)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise MHFDLibraryError(
            f"{p} not found: build it with `python -m paper_2108_12050_amd.build`")
    try:
        L = C.CDLL(p)
    except OSError as e:  # pragma: no cover - depends on the machine
        raise MHFDLibraryError(f"cannot load {p}: {e}") from e
    vp, i32, i64, f32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
    L.mhfd_create_plan.argtypes = [C.POINTER(Config), C.POINTER(vp)]
    L.mhfd_create_plan.restype = C.c_int
    L.mhfd_destroy_plan.argtypes = [vp]
    L.mhfd_destroy_plan.restype = C.c_int
    L.mhfd_plan_scales.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_int32)]
    L.mhfd_plan_scales.restype = i32
    L.mhfd_detect_workspace_size.argtypes = [vp, i32, i32]
    L.mhfd_detect_workspace_size.restype = sz
    L.mhfd_detect.argtypes = [vp, vp, i32, i32, i64, vp, i32, vp, vp, vp, sz, vp]
    L.mhfd_detect.restype = C.c_int
    L.mhfd_log_stack_workspace_size.argtypes = [vp, i32, i32]
    L.mhfd_log_stack_workspace_size.restype = sz
    L.mhfd_log_stack.argtypes = [vp, vp, i32, i32, i64, vp, vp, sz, vp]
    L.mhfd_log_stack.restype = C.c_int
    L.mhfd_log_stack_static.argtypes = [vp, vp, i32, i32, i64, vp, vp]
    L.mhfd_log_stack_static.restype = C.c_int
    L.mhfd_activity_bytes.argtypes = [vp, i32, i32]
    L.mhfd_activity_bytes.restype = sz
    L.mhfd_log_stack_sparse.argtypes = [vp, vp, i32, i32, i64, vp, vp, vp, sz, vp]
    L.mhfd_log_stack_sparse.restype = C.c_int
    L.mhfd_detect_stack_sparse.argtypes = [vp, vp, vp, i32, i32, vp, i32, vp, vp, sz, vp]
    L.mhfd_detect_stack_sparse.restype = C.c_int
    L.mhfd_detect_stack.argtypes = [vp, vp, i32, i32, vp, i32, vp, vp, sz, vp]
    L.mhfd_detect_stack.restype = C.c_int
    L.mhfd_stretch_levels.argtypes = [vp, i32, i32, i64, vp, vp, vp]
    L.mhfd_stretch_levels.restype = C.c_int
    L.mhfd_batch_workspace_size.argtypes = [vp, i32, i64]
    L.mhfd_batch_workspace_size.restype = sz
    L.mhfd_detect_batched.argtypes = [vp, i32, vp, i64, C.POINTER(BatchOpts), vp, sz, vp]
    L.mhfd_detect_batched.restype = C.c_int
    L.mhfd_focus_workspace_size.argtypes = [vp, i32, i32, i32]
    L.mhfd_focus_workspace_size.restype = sz
    L.mhfd_focus_score.argtypes = [vp, vp, i32, i32, i32, vp, f32, f32, vp, vp, vp, sz, vp]
    L.mhfd_focus_score.restype = C.c_int
    L.mhfd_focus_score_backward.argtypes = [vp, vp, i32, i32, i32, vp, f32, f32, vp, vp, vp,
                                            vp, vp, sz, vp]
    L.mhfd_focus_score_backward.restype = C.c_int
    L.mhfd_status_string.argtypes = [C.c_int]
    L.mhfd_status_string.restype = C.c_char_p
    L.mhfd_last_error.argtypes = []
    L.mhfd_last_error.restype = C.c_char_p
    if path is None:
        _lib = L
    return L


def check(status: int, where: str) -> None:
    if status != 0:
        detail = load().mhfd_last_error().decode(errors="replace")
        raise MHFDError(status, where, detail)
