"""ctypes declarations of the C ABI in include/vca.h (argument marshalling only).

Loads ``libvca.so`` from this package directory.  A missing library is an
error: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvca.so")

VCA_OK = 0
VCA_ERR_INVALID_ARG = 1
VCA_ERR_UNSUPPORTED = 2
VCA_ERR_OOM = 3
VCA_ERR_DEVICE = 4
VCA_ERR_STATE = 5

VCA_F_KEEP_COEFFS = 0x1
VCA_F_VALIDATE = 0x2
VCA_F_TIMING = 0x4
VCA_F_DOWNSAMPLE = 0x8

# Every symbol include/vca.h declares.
EXPORTS = (
    "vca_block_counts", "vca_open", "vca_analyze_frames", "vca_analyze_yuv_file", "vca_read_yuv",
    "vca_features", "vca_block_coeffs",
    "vca_block_stats", "vca_block_maps", "vca_get_timing", "vca_tune", "vca_tuned_launch", "vca_reset",
    "vca_frames_submitted", "vca_close", "vca_status_str", "vca_last_error",
    "vca_open_batch", "vca_analyze_batch", "vca_batch_features", "vca_batch_features_many",
    "vca_tune_batch",
    "vca_batch_tuned_launch", "vca_batch_class_times", "vca_batch_arrangement", "vca_batch_set_arrangement", "vca_batch_set_class_shape", "vca_batch_timing", "vca_reset_batch", "vca_batch_submitted",
    "vca_batch_last_error", "vca_close_batch",
    "vca_grad_workspace", "vca_energy_forward", "vca_energy_backward",
    "vca_analyze_noalloc",
)


class VcaConfig(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("bit_depth", ctypes.c_int32), ("chroma_format", ctypes.c_int32),
        ("block_size", ctypes.c_int32), ("lowpass_k", ctypes.c_int32),
        ("device", ctypes.c_int32), ("flags", ctypes.c_uint32), ("max_batch", ctypes.c_int32),
        ("feature_capacity", ctypes.c_int32),
    ]


class VcaFrames(ctypes.Structure):
    _fields_ = [
        ("y", ctypes.c_void_p), ("u", ctypes.c_void_p), ("v", ctypes.c_void_p),
        ("pitch_y", ctypes.c_int64), ("pitch_uv", ctypes.c_int64),
        ("fstride_y", ctypes.c_int64), ("fstride_uv", ctypes.c_int64),
        ("on_device", ctypes.c_int32),
    ]


class VcaFrameFeatures(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("E_Y", "h", "L_Y", "E_U", "E_V", "L_U", "L_V")]


class VcaTiming(ctypes.Structure):
    _fields_ = [("forward_ms", ctypes.c_double), ("reduce_ms", ctypes.c_double),
                ("forward_launches", ctypes.c_int64), ("reduce_launches", ctypes.c_int64),
                ("frames", ctypes.c_int64)]


class VcaGradConfig(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("block_size", ctypes.c_int32), ("lowpass_k", ctypes.c_int32),
        ("bit_depth", ctypes.c_int32), ("n_seq", ctypes.c_int32), ("seq_len", ctypes.c_int32),
        ("device", ctypes.c_int32), ("pitch", ctypes.c_int64), ("fstride", ctypes.c_int64),
    ]


class VcaError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_str(status)}" + (f" ({detail})" if detail else ""))


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_2304_12384_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        St = ctypes.c_int
        sig = {
            "vca_block_counts": (St, [ctypes.POINTER(VcaConfig), P]),
            "vca_open": (St, [ctypes.POINTER(VcaConfig), P, ctypes.POINTER(P)]),
            "vca_analyze_frames": (St, [P, ctypes.POINTER(VcaFrames), ctypes.c_int32]),
            "vca_analyze_yuv_file": (St, [P, ctypes.c_char_p, ctypes.c_int64, ctypes.c_int32]),
            "vca_read_yuv": (St, [ctypes.c_char_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int64, ctypes.c_int32, P, P, P]),
            "vca_features": (St, [P, ctypes.c_int64, ctypes.c_int32, P]),
            "vca_block_coeffs": (St, [P, ctypes.c_int64, P, ctypes.c_size_t]),
            "vca_block_stats": (St, [P, ctypes.c_int64, P, P, ctypes.c_size_t]),
            "vca_block_maps": (St, [P, ctypes.c_int64, ctypes.c_int32, P, P, P]),
            "vca_get_timing": (St, [P, ctypes.POINTER(VcaTiming), ctypes.c_int32]),
            "vca_tune": (St, [P, ctypes.POINTER(VcaFrames), ctypes.c_int32, ctypes.c_int32]),
            "vca_tuned_launch": (St, [P, P, P, P]),
            "vca_reset": (St, [P]),
            "vca_open_batch": (St, [ctypes.POINTER(VcaConfig), ctypes.c_int32, P, ctypes.POINTER(P)]),
            "vca_analyze_batch": (St, [P, ctypes.POINTER(VcaFrames), P]),
            "vca_batch_features": (St, [P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, P]),
            "vca_batch_features_many": (St, [P, ctypes.c_int32, P, P, P, P]),
            "vca_tune_batch": (St, [P, ctypes.POINTER(VcaFrames), P, ctypes.c_int32]),
            "vca_batch_tuned_launch": (St, [P, P, P, P]),
            "vca_batch_class_times": (St, [P, P, P, P, P, P]),
            "vca_batch_arrangement": (St, [P, P, P, P]),
            "vca_batch_set_arrangement": (St, [P, ctypes.c_int32]),
            "vca_batch_set_class_shape": (St, [P] + [ctypes.c_int32] * 5),
            "vca_batch_timing": (St, [P, P, P, P, ctypes.c_int32]),
            "vca_reset_batch": (St, [P, ctypes.c_int32]),
            "vca_batch_submitted": (ctypes.c_int64, [P, ctypes.c_int32]),
            "vca_batch_last_error": (ctypes.c_char_p, [P]),
            "vca_close_batch": (None, [P]),
            "vca_frames_submitted": (ctypes.c_int64, [P]),
            "vca_close": (None, [P]),
            "vca_grad_workspace": (ctypes.c_int64, [ctypes.POINTER(VcaGradConfig)]),
            "vca_energy_forward": (St, [ctypes.POINTER(VcaGradConfig), P, P, P, P, P]),
            "vca_energy_backward": (St, [ctypes.POINTER(VcaGradConfig), P, P, P, P, P]),
            "vca_analyze_noalloc": (St, [ctypes.POINTER(VcaConfig), ctypes.POINTER(VcaFrames),
                                         ctypes.c_int32, P, P]),
            "vca_status_str": (ctypes.c_char_p, [ctypes.c_int]),
            "vca_last_error": (ctypes.c_char_p, [P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(status: int) -> str:
    return lib().vca_status_str(status).decode()


def check(status: int, what: str, ctx=None, batch=None) -> None:
    if status != VCA_OK:
        detail = ""
        if ctx:
            detail = lib().vca_last_error(ctx).decode()
        elif batch:
            detail = lib().vca_batch_last_error(batch).decode()
        raise VcaError(status, what, detail)
