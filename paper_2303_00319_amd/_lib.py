"""ctypes declarations of librift2.so (mirrors include/rift2.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librift2.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_DEVICE, ERR_NOT_INITIALIZED = 0, 1, 2, 3, 4, 5
U8, U16, F32 = 0, 1, 2
PREC_FP32, PREC_BF16, PREC_FP8 = 0, 1, 2
DESC_DOMINANT, DESC_PLAIN, DESC_RING, DESC_TURNED = 0, 1, 2, 3


class PCParams(ctypes.Structure):
    _fields_ = [
        ("n_scales", ctypes.c_int32),
        ("n_orient", ctypes.c_int32),
        ("min_wavelength", ctypes.c_float),
        ("mult", ctypes.c_float),
        ("sigma_onf", ctypes.c_float),
        ("dtheta_on_sigma", ctypes.c_float),
        ("lp_cutoff", ctypes.c_float),
        ("lp_order", ctypes.c_int32),
        ("k", ctypes.c_float),
        ("cutoff", ctypes.c_float),
        ("g", ctypes.c_float),
        ("eps", ctypes.c_float),
    ]


class DetectParams(ctypes.Structure):
    _fields_ = [("fast_threshold", ctypes.c_float), ("max_keypoints", ctypes.c_int32), ("patch_size", ctypes.c_int32)]


class DescParams(ctypes.Structure):
    _fields_ = [
        ("patch_size", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("n_orient", ctypes.c_int32),
        ("dominant_num", ctypes.c_int32),
        ("dominant_den", ctypes.c_int32),
        ("mode", ctypes.c_int32),
    ]


class MatchParams(ctypes.Structure):
    _fields_ = [("ratio_sq", ctypes.c_float), ("precision", ctypes.c_int32), ("ring", ctypes.c_int32),
                ("mutual", ctypes.c_int32)]


class RansacParams(ctypes.Structure):
    _fields_ = [("threshold", ctypes.c_double), ("refine", ctypes.c_int32)]


MAX_FILTER_BATCH = 8


class FilterJob(ctypes.Structure):
    _fields_ = [
        ("img", ctypes.c_void_p),
        ("mim", ctypes.c_void_p),
        ("max_moment", ctypes.c_void_p),
        ("min_moment", ctypes.c_void_p),
        ("amp_sums", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64),
        ("img_a", ctypes.c_void_p),
        ("img_b", ctypes.c_void_p),
        ("dtype", ctypes.c_int32),
        ("H", ctypes.c_int32),
        ("W", ctypes.c_int32),
        ("max_keypoints", ctypes.c_int32),
        ("out", ctypes.c_void_p),
        ("n_out", ctypes.c_void_p),
        ("ready", ctypes.c_void_p),
    ]


class Completion(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("gpu_ms", ctypes.c_float),
        ("admit_ms", ctypes.c_double),
        ("done_ms", ctypes.c_double),
        ("batch", ctypes.c_int32),
    ]


EXPORTS = [
    "rift2_default_params", "rift2_status_string", "rift2_init", "rift2_size_supported",
    "rift2_filter_workspace_size", "rift2_detect_workspace_size", "rift2_describe_workspace_size",
    "rift2_match_workspace_size", "rift2_filter_mim", "rift2_detect", "rift2_describe", "rift2_match",
    "rift2_profile_enable", "rift2_profile_read", "rift2_engine_request_bytes", "rift2_engine_create",
    "rift2_engine_submit", "rift2_engine_poll", "rift2_engine_pending", "rift2_engine_destroy",
    "rift2_ransac_workspace_size", "rift2_ransac", "rift2_consensus", "rift2_detect_union_workspace_size",
    "rift2_detect_union", "rift2_debug_response", "rift2_debug_noise", "rift2_desc_normalize",
    "rift2_detect_noalloc", "rift2_filter_mim_batch", "rift2_engine_set_batch", "rift2_debug_mfma_rate",
]
STAGES = ["row_dft", "pass_a", "noise_pre", "noise_sel", "pass_b", "detect", "describe", "match_prep",
          "match_gemm", "match_merge", "pass_b_reduce", "ransac"]

_LIB = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librift2.so; raises if it has not been built (there is no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"librift2.so not found at {path}: build it with python -m paper_2303_00319_amd.build")
    try:
        # torch ships its own HIP runtime; load it first so that the library
        # binds to the same runtime instance instead of a second copy
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64
    lib.rift2_default_params.argtypes = [P(PCParams), P(DetectParams), P(DescParams), P(MatchParams)]
    lib.rift2_default_params.restype = None
    lib.rift2_status_string.argtypes = [ctypes.c_int]
    lib.rift2_status_string.restype = ctypes.c_char_p
    lib.rift2_init.argtypes = [ctypes.c_int]
    lib.rift2_init.restype = ctypes.c_int
    lib.rift2_size_supported.argtypes = [ctypes.c_int]
    lib.rift2_size_supported.restype = ctypes.c_int
    lib.rift2_filter_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, P(PCParams)]
    lib.rift2_filter_workspace_size.restype = sz
    lib.rift2_detect_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, P(DetectParams)]
    lib.rift2_detect_workspace_size.restype = sz
    lib.rift2_describe_workspace_size.argtypes = [i32]
    lib.rift2_describe_workspace_size.restype = sz
    lib.rift2_match_workspace_size.argtypes = [i32, i32, i32, P(MatchParams)]
    lib.rift2_match_workspace_size.restype = sz
    lib.rift2_filter_mim.argtypes = [vp, i32, i32, i32, i64, P(PCParams), vp, vp, vp, vp, vp, sz, vp]
    lib.rift2_filter_mim.restype = ctypes.c_int
    lib.rift2_filter_mim_batch.argtypes = [i32, P(FilterJob), i32, i32, i32, i64, P(PCParams), vp]
    lib.rift2_filter_mim_batch.restype = ctypes.c_int
    lib.rift2_engine_set_batch.argtypes = [vp, i32]
    lib.rift2_engine_set_batch.restype = ctypes.c_int
    lib.rift2_detect.argtypes = [vp, i32, i32, P(DetectParams), vp, vp, vp, sz, vp]
    lib.rift2_detect.restype = ctypes.c_int
    lib.rift2_detect_noalloc.argtypes = [vp, i32, i32, P(DetectParams), vp, vp, vp]
    lib.rift2_detect_noalloc.restype = ctypes.c_int
    lib.rift2_describe.argtypes = [vp, i32, i32, vp, vp, i32, P(DescParams), vp, vp, vp, i32, vp, vp, sz, vp]
    lib.rift2_describe.restype = ctypes.c_int
    lib.rift2_match.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp, i32, i32, P(MatchParams), vp, vp, vp, sz, vp]
    lib.rift2_match.restype = ctypes.c_int
    lib.rift2_detect_union_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, P(DetectParams)]
    lib.rift2_detect_union_workspace_size.restype = sz
    lib.rift2_detect_union.argtypes = [vp, vp, i32, i32, P(DetectParams), vp, vp, vp, sz, vp]
    lib.rift2_detect_union.restype = ctypes.c_int
    lib.rift2_ransac_workspace_size.argtypes = [i32, i32]
    lib.rift2_ransac_workspace_size.restype = sz
    lib.rift2_ransac.argtypes = [vp, vp, i32, vp, i32, vp, i32, vp, i32, P(RansacParams), vp, vp, vp, vp, sz, vp]
    lib.rift2_ransac.restype = ctypes.c_int
    lib.rift2_consensus.argtypes = [vp, vp, vp, i32, vp, i32, vp, i32, ctypes.c_double, vp, vp, vp, sz, vp]
    lib.rift2_consensus.restype = ctypes.c_int
    lib.rift2_debug_response.argtypes = [vp, i32, i32, i32, i64, P(PCParams), i32, i32, vp, vp, sz, vp]
    lib.rift2_debug_response.restype = ctypes.c_int
    lib.rift2_debug_noise.argtypes = [vp, sz, i32, i32, P(PCParams), vp, vp, vp, vp]
    lib.rift2_debug_noise.restype = ctypes.c_int
    lib.rift2_debug_mfma_rate.argtypes = [i32, i32, i32, i32, vp, P(ctypes.c_float), vp]
    lib.rift2_debug_mfma_rate.restype = ctypes.c_int
    lib.rift2_desc_normalize.argtypes = [vp, vp, vp, i32, i32, vp, vp]
    lib.rift2_desc_normalize.restype = ctypes.c_int
    lib.rift2_profile_enable.argtypes = [ctypes.c_int]
    lib.rift2_profile_enable.restype = ctypes.c_int
    lib.rift2_profile_read.argtypes = [P(ctypes.c_double), P(ctypes.c_int64), ctypes.c_int]
    lib.rift2_profile_read.restype = ctypes.c_int
    lib.rift2_engine_request_bytes.argtypes = [i32, i32, i32, P(PCParams), P(DetectParams), P(DescParams),
                                               P(MatchParams)]
    lib.rift2_engine_request_bytes.restype = sz
    lib.rift2_engine_create.argtypes = [ctypes.c_int, vp, sz, i32, P(PCParams), P(DetectParams), P(DescParams),
                                        P(MatchParams), P(vp)]
    lib.rift2_engine_create.restype = ctypes.c_int
    lib.rift2_engine_submit.argtypes = [vp, P(Request)]
    lib.rift2_engine_submit.restype = ctypes.c_int
    lib.rift2_engine_poll.argtypes = [vp, P(Completion), i32]
    lib.rift2_engine_poll.restype = i32
    lib.rift2_engine_pending.argtypes = [vp]
    lib.rift2_engine_pending.restype = i32
    lib.rift2_engine_destroy.argtypes = [vp]
    lib.rift2_engine_destroy.restype = ctypes.c_int
    _LIB = lib
    return lib


class Rift2Error(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = _LIB
        msg = lib.rift2_status_string(status).decode() if lib is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def check(status: int, where: str) -> None:
    if status != OK:
        raise Rift2Error(status, where)
