"""MI355X (gfx950) RIFT2 hot path: thin torch binding over librift2.so.

Every stage runs in the library's HIP kernels; this module only marshals
torch device tensors, streams and parameter records into the C ABI declared
in include/rift2.h.  There is no CPU fallback: without the built library or
a GPU every call raises.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import PCParams, DetectParams, DescParams, MatchParams, PREC_FP32, PREC_BF16, Rift2Error  # noqa: F401

__all__ = [
    "defaults", "init", "filter_mim", "detect", "describe", "match", "Rift2Error",
    "PCParams", "DetectParams", "DescParams", "MatchParams", "PREC_FP32", "PREC_BF16",
]


def defaults():
    """(PCParams, DetectParams, DescParams, MatchParams) with the library defaults."""
    lib = _lib.load()
    pc, det, desc, mp = PCParams(), DetectParams(), DescParams(), MatchParams()
    lib.rift2_default_params(ctypes.byref(pc), ctypes.byref(det), ctypes.byref(desc), ctypes.byref(mp))
    return pc, det, desc, mp


_inited = set()


def init(device: int = 0) -> None:
    lib = _lib.load()
    if device not in _inited:
        _lib.check(lib.rift2_init(device), "rift2_init")
        _inited.add(device)


def _torch():
    import torch

    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _workspace(nbytes: int, device, ws=None):
    torch = _torch()
    if ws is not None:
        if ws.numel() * ws.element_size() < nbytes:
            raise ValueError("workspace too small")
        return ws
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def filter_mim(img, pc: PCParams | None = None, want_min: bool = False, want_amp: bool = False,
               workspace=None, stream=None):
    """MIM, max moment (and optionally min moment and A_o) of one H x W device image."""
    torch = _torch()
    lib = _lib.load()
    if pc is None:
        pc = defaults()[0]
    if img.dim() != 2 or not img.is_cuda:
        raise ValueError("img must be a 2-D device tensor")
    dtype = {torch.uint8: _lib.U8, torch.int16: _lib.U16, torch.uint16: _lib.U16, torch.float32: _lib.F32}.get(img.dtype)
    if dtype is None:
        raise ValueError(f"unsupported image dtype {img.dtype}")
    init(img.device.index or 0)
    h, w = img.shape
    dev = img.device
    mim = torch.empty((h, w), dtype=torch.uint8, device=dev)
    mmax = torch.empty((h, w), dtype=torch.float32, device=dev)
    mmin = torch.empty((h, w), dtype=torch.float32, device=dev) if want_min else None
    amp = torch.empty((pc.n_orient, h, w), dtype=torch.float32, device=dev) if want_amp else None
    nbytes = lib.rift2_filter_workspace_size(h, w, ctypes.byref(pc))
    if nbytes == 0:
        raise Rift2Error(_lib.ERR_UNSUPPORTED, "rift2_filter_workspace_size")
    ws = _workspace(nbytes, dev, workspace)
    st = lib.rift2_filter_mim(_ptr(img), dtype, h, w, img.stride(0), ctypes.byref(pc), _ptr(mim), _ptr(mmax),
                              _ptr(mmin), _ptr(amp), _ptr(ws), nbytes, _stream(stream))
    _lib.check(st, "rift2_filter_mim")
    out = {"mim": mim, "M": mmax}
    if want_min:
        out["m"] = mmin
    if want_amp:
        out["amp"] = amp
    return out


def detect(moment, det: DetectParams | None = None, workspace=None, stream=None):
    """(kpts int32 [K, 3] = x, y, score bits; n int32 [1]) on the device, strongest first."""
    torch = _torch()
    lib = _lib.load()
    if det is None:
        det = defaults()[1]
    init(moment.device.index or 0)
    h, w = moment.shape
    dev = moment.device
    kpts = torch.empty((det.max_keypoints, 3), dtype=torch.int32, device=dev)
    n = torch.zeros((1,), dtype=torch.int32, device=dev)
    nbytes = lib.rift2_detect_workspace_size(h, w, ctypes.byref(det))
    ws = _workspace(nbytes, dev, workspace)
    st = lib.rift2_detect(_ptr(moment), h, w, ctypes.byref(det), _ptr(kpts), _ptr(n), _ptr(ws), nbytes, _stream(stream))
    _lib.check(st, "rift2_detect")
    return kpts, n


def describe(mim, kpts, n_kpts, dp: DescParams | None = None, workspace=None, stream=None):
    """(desc int16 [2K, D] holding uint16 counts, inv_norm f32 [2K], desc_kp int32 [2K], n_desc int32 [1])."""
    torch = _torch()
    lib = _lib.load()
    if dp is None:
        dp = defaults()[2]
    init(mim.device.index or 0)
    h, w = mim.shape
    dev = mim.device
    cap = kpts.shape[0]
    d = dp.grid * dp.grid * dp.n_orient
    desc = torch.empty((2 * cap, d), dtype=torch.int16, device=dev)
    inv = torch.empty((2 * cap,), dtype=torch.float32, device=dev)
    dkp = torch.empty((2 * cap,), dtype=torch.int32, device=dev)
    nd = torch.zeros((1,), dtype=torch.int32, device=dev)
    nbytes = lib.rift2_describe_workspace_size(cap)
    ws = _workspace(nbytes, dev, workspace)
    st = lib.rift2_describe(_ptr(mim), h, w, _ptr(kpts), _ptr(n_kpts), cap, ctypes.byref(dp), _ptr(desc), _ptr(inv),
                            _ptr(dkp), 2 * cap, _ptr(nd), _ptr(ws), nbytes, _stream(stream))
    _lib.check(st, "rift2_describe")
    return desc, inv, dkp, nd


def match(desc_a, inv_a, kp_a, n_a, desc_b, inv_b, kp_b, n_b, mp: MatchParams | None = None,
          workspace=None, stream=None):
    """(matches int32 [cap_a, 3] = kp_a, kp_b, d2 bits; n int32 [1]) sorted by kp_a."""
    torch = _torch()
    lib = _lib.load()
    if mp is None:
        mp = defaults()[3]
    init(desc_a.device.index or 0)
    cap_a, d = desc_a.shape
    cap_b = desc_b.shape[0]
    dev = desc_a.device
    out = torch.empty((cap_a, 3), dtype=torch.int32, device=dev)
    n = torch.zeros((1,), dtype=torch.int32, device=dev)
    nbytes = lib.rift2_match_workspace_size(cap_a, cap_b, d, ctypes.byref(mp))
    if nbytes == 0:
        raise Rift2Error(_lib.ERR_INVALID_ARG, "rift2_match_workspace_size")
    ws = _workspace(nbytes, dev, workspace)
    st = lib.rift2_match(_ptr(desc_a), _ptr(inv_a), _ptr(kp_a), _ptr(n_a), cap_a, _ptr(desc_b), _ptr(inv_b),
                         _ptr(kp_b), _ptr(n_b), cap_b, d, ctypes.byref(mp), _ptr(out), _ptr(n), _ptr(ws), nbytes,
                         _stream(stream))
    _lib.check(st, "rift2_match")
    return out, n
