"""MI355X (gfx950) RIFT2 hot path: thin torch binding over librift2.so.

Every stage runs in the library's HIP kernels; this module only marshals
torch device tensors, streams and parameter records into the C ABI declared
in include/rift2.h.  There is no CPU fallback: without the built library or
a GPU every call raises.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (PCParams, DetectParams, DescParams, MatchParams, RansacParams, PREC_FP32, PREC_BF16,  # noqa: F401
                   PREC_FP8, DESC_DOMINANT, DESC_PLAIN, DESC_RING, DESC_TURNED, Rift2Error, STAGES)

__all__ = [
    "defaults", "init", "filter_mim", "detect", "describe", "match", "Rift2Error", "PairPipeline", "PipelinedPairs",
    "profile_enable", "profile_read", "PCParams", "DetectParams", "DescParams", "MatchParams", "Engine",
    "PREC_FP32", "PREC_BF16", "PREC_FP8", "STAGES", "RansacParams", "ransac", "consensus", "ransac_workspace_bytes",
    "SIMILARITY_BYTES", "CONSENSUS_BYTES", "similarity_fields", "consensus_fields", "DESC_DOMINANT", "DESC_PLAIN",
    "DESC_RING", "DESC_TURNED", "rows_per_keypoint", "detect_union", "debug_response", "debug_noise",
    "desc_normalize", "filter_workspace_bytes", "filter_mim_batch_into", "mfma_rate",
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
    """Device address of a tensor that the library reads or writes as one dense block."""
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_contiguous():
        raise ValueError("the library takes dense (contiguous) tensors")
    return ctypes.c_void_p(t.data_ptr())


def _img_ptr(img):
    """Device address of an H x W image whose rows may be pitched (unit column stride)."""
    if img.dim() != 2 or img.stride(1) != 1 or img.stride(0) < img.shape[1]:
        raise ValueError("an image is H x W with unit column stride and a row pitch of at least W")
    return ctypes.c_void_p(img.data_ptr())


def _nbytes(t):
    return t.numel() * t.element_size()


def _image_dtype(img):
    torch = _torch()
    code = {torch.uint8: _lib.U8, torch.int16: _lib.U16, torch.uint16: _lib.U16, torch.float32: _lib.F32}.get(img.dtype)
    if code is None:
        raise ValueError(f"unsupported image dtype {img.dtype}")
    return code


# ----------------------------------------------------------------- workspace sizes

def filter_workspace_bytes(h, w, pc):
    n = _lib.load().rift2_filter_workspace_size(h, w, ctypes.byref(pc))
    if n == 0:
        raise Rift2Error(_lib.ERR_UNSUPPORTED, "rift2_filter_workspace_size")
    return n


def detect_workspace_bytes(h, w, det):
    return _lib.load().rift2_detect_workspace_size(h, w, ctypes.byref(det))


def detect_union_workspace_bytes(h, w, det):
    return _lib.load().rift2_detect_union_workspace_size(h, w, ctypes.byref(det))


def describe_workspace_bytes(cap):
    return _lib.load().rift2_describe_workspace_size(cap)


def match_workspace_bytes(cap_a, cap_b, d, mp):
    n = _lib.load().rift2_match_workspace_size(cap_a, cap_b, d, ctypes.byref(mp))
    if n == 0:
        raise Rift2Error(_lib.ERR_INVALID_ARG, "rift2_match_workspace_size")
    return n


def ransac_workspace_bytes(match_cap, n_hyp):
    n = _lib.load().rift2_ransac_workspace_size(match_cap, n_hyp)
    if n == 0:
        raise Rift2Error(_lib.ERR_UNSUPPORTED, "rift2_ransac_workspace_size")
    return n


# ----------------------------------------------------------------- calls on caller buffers

def filter_mim_into(img, pc, mim, mmax, mmin, amp, ws, stream=None):
    lib = _lib.load()
    h, w = img.shape
    st = lib.rift2_filter_mim(_img_ptr(img), _image_dtype(img), h, w, img.stride(0), ctypes.byref(pc), _ptr(mim),
                              _ptr(mmax), _ptr(mmin), _ptr(amp), _ptr(ws), _nbytes(ws), _stream(stream))
    _lib.check(st, "rift2_filter_mim")


def filter_mim_batch_into(imgs, pc, outs, stream=None):
    """rift2_filter_mim_batch: the filter bank of same-size, same-type images in shared launches.
    outs[i] = (mim, mmax, mmin or None, amp or None, workspace) of image i."""
    lib = _lib.load()
    n = len(imgs)
    if n != len(outs) or not 1 <= n <= _lib.MAX_FILTER_BATCH:
        raise ValueError(f"1..{_lib.MAX_FILTER_BATCH} images with one output set each")
    h, w = imgs[0].shape
    for im in imgs:
        if im.shape != (h, w) or im.dtype != imgs[0].dtype or im.stride(0) != imgs[0].stride(0):
            raise ValueError("a batch holds images of one size, type and pitch")
    jobs = (_lib.FilterJob * n)()
    for i, (im, (mim, mmax, mmin, amp, ws)) in enumerate(zip(imgs, outs)):
        jobs[i] = _lib.FilterJob(_img_ptr(im), _ptr(mim), _ptr(mmax), _ptr(mmin), _ptr(amp), _ptr(ws), _nbytes(ws))
    st = lib.rift2_filter_mim_batch(n, jobs, _image_dtype(imgs[0]), h, w, imgs[0].stride(0), ctypes.byref(pc),
                                    _stream(stream))
    _lib.check(st, "rift2_filter_mim_batch")


def detect_into(moment, det, kpts, n, ws, stream=None):
    lib = _lib.load()
    h, w = moment.shape
    st = lib.rift2_detect(_ptr(moment), h, w, ctypes.byref(det), _ptr(kpts), _ptr(n), _ptr(ws), _nbytes(ws),
                          _stream(stream))
    _lib.check(st, "rift2_detect")


def detect_noalloc_into(moment, det, kpts, n, stream=None):
    """rift2_detect_noalloc: detection on the library's own scratch (no workspace argument)."""
    lib = _lib.load()
    h, w = moment.shape
    st = lib.rift2_detect_noalloc(_ptr(moment), h, w, ctypes.byref(det), _ptr(kpts), _ptr(n), _stream(stream))
    _lib.check(st, "rift2_detect_noalloc")


def detect_union_into(max_moment, min_moment, det, kpts, n, ws, stream=None):
    lib = _lib.load()
    h, w = max_moment.shape
    st = lib.rift2_detect_union(_ptr(max_moment), _ptr(min_moment), h, w, ctypes.byref(det), _ptr(kpts), _ptr(n),
                                _ptr(ws), _nbytes(ws), _stream(stream))
    _lib.check(st, "rift2_detect_union")


def describe_into(mim, kpts, n_kpts, dp, desc, inv, dkp, nd, ws, stream=None):
    lib = _lib.load()
    h, w = mim.shape
    cap = kpts.shape[0]
    st = lib.rift2_describe(_ptr(mim), h, w, _ptr(kpts), _ptr(n_kpts), cap, ctypes.byref(dp), _ptr(desc), _ptr(inv),
                            _ptr(dkp), desc.shape[0], _ptr(nd), _ptr(ws), _nbytes(ws), _stream(stream))
    _lib.check(st, "rift2_describe")


def match_into(desc_a, inv_a, kp_a, n_a, desc_b, inv_b, kp_b, n_b, mp, out, n_out, ws, stream=None):
    lib = _lib.load()
    cap_a, d = desc_a.shape
    st = lib.rift2_match(_ptr(desc_a), _ptr(inv_a), _ptr(kp_a), _ptr(n_a), cap_a, _ptr(desc_b), _ptr(inv_b),
                         _ptr(kp_b), _ptr(n_b), desc_b.shape[0], d, ctypes.byref(mp), _ptr(out), _ptr(n_out),
                         _ptr(ws), _nbytes(ws), _stream(stream))
    _lib.check(st, "rift2_match")


def ransac_into(matches, n_matches, kpts_a, kpts_b, words, rp, counts, mask, result, ws, stream=None):
    """RANSAC on device buffers: matches int32 [cap, 3] (kp_a, kp_b, d2 bits), keypoints int32 [cap_k, 3],
    words uint32/int32 [n_hyp, 2]; counts int32 [n_hyp] or None, mask uint8 [cap], result uint8 [48]."""
    lib = _lib.load()
    st = lib.rift2_ransac(_ptr(matches), _ptr(n_matches), matches.shape[0], _ptr(kpts_a), kpts_a.shape[0],
                          _ptr(kpts_b), kpts_b.shape[0], _ptr(words), words.shape[0], ctypes.byref(rp),
                          _ptr(counts), _ptr(mask), _ptr(result), _ptr(ws), _nbytes(ws), _stream(stream))
    _lib.check(st, "rift2_ransac")


def consensus_into(model, matches, n_matches, kpts_a, kpts_b, threshold, mask, result, ws, stream=None):
    """Consensus of a device model (float64 [4] = a, b, tx, ty); result uint8 [16]."""
    lib = _lib.load()
    st = lib.rift2_consensus(_ptr(model), _ptr(matches), _ptr(n_matches), matches.shape[0], _ptr(kpts_a),
                             kpts_a.shape[0], _ptr(kpts_b), kpts_b.shape[0], float(threshold), _ptr(mask),
                             _ptr(result), _ptr(ws), _nbytes(ws), _stream(stream))
    _lib.check(st, "rift2_consensus")


# ----------------------------------------------------------------- allocating convenience calls

def _on_stream(fn):
    """An allocating call given a `stream` runs with that stream current, so its outputs are allocated,
    and their fills enqueued, on the stream its kernels run on."""
    import functools
    import inspect

    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapped(*args, **kw):
        stream = sig.bind(*args, **kw).arguments.get("stream")
        if stream is None:
            return fn(*args, **kw)
        with _torch().cuda.stream(stream):
            return fn(*args, **kw)

    return wrapped


@_on_stream
def filter_mim(img, pc: PCParams | None = None, want_min: bool = False, want_amp: bool = False,
               workspace=None, stream=None):
    """MIM, max moment (and optionally min moment and A_o) of one H x W device image."""
    torch = _torch()
    if pc is None:
        pc = defaults()[0]
    if img.dim() != 2 or not img.is_cuda:
        raise ValueError("img must be a 2-D device tensor")
    init(img.device.index or 0)
    h, w = img.shape
    dev = img.device
    mim = torch.empty((h, w), dtype=torch.uint8, device=dev)
    mmax = torch.empty((h, w), dtype=torch.float32, device=dev)
    mmin = torch.empty((h, w), dtype=torch.float32, device=dev) if want_min else None
    amp = torch.empty((pc.n_orient, h, w), dtype=torch.float32, device=dev) if want_amp else None
    ws = workspace if workspace is not None else torch.empty(filter_workspace_bytes(h, w, pc), dtype=torch.uint8,
                                                             device=dev)
    filter_mim_into(img, pc, mim, mmax, mmin, amp, ws, stream)
    out = {"mim": mim, "M": mmax}
    if want_min:
        out["m"] = mmin
    if want_amp:
        out["amp"] = amp
    return out


@_on_stream
def detect(moment, det: DetectParams | None = None, workspace=None, stream=None):
    """(kpts int32 [K, 3] = x, y, score bits; n int32 [1]) on the device, strongest first."""
    torch = _torch()
    if det is None:
        det = defaults()[1]
    init(moment.device.index or 0)
    h, w = moment.shape
    dev = moment.device
    kpts = torch.empty((det.max_keypoints, 3), dtype=torch.int32, device=dev)
    n = torch.zeros((1,), dtype=torch.int32, device=dev)
    ws = workspace if workspace is not None else torch.empty(detect_workspace_bytes(h, w, det), dtype=torch.uint8,
                                                             device=dev)
    detect_into(moment, det, kpts, n, ws, stream)
    return kpts, n


def rows_per_keypoint(dp):
    """Descriptor rows a keypoint may produce in the form dp.mode."""
    return {_lib.DESC_DOMINANT: 2, _lib.DESC_PLAIN: 1, _lib.DESC_RING: dp.n_orient, _lib.DESC_TURNED: 2}[dp.mode]


@_on_stream
def detect_union(max_moment, min_moment, det: DetectParams | None = None, workspace=None, stream=None):
    """RIFT's corner + edge union: (keypoints int32 [K, 3] = x, y, score bits; n int32 [1])."""
    torch = _torch()
    if det is None:
        det = defaults()[1]
    init(max_moment.device.index or 0)
    h, w = max_moment.shape
    dev = max_moment.device
    kpts = torch.empty((det.max_keypoints, 3), dtype=torch.int32, device=dev)
    n = torch.zeros((1,), dtype=torch.int32, device=dev)
    ws = workspace if workspace is not None else torch.empty(detect_union_workspace_bytes(h, w, det),
                                                             dtype=torch.uint8, device=dev)
    detect_union_into(max_moment, min_moment, det, kpts, n, ws, stream)
    return kpts, n


@_on_stream
def describe(mim, kpts, n_kpts, dp: DescParams | None = None, workspace=None, stream=None):
    """(desc int16 [R K, D] holding uint16 counts, inv_norm f32 [R K], desc_kp int32 [R K], n_desc int32 [1]),
    R = rows_per_keypoint(dp)."""
    torch = _torch()
    if dp is None:
        dp = defaults()[2]
    init(mim.device.index or 0)
    dev = mim.device
    cap = kpts.shape[0]
    d = dp.grid * dp.grid * dp.n_orient
    rows = rows_per_keypoint(dp) * cap
    desc = torch.empty((rows, d), dtype=torch.int16, device=dev)
    inv = torch.empty((rows,), dtype=torch.float32, device=dev)
    dkp = torch.empty((rows,), dtype=torch.int32, device=dev)
    nd = torch.zeros((1,), dtype=torch.int32, device=dev)
    ws = workspace if workspace is not None else torch.empty(describe_workspace_bytes(cap), dtype=torch.uint8,
                                                             device=dev)
    describe_into(mim, kpts, n_kpts, dp, desc, inv, dkp, nd, ws, stream)
    return desc, inv, dkp, nd


@_on_stream
def match(desc_a, inv_a, kp_a, n_a, desc_b, inv_b, kp_b, n_b, mp: MatchParams | None = None,
          workspace=None, stream=None):
    """(matches int32 [cap_a, 3] = kp_a, kp_b, d2 bits; n int32 [1]) sorted by kp_a."""
    torch = _torch()
    if mp is None:
        mp = defaults()[3]
    init(desc_a.device.index or 0)
    cap_a, d = desc_a.shape
    dev = desc_a.device
    out = torch.empty((cap_a, 3), dtype=torch.int32, device=dev)
    n = torch.zeros((1,), dtype=torch.int32, device=dev)
    ws = workspace if workspace is not None else torch.empty(match_workspace_bytes(cap_a, desc_b.shape[0], d, mp),
                                                             dtype=torch.uint8, device=dev)
    match_into(desc_a, inv_a, kp_a, n_a, desc_b, inv_b, kp_b, n_b, mp, out, n, ws, stream)
    return out, n


@_on_stream
def debug_response(img, scale, orient, pc: PCParams | None = None, workspace=None, stream=None):
    """Complex response EO_{scale,orient} (complex64 H x W) of one filter of the bank, by the library's kernels."""
    torch = _torch()
    if pc is None:
        pc = defaults()[0]
    init(img.device.index or 0)
    h, w = img.shape
    eo = torch.empty((h, w, 2), dtype=torch.float32, device=img.device)
    ws = workspace if workspace is not None else torch.empty(filter_workspace_bytes(h, w, pc), dtype=torch.uint8,
                                                             device=img.device)
    st = _lib.load().rift2_debug_response(_img_ptr(img), _image_dtype(img), h, w, img.stride(0), ctypes.byref(pc),
                                          int(scale), int(orient), _ptr(eo), _ptr(ws), _nbytes(ws), _stream(stream))
    _lib.check(st, "rift2_debug_response")
    return torch.view_as_complex(eo)


@_on_stream
def debug_noise(workspace, h, w, pc: PCParams | None = None, stream=None):
    """(A0 float [N_o, H, W], order statistics float [N_o, 2], T_o float64 [N_o]) that the last
    filter_mim on `workspace` left there."""
    torch = _torch()
    if pc is None:
        pc = defaults()[0]
    dev = workspace.device
    a0 = torch.empty((pc.n_orient, h, w), dtype=torch.float32, device=dev)
    ostat = torch.empty((pc.n_orient, 2), dtype=torch.float32, device=dev)
    t_o = torch.empty((pc.n_orient,), dtype=torch.float64, device=dev)
    st = _lib.load().rift2_debug_noise(_ptr(workspace), _nbytes(workspace), h, w, ctypes.byref(pc), _ptr(a0),
                                       _ptr(ostat), _ptr(t_o), _stream(stream))
    _lib.check(st, "rift2_debug_noise")
    return a0, ostat, t_o


@_on_stream
def mfma_rate(precision=_lib.PREC_FP32, waves_per_simd=3, iters=2000, reps=5, stream=None):
    """Sustained MFMA rate (TFLOP/s) of register-only chains of the FP32 (v_mfma_f32_32x32x2f32) or BF16
    (v_mfma_f32_32x32x16_bf16) GEMM's instruction with `waves_per_simd` waves on every SIMD
    (rift2_debug_mfma_rate)."""
    torch = _torch()
    sink = torch.empty((256 * 256 * waves_per_simd,), dtype=torch.float32, device="cuda")
    ms = ctypes.c_float(0.0)
    _lib.check(_lib.load().rift2_debug_mfma_rate(int(precision), int(waves_per_simd), int(iters), int(reps),
                                                 _ptr(sink), ctypes.byref(ms), _stream(stream)),
               "rift2_debug_mfma_rate")
    per_instr = 4096 if precision == _lib.PREC_FP32 else 32768
    flops = float(reps) * 256 * 4 * waves_per_simd * 32 * iters * per_instr
    return flops / (ms.value * 1e-3) / 1e12


@_on_stream
def desc_normalize(desc, inv_norm, n_rows, stream=None):
    """FP32 view fl(count * inv_norm) of the first n_rows descriptor rows (rows past it are zero)."""
    torch = _torch()
    cap, d = desc.shape
    out = torch.zeros((cap, d), dtype=torch.float32, device=desc.device)
    st = _lib.load().rift2_desc_normalize(_ptr(desc), _ptr(inv_norm), _ptr(n_rows), cap, d, _ptr(out),
                                          _stream(stream))
    _lib.check(st, "rift2_desc_normalize")
    return out


SIMILARITY_BYTES = 48  # rift2_similarity
CONSENSUS_BYTES = 16  # rift2_consensus_result


def similarity_fields(result):
    """Host dict of a rift2_similarity held in a uint8 [48] tensor."""
    raw = result.cpu()
    d = raw[:32].view(_torch().float64).tolist()
    i = raw[32:48].view(_torch().int32).tolist()
    return {"model": tuple(d), "best": i[0], "n_inliers": i[1], "n_matches": i[2], "status": i[3]}


def consensus_fields(result):
    """Host dict of a rift2_consensus_result held in a uint8 [16] tensor."""
    raw = result.cpu()
    i = raw[:8].view(_torch().int32).tolist()
    return {"n_inliers": i[0], "status": i[1], "sum_sq": raw[8:16].view(_torch().float64).item()}


@_on_stream
def ransac(matches, n_matches, kpts_a, kpts_b, words, threshold=3.0, refine=2, stream=None):
    """RANSAC over a similarity on device matches: (result uint8 [48], mask uint8 [cap], counts int32 [n_hyp]).

    words: uint32 (as int32) [n_hyp, 2] uniform sample words on the device."""
    torch = _torch()
    dev = matches.device
    init(dev.index or 0)
    cap, n_hyp = matches.shape[0], words.shape[0]
    rp = RansacParams(float(threshold), int(refine))
    counts = torch.empty((n_hyp,), dtype=torch.int32, device=dev)
    mask = torch.empty((cap,), dtype=torch.uint8, device=dev)
    result = torch.empty((SIMILARITY_BYTES,), dtype=torch.uint8, device=dev)
    ws = torch.empty(ransac_workspace_bytes(cap, n_hyp), dtype=torch.uint8, device=dev)
    ransac_into(matches, n_matches, kpts_a, kpts_b, words, rp, counts, mask, result, ws, stream)
    return result, mask, counts


@_on_stream
def consensus(model, matches, n_matches, kpts_a, kpts_b, threshold=3.0, stream=None):
    """Consensus of a model (device float64 [4]) over device matches: (result uint8 [16], mask uint8 [cap])."""
    torch = _torch()
    dev = matches.device
    init(dev.index or 0)
    cap = matches.shape[0]
    mask = torch.empty((cap,), dtype=torch.uint8, device=dev)
    result = torch.empty((CONSENSUS_BYTES,), dtype=torch.uint8, device=dev)
    ws = torch.empty(ransac_workspace_bytes(cap, 0), dtype=torch.uint8, device=dev)
    consensus_into(model, matches, n_matches, kpts_a, kpts_b, threshold, mask, result, ws, stream)
    return result, mask


# ----------------------------------------------------------------- whole pair with resident buffers

class _ImageBuffers:
    def __init__(self, h, w, pc, det, dp, dev, union=False):
        torch = _torch()
        self.union = union
        self.m = torch.empty((h, w), dtype=torch.float32, device=dev) if union else None
        cap = det.max_keypoints
        d = dp.grid * dp.grid * dp.n_orient
        self.mim = torch.empty((h, w), dtype=torch.uint8, device=dev)
        self.M = torch.empty((h, w), dtype=torch.float32, device=dev)
        self.kpts = torch.empty((cap, 3), dtype=torch.int32, device=dev)
        self.nk = torch.zeros((1,), dtype=torch.int32, device=dev)
        self.dp = dp
        self.rows = rows_per_keypoint(dp) * cap
        self.desc = torch.empty((self.rows, d), dtype=torch.int16, device=dev)
        self.inv = torch.empty((self.rows,), dtype=torch.float32, device=dev)
        self.dkp = torch.empty((self.rows,), dtype=torch.int32, device=dev)
        self.nd = torch.zeros((1,), dtype=torch.int32, device=dev)
        self.ws_filter = torch.empty(filter_workspace_bytes(h, w, pc), dtype=torch.uint8, device=dev)
        ws_det = detect_union_workspace_bytes(h, w, det) if union else detect_workspace_bytes(h, w, det)
        self.ws_detect = torch.empty(ws_det, dtype=torch.uint8, device=dev)
        self.ws_desc = torch.empty(describe_workspace_bytes(cap), dtype=torch.uint8, device=dev)


class PairPipeline:
    """All stages of one image pair on buffers that stay resident in HBM.

    run(img_a, img_b) only enqueues kernels (no host synchronisation, no
    allocation), so it can be captured into a HIP graph and replayed.
    """

    def __init__(self, h, w, pc=None, det=None, dp=None, mp=None, device=0, serial=False, ransac_words=None,
                 ransac_params=None, ring=False, union=False, batched=False):
        """ransac_words: optional device int32 [n_hyp, 2] uniform sample words; when given, every run ends
        with rift2_ransac on the pair's matches (threshold 3 px, 2 refits unless ransac_params says
        otherwise), results in ransac_result / ransac_mask.

        ring=True runs RIFT's convolution-sequence ring instead of RIFT2's dominant index (the baseline
        the paper compares against): image A is the template, described with n_orient ring rows per
        keypoint (the ring's cost sits on A's side, see rift2_match_params), image B the reference with
        one plain row per keypoint, and the matching is the ring matching.

        union=True detects with RIFT's corner + edge union (FAST on the minimum- and the maximum-moment
        maps) instead of the maximum-moment map alone.

        batched=True runs both images' filter banks as one batch (rift2_filter_mim_batch: shared
        launches) before their detection and description, instead of one image per stream."""
        torch = _torch()
        d_pc, d_det, d_dp, d_mp = defaults()
        self.pc = pc or d_pc
        self.det = det or d_det
        self.dp = dp or d_dp
        self.mp = mp or d_mp
        self.dev = torch.device("cuda", device)
        init(device)
        self.h, self.w = h, w
        self.ring = ring
        dp_a, dp_b = self.dp, self.dp
        if ring:
            dp_a, dp_b = DescParams.from_buffer_copy(self.dp), DescParams.from_buffer_copy(self.dp)
            dp_a.mode, dp_b.mode = DESC_RING, DESC_PLAIN
            self.mp = MatchParams.from_buffer_copy(self.mp)
            self.mp.ring = self.dp.n_orient
        self.a = _ImageBuffers(h, w, self.pc, self.det, dp_a, self.dev, union)
        self.b = _ImageBuffers(h, w, self.pc, self.det, dp_b, self.dev, union)
        cap = 2 * self.det.max_keypoints
        d = self.dp.grid * self.dp.grid * self.dp.n_orient
        self.out = torch.empty((cap, 3), dtype=torch.int32, device=self.dev)
        self.n_out = torch.zeros((1,), dtype=torch.int32, device=self.dev)
        self.ws_match = torch.empty(match_workspace_bytes(self.a.rows, self.b.rows, d, self.mp), dtype=torch.uint8,
                                    device=self.dev)
        self.ransac_words = ransac_words
        if ransac_words is not None:
            self.ransac_params = ransac_params or RansacParams(3.0, 2)
            self.ransac_result = torch.zeros((SIMILARITY_BYTES,), dtype=torch.uint8, device=self.dev)
            self.ransac_mask = torch.zeros((cap,), dtype=torch.uint8, device=self.dev)
            self.ws_ransac = torch.empty(ransac_workspace_bytes(cap, ransac_words.shape[0]), dtype=torch.uint8,
                                         device=self.dev)
        self.graph = None
        self._side = None
        self.serial = serial
        self.batched = batched

    def _filter_both(self, img_a, img_b, stream):
        filter_mim_batch_into([img_a, img_b], self.pc,
                              [(buf.mim, buf.M, buf.m, None, buf.ws_filter) for buf in (self.a, self.b)], stream)

    def _filter(self, img, buf, stream):
        filter_mim_into(img, self.pc, buf.mim, buf.M, buf.m, None, buf.ws_filter, stream)

    def _keypoints(self, buf, stream):
        if buf.union:
            detect_union_into(buf.M, buf.m, self.det, buf.kpts, buf.nk, buf.ws_detect, stream)
        else:
            detect_into(buf.M, self.det, buf.kpts, buf.nk, buf.ws_detect, stream)
        describe_into(buf.mim, buf.kpts, buf.nk, buf.dp, buf.desc, buf.inv, buf.dkp, buf.nd, buf.ws_desc, stream)

    def _image(self, img, buf, stream):
        self._filter(img, buf, stream)
        self._keypoints(buf, stream)

    def _match(self, stream):
        a, b = self.a, self.b
        match_into(a.desc, a.inv, a.dkp, a.nd, b.desc, b.inv, b.dkp, b.nd, self.mp, self.out, self.n_out,
                   self.ws_match, stream)
        if self.ransac_words is not None:
            ransac_into(self.out, self.n_out, a.kpts, b.kpts, self.ransac_words, self.ransac_params, None,
                        self.ransac_mask, self.ransac_result, self.ws_ransac, stream)

    def run_serial(self, img_a, img_b, stream=None):
        """Every stage on one stream, in order (used to time kernels one at a time)."""
        if self.batched:
            self._filter_both(img_a, img_b, stream)
            self._keypoints(self.a, stream)
            self._keypoints(self.b, stream)
        else:
            self._image(img_a, self.a, stream)
            self._image(img_b, self.b, stream)
        self._match(stream)

    def run(self, img_a, img_b, stream=None):
        """Image B's stages run on a second stream, overlapping image A's; matching waits for both."""
        if self.serial:
            return self.run_serial(img_a, img_b, stream)
        torch = _torch()
        main = stream if stream is not None else torch.cuda.current_stream(self.dev)
        if self._side is None:
            self._side = torch.cuda.Stream(device=self.dev)
        side = self._side
        if self.batched:
            # both filter banks in shared launches, then the two images' keypoints side by side
            self._filter_both(img_a, img_b, main)
            side.wait_stream(main)
            self._keypoints(self.a, main)
            self._keypoints(self.b, side)
        else:
            side.wait_stream(main)
            self._image(img_a, self.a, main)
            self._image(img_b, self.b, side)
        main.wait_stream(side)
        self._match(main)

    def capture(self, img_a, img_b):
        """Capture run() on static input buffers into a graph; replay() re-runs it."""
        torch = _torch()
        s = torch.cuda.Stream(device=self.dev)
        s.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(s):
            self.run(img_a, img_b, s)  # warm (module load, first-touch)
        torch.cuda.current_stream(self.dev).wait_stream(s)
        torch.cuda.synchronize(self.dev)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.run(img_a, img_b, s)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def matches(self):
        """Host copy of the matches: list of (kp_a, kp_b, d2)."""
        n = int(self.n_out.item())
        o = self.out[:n].cpu()
        return o


class PipelinedPairs:
    """Consecutive pairs overlapped: step k runs pair k's filter bank,
    detection and description (image A and image B on two streams) while
    pair k-1's matching runs on a third stream.

    Two PairPipeline buffer sets alternate: step k writes set k % 2 and
    matches set (k - 1) % 2, so a step never touches what the other half of
    the same step writes.  Steps must run in order; each step completes
    before the next one starts (both are enqueued on one stream, or replayed
    as graphs on one stream), so step k + 1 reuses the set that step k's
    matching read only after it is done.  After step k, set (k - 1) % 2
    holds pair k - 1's matches.
    """

    def __init__(self, h, w, pc=None, det=None, dp=None, mp=None, device=0):
        self.sets = [PairPipeline(h, w, pc, det, dp, mp, device) for _ in range(2)]
        self.dev = self.sets[0].dev
        self._side = None
        self._mstream = None
        self.graphs = {}

    def matched_set(self, k):
        """The buffer set holding pair k - 1's matches once step k is done."""
        return self.sets[(k + 1) % 2]

    def step(self, k, img_a, img_b, stream=None):
        """Enqueue step k (pair k's image stages, pair k - 1's matching); k = 0 matches nothing."""
        torch = _torch()
        main = stream if stream is not None else torch.cuda.current_stream(self.dev)
        if self._side is None:
            self._side = torch.cuda.Stream(device=self.dev)
            self._mstream = torch.cuda.Stream(device=self.dev)
        side, ms = self._side, self._mstream
        cur, prev = self.sets[k % 2], self.sets[(k + 1) % 2]
        side.wait_stream(main)
        if k > 0:
            ms.wait_stream(main)
            prev._match(ms)
        cur._image(img_a, cur.a, main)
        cur._image(img_b, cur.b, side)
        main.wait_stream(side)
        if k > 0:
            main.wait_stream(ms)

    def capture(self, k, img_a, img_b):
        """Graph of step k (k >= 1) on static inputs; steps with the same parity share buffer sets."""
        torch = _torch()
        s = torch.cuda.Stream(device=self.dev)
        s.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(s):
            self.step(k, img_a, img_b, s)  # warm
        torch.cuda.current_stream(self.dev).wait_stream(s)
        torch.cuda.synchronize(self.dev)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.step(k, img_a, img_b, s)
        self.graphs[k] = g
        return g


# ----------------------------------------------------------------- serving engine

class Engine:
    """Continuous batching of image-pair requests (rift2_engine_* in include/rift2.h).

    The arena (the HBM budget) is one device tensor; requests are admitted in
    arrival order as their buffers fit into it and a stream pair is free.
    submit() records an event on the current stream, and the request's first
    stage waits for it, so inputs still being written there are safe; the
    engine keeps a reference to every tensor of a request until its
    completion is polled.
    """

    def __init__(self, arena_bytes, max_inflight=8, pc=None, det=None, dp=None, mp=None, device=0):
        torch = _torch()
        d_pc, d_det, d_dp, d_mp = defaults()
        self.pc, self.det, self.dp, self.mp = pc or d_pc, det or d_det, dp or d_dp, mp or d_mp
        self.dev = torch.device("cuda", device)
        init(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.dev)
        lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(lib.rift2_engine_create(device, _ptr(self.arena), _nbytes(self.arena), max_inflight,
                                           ctypes.byref(self.pc), ctypes.byref(self.det), ctypes.byref(self.dp),
                                           ctypes.byref(self.mp), ctypes.byref(h)), "rift2_engine_create")
        self._h = h
        self._live = {}

    def set_batch(self, max_requests):
        """Queued requests of one shape admitted together, their filter banks in shared launches (1: none)."""
        _lib.check(_lib.load().rift2_engine_set_batch(self._h, int(max_requests)), "rift2_engine_set_batch")

    def request_bytes(self, h, w, max_keypoints=0):
        return _lib.load().rift2_engine_request_bytes(h, w, max_keypoints, ctypes.byref(self.pc),
                                                      ctypes.byref(self.det), ctypes.byref(self.dp),
                                                      ctypes.byref(self.mp))

    @staticmethod
    def keypoints(h, w, max_keypoints=0):
        return max_keypoints if max_keypoints > 0 else int(2e-3 * h * w)

    def submit(self, rid, img_a, img_b, max_keypoints=0, out=None, n_out=None):
        """Queue one pair; returns the (out, n_out) device tensors the match stage writes."""
        torch = _torch()
        h, w = img_a.shape
        k = self.keypoints(h, w, max_keypoints)
        if out is None:
            out = torch.empty((2 * k, 3), dtype=torch.int32, device=self.dev)
        if n_out is None:
            n_out = torch.empty((1,), dtype=torch.int32, device=self.dev)  # the match stage always writes it
        ready = torch.cuda.Event()
        ready.record(torch.cuda.current_stream(self.dev))
        if img_b.shape != img_a.shape or img_b.dtype != img_a.dtype:
            raise ValueError("both images of a request have one size and type")
        # the engine reads images with a row pitch of W
        r = _lib.Request(int(rid), _ptr(img_a), _ptr(img_b), _image_dtype(img_a), h, w, max_keypoints,
                         _ptr(out), _ptr(n_out), ready.cuda_event)
        _lib.check(_lib.load().rift2_engine_submit(self._h, ctypes.byref(r)), "rift2_engine_submit")
        self._live[int(rid)] = (img_a, img_b, out, n_out, ready)
        return out, n_out

    def poll(self, max_done=256):
        """Completed requests: [{id, status, gpu_ms, admit_ms, done_ms, batch, out, n_out}]."""
        buf = (_lib.Completion * max_done)()
        n = _lib.load().rift2_engine_poll(self._h, buf, max_done)
        if n < 0:
            raise Rift2Error(-n, "rift2_engine_poll")
        res = []
        for c in buf[:n]:
            live = self._live.pop(int(c.id), None)
            res.append({"id": int(c.id), "status": int(c.status), "gpu_ms": float(c.gpu_ms),
                        "admit_ms": float(c.admit_ms), "done_ms": float(c.done_ms), "batch": int(c.batch),
                        "out": live[2] if live else None, "n_out": live[3] if live else None})
        return res

    def pending(self):
        return int(_lib.load().rift2_engine_pending(self._h))

    def drain(self, sleep_s=0.0):
        import time

        done = []
        while self.pending():
            done += self.poll()
            if sleep_s:
                time.sleep(sleep_s)
        return done

    def close(self):
        if self._h is not None:
            _lib.load().rift2_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- diagnostics

def profile_enable(on: bool = True) -> None:
    _lib.check(_lib.load().rift2_profile_enable(1 if on else 0), "rift2_profile_enable")


def profile_read():
    """{stage: (total_ms, launches)} accumulated since the last read (waits for the events)."""
    lib = _lib.load()
    n = len(STAGES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    lib.rift2_profile_read(ms, cnt, n)
    return {STAGES[i]: (ms[i], cnt[i]) for i in range(n)}
