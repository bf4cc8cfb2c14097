"""The C ABI library loads, exports every declared symbol and validates arguments on the host.

No compute call reaches a kernel here: every call below fails validation
before anything is enqueued, so these run without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rift2.h")


def _lib():
    from paper_2303_00319_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("librift2.so not built")
    return _lib, _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rift2_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    _l, lib = _lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), f"{name} missing from librift2.so"
    assert set(names) == set(_l.EXPORTS)


def test_defaults_match_the_paper_settings():
    _l, lib = _lib()
    pc, det, desc, mp = _l.PCParams(), _l.DetectParams(), _l.DescParams(), _l.MatchParams()
    lib.rift2_default_params(ctypes.byref(pc), ctypes.byref(det), ctypes.byref(desc), ctypes.byref(mp))
    assert (pc.n_scales, pc.n_orient) == (4, 6)
    assert det.max_keypoints == 5000 and det.patch_size == 96 and abs(det.fast_threshold - 0.001) < 1e-9
    assert (desc.patch_size, desc.grid, desc.n_orient, desc.dominant_num, desc.dominant_den) == (96, 6, 6, 4, 5)
    assert abs(mp.ratio_sq - 0.81) < 1e-7 and mp.precision == _l.PREC_FP32
    lib.rift2_default_params(None, None, None, None)


def test_sizes_and_workspaces():
    _l, lib = _lib()
    for n in (256, 512, 768, 1024, 1536, 2048, 4096):
        assert lib.rift2_size_supported(n) == 1
    for n in (0, 100, 1000, 640, 8192):
        assert lib.rift2_size_supported(n) == 0
    pc = _l.PCParams()
    lib.rift2_default_params(ctypes.byref(pc), None, None, None)
    ws = lib.rift2_filter_workspace_size(1024, 1024, ctypes.byref(pc))
    # row spectrum + 24 filter planes (complex64) + A0 + candidate list
    assert ws >= 1024 * 1024 * (8 + 24 * 8 + 6 * 4 + 6 * 4)
    assert lib.rift2_filter_workspace_size(1000, 1024, ctypes.byref(pc)) == 0
    bad = _l.PCParams.from_buffer_copy(pc)
    bad.n_orient = 9
    assert lib.rift2_filter_workspace_size(1024, 1024, ctypes.byref(bad)) == 0
    det = _l.DetectParams(0.001, 5000, 96)
    assert lib.rift2_detect_workspace_size(1024, 1024, ctypes.byref(det)) > 0
    assert lib.rift2_describe_workspace_size(5000) >= 5000 * 4
    mp = _l.MatchParams(0.81, _l.PREC_BF16)
    assert lib.rift2_match_workspace_size(10000, 10000, 216, ctypes.byref(mp)) > 10000 * 224 * 2 * 2
    assert lib.rift2_match_workspace_size(0, 10, 216, ctypes.byref(mp)) == 0


def test_argument_errors_return_before_any_launch():
    _l, lib = _lib()
    pc = _l.PCParams()
    det = _l.DetectParams(0.001, 5000, 96)
    desc = _l.DescParams()
    mp = _l.MatchParams(0.81, 0)
    lib.rift2_default_params(ctypes.byref(pc), None, ctypes.byref(desc), None)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    null = ctypes.c_void_p(0)
    # null image
    assert lib.rift2_filter_mim(null, 0, 1024, 1024, 1024, ctypes.byref(pc), fake, fake, null, null, fake,
                                1 << 40, null) == _l.ERR_INVALID_ARG
    # unsupported size
    assert lib.rift2_filter_mim(fake, 0, 1000, 1024, 1024, ctypes.byref(pc), fake, fake, null, null, fake,
                                1 << 40, null) == _l.ERR_UNSUPPORTED
    # pitch smaller than width
    assert lib.rift2_filter_mim(fake, 0, 1024, 1024, 512, ctypes.byref(pc), fake, fake, null, null, fake,
                                1 << 40, null) == _l.ERR_INVALID_ARG
    # bad dtype
    assert lib.rift2_filter_mim(fake, 7, 1024, 1024, 1024, ctypes.byref(pc), fake, fake, null, null, fake,
                                1 << 40, null) == _l.ERR_INVALID_ARG
    # workspace too small
    assert lib.rift2_filter_mim(fake, 0, 1024, 1024, 1024, ctypes.byref(pc), fake, fake, null, null, fake,
                                1024, null) == _l.ERR_WORKSPACE
    # (N_s, N_o) not instantiated
    odd = _l.PCParams.from_buffer_copy(pc)
    odd.n_scales = 3
    assert lib.rift2_filter_mim(fake, 0, 1024, 1024, 1024, ctypes.byref(odd), fake, fake, null, null, fake,
                                1 << 40, null) == _l.ERR_UNSUPPORTED
    # detect: negative threshold, small workspace
    neg = _l.DetectParams(-1.0, 10, 96)
    assert lib.rift2_detect(fake, 256, 256, ctypes.byref(neg), fake, fake, fake, 1 << 30, null) == _l.ERR_INVALID_ARG
    assert lib.rift2_detect(fake, 256, 256, ctypes.byref(det), fake, fake, fake, 16, null) == _l.ERR_WORKSPACE
    # describe: descriptor capacity below 2 x keypoint capacity
    assert lib.rift2_describe(fake, 256, 256, fake, fake, 100, ctypes.byref(desc), fake, fake, fake, 150, fake, fake,
                              1 << 20, null) == _l.ERR_INVALID_ARG
    # describe: geometry without a kernel
    odd_d = _l.DescParams(36, 6, 6, 4, 5)
    assert lib.rift2_describe(fake, 256, 256, fake, fake, 100, ctypes.byref(odd_d), fake, fake, fake, 200, fake, fake,
                              1 << 20, null) == _l.ERR_UNSUPPORTED
    # match: unsupported depth, bad precision, bad ratio
    assert lib.rift2_match(fake, fake, fake, fake, 10, fake, fake, fake, fake, 10, 100, ctypes.byref(mp), fake, fake,
                           fake, 1 << 30, null) == _l.ERR_UNSUPPORTED
    mp_bad = _l.MatchParams(0.81, 5)
    assert lib.rift2_match(fake, fake, fake, fake, 10, fake, fake, fake, fake, 10, 216, ctypes.byref(mp_bad), fake,
                           fake, fake, 1 << 30, null) == _l.ERR_INVALID_ARG
    mp_bad = _l.MatchParams(0.0, 0)
    assert lib.rift2_match(fake, fake, fake, fake, 10, fake, fake, fake, fake, 10, 216, ctypes.byref(mp_bad), fake,
                           fake, fake, 1 << 30, null) == _l.ERR_INVALID_ARG
    assert lib.rift2_status_string(_l.ERR_WORKSPACE) == b"workspace too small"


def test_ransac_validation_and_workspace():
    _l, lib = _lib()
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    rp = _l.RansacParams(3.0, 2)
    assert lib.rift2_ransac_workspace_size(5000, 4096) >= 5000 * 16 + 4096 * 4
    assert lib.rift2_ransac_workspace_size(0, 10) == 0
    assert lib.rift2_ransac_workspace_size((1 << 17) + 1, 10) == 0
    assert lib.rift2_ransac_workspace_size(10, (1 << 20) + 1) == 0

    def call(matches=fake, cap=100, words=fake, n_hyp=64, params=rp, ws_bytes=1 << 20, mask=fake):
        return lib.rift2_ransac(matches, fake, cap, fake, 10, fake, 10, words, n_hyp, ctypes.byref(params), null,
                                mask, fake, fake, ws_bytes, null)

    assert call(matches=null) == _l.ERR_INVALID_ARG
    assert call(mask=null) == _l.ERR_INVALID_ARG
    assert call(n_hyp=0) == _l.ERR_INVALID_ARG
    assert call(params=_l.RansacParams(0.0, 2)) == _l.ERR_INVALID_ARG
    assert call(params=_l.RansacParams(float("nan"), 2)) == _l.ERR_INVALID_ARG
    assert call(params=_l.RansacParams(3.0, 17)) == _l.ERR_INVALID_ARG
    assert call(words=ctypes.c_void_p(0x1004)) == _l.ERR_INVALID_ARG  # misaligned word pairs
    assert call(cap=(1 << 17) + 1) == _l.ERR_UNSUPPORTED
    assert call(ws_bytes=64) == _l.ERR_WORKSPACE
    assert lib.rift2_consensus(fake, fake, fake, 100, fake, 10, fake, 10, -1.0, null, fake, fake, 1 << 20,
                               null) == _l.ERR_INVALID_ARG
    assert lib.rift2_consensus(null, fake, fake, 100, fake, 10, fake, 10, 3.0, null, fake, fake, 1 << 20,
                               null) == _l.ERR_INVALID_ARG
    assert lib.rift2_consensus(fake, fake, fake, 100, fake, 10, fake, 10, 3.0, null, fake, fake, 16,
                               null) == _l.ERR_WORKSPACE


def test_binding_fails_loudly_without_the_library(tmp_path):
    from paper_2303_00319_amd import _lib as l

    with pytest.raises(RuntimeError):
        saved = l._LIB
        l._LIB = None
        try:
            l.load(str(tmp_path / "missing.so"))
        finally:
            l._LIB = saved


def test_variant_forms_are_validated_on_the_host():
    _l, lib = _lib()
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    pc, det, desc, mp = _l.PCParams(), _l.DetectParams(), _l.DescParams(), _l.MatchParams()
    lib.rift2_default_params(ctypes.byref(pc), ctypes.byref(det), ctypes.byref(desc), ctypes.byref(mp))
    assert desc.mode == _l.DESC_DOMINANT and mp.ring == 0
    # describe: unknown form; ring rows need n_orient x kpt_cap rows; plain needs kpt_cap
    for mode, cap, want in ((7, 1000, _l.ERR_INVALID_ARG), (_l.DESC_RING, 599, _l.ERR_INVALID_ARG),
                            (_l.DESC_PLAIN, 99, _l.ERR_INVALID_ARG), (_l.DESC_TURNED, 199, _l.ERR_INVALID_ARG)):
        d = _l.DescParams.from_buffer_copy(desc)
        d.mode = mode
        assert lib.rift2_describe(fake, 256, 256, fake, fake, 100, ctypes.byref(d), fake, fake, fake, cap, fake, fake,
                                  1 << 30, null) == want, mode
    assert lib.rift2_describe_workspace_size(100) >= 100 * (4 + 288 * 2 + 4)
    # match: ring of 1 row, ring beyond 8, ring with FP8 candidates
    for ring, prec, want in ((1, 0, _l.ERR_INVALID_ARG), (9, 0, _l.ERR_INVALID_ARG), (6, _l.PREC_FP8, _l.ERR_UNSUPPORTED)):
        m = _l.MatchParams(0.81, prec, ring)
        assert lib.rift2_match(fake, fake, fake, fake, 60, fake, fake, fake, fake, 10, 216, ctypes.byref(m), fake, fake,
                               fake, 1 << 30, null) == want, (ring, prec)
    # corner + edge union: the second map is required and 16-byte aligned; its workspace is larger
    assert lib.rift2_detect_union(fake, null, 256, 256, ctypes.byref(det), fake, fake, fake, 1 << 30,
                                  null) == _l.ERR_INVALID_ARG
    assert lib.rift2_detect_union(fake, ctypes.c_void_p(0x1004), 256, 256, ctypes.byref(det), fake, fake, fake,
                                  1 << 30, null) == _l.ERR_INVALID_ARG
    assert (lib.rift2_detect_union_workspace_size(1024, 1024, ctypes.byref(det)) >
            lib.rift2_detect_workspace_size(1024, 1024, ctypes.byref(det)))
    # the serving engine serves RIFT2's form only
    ring_dp = _l.DescParams.from_buffer_copy(desc)
    ring_dp.mode = _l.DESC_RING
    handle = ctypes.c_void_p(0)
    assert lib.rift2_engine_create(0, ctypes.c_void_p(0x10000), 1 << 30, 4, ctypes.byref(pc), ctypes.byref(det),
                                   ctypes.byref(ring_dp), ctypes.byref(mp), ctypes.byref(handle)) == _l.ERR_UNSUPPORTED


def test_fft_calls_refuse_a_device_without_rift2_init():
    """Without rift2_init on the current device (here: no device at all) the FFT calls return
    RIFT2_ERR_NOT_INITIALIZED instead of running against empty twiddle tables."""
    _l, lib = _lib()
    try:
        import torch

        if torch.cuda.is_available():
            pytest.skip("a GPU is present; this process may already have initialised it")
    except ImportError:
        pass
    pc = _l.PCParams()
    lib.rift2_default_params(ctypes.byref(pc), None, None, None)
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    assert lib.rift2_filter_mim(fake, 0, 1024, 1024, 1024, ctypes.byref(pc), fake, fake, null, null, fake,
                                1 << 40, null) == _l.ERR_NOT_INITIALIZED
    assert lib.rift2_debug_response(fake, 0, 512, 512, 512, ctypes.byref(pc), 1, 2, fake, fake, 1 << 40,
                                    null) == _l.ERR_NOT_INITIALIZED
    assert b"rift2_init" in lib.rift2_status_string(_l.ERR_NOT_INITIALIZED)


def test_debug_and_normalize_calls_validate_on_the_host():
    _l, lib = _lib()
    pc = _l.PCParams()
    lib.rift2_default_params(ctypes.byref(pc), None, None, None)
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    # filter index out of range, misaligned output, unsupported size, small workspace
    for s, o in ((4, 0), (0, 6), (-1, 0)):
        assert lib.rift2_debug_response(fake, 0, 256, 256, 256, ctypes.byref(pc), s, o, fake, fake, 1 << 40,
                                        null) == _l.ERR_INVALID_ARG
    assert lib.rift2_debug_response(fake, 0, 256, 256, 256, ctypes.byref(pc), 0, 0, ctypes.c_void_p(0x1004), fake,
                                    1 << 40, null) == _l.ERR_INVALID_ARG
    assert lib.rift2_debug_response(fake, 0, 250, 256, 256, ctypes.byref(pc), 0, 0, fake, fake, 1 << 40,
                                    null) == _l.ERR_UNSUPPORTED
    assert lib.rift2_debug_response(fake, 0, 256, 256, 256, ctypes.byref(pc), 0, 0, fake, fake, 64,
                                    null) == _l.ERR_WORKSPACE
    assert lib.rift2_debug_noise(null, 1 << 40, 256, 256, ctypes.byref(pc), fake, fake, fake, null) == _l.ERR_INVALID_ARG
    assert lib.rift2_debug_noise(fake, 64, 256, 256, ctypes.byref(pc), fake, fake, fake, null) == _l.ERR_WORKSPACE
    assert lib.rift2_desc_normalize(null, fake, fake, 10, 216, fake, null) == _l.ERR_INVALID_ARG
    assert lib.rift2_desc_normalize(fake, fake, fake, 0, 216, fake, null) == _l.ERR_INVALID_ARG


def test_mutual_matching_is_validated_and_sized():
    _l, lib = _lib()
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    for prec in (_l.PREC_FP32, _l.PREC_BF16, _l.PREC_FP8):
        plain = lib.rift2_match_workspace_size(10000, 9000, 216, ctypes.byref(_l.MatchParams(0.81, prec, 0, 0)))
        mutual = lib.rift2_match_workspace_size(10000, 9000, 216, ctypes.byref(_l.MatchParams(0.81, prec, 0, 1)))
        # the reverse pass adds its candidate lists and one nearest A row per B row
        assert mutual >= plain + 9000 * 4 + 9000 * 6 * 8
    bad = _l.MatchParams(0.81, 0, 0, 2)
    assert lib.rift2_match(fake, fake, fake, fake, 10, fake, fake, fake, fake, 10, 216, ctypes.byref(bad), fake, fake,
                           fake, 1 << 30, null) == _l.ERR_INVALID_ARG
    ring = _l.MatchParams(0.81, 0, 6, 1)
    assert lib.rift2_match(fake, fake, fake, fake, 60, fake, fake, fake, fake, 10, 216, ctypes.byref(ring), fake, fake,
                           fake, 1 << 30, null) == _l.ERR_UNSUPPORTED


def test_detect_noalloc_validates_on_the_host():
    """rift2_detect_noalloc checks its arguments and its 20 MiB scratch limit before touching a device."""
    _l, lib = _lib()
    det = _l.DetectParams()
    lib.rift2_default_params(None, ctypes.byref(det), None, None)
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    assert lib.rift2_detect_noalloc(null, 1024, 1024, ctypes.byref(det), fake, fake, null) == _l.ERR_INVALID_ARG
    assert lib.rift2_detect_noalloc(fake, 4, 1024, ctypes.byref(det), fake, fake, null) == _l.ERR_INVALID_ARG
    det.max_keypoints = 50000
    assert lib.rift2_detect_workspace_size(4096, 4096, ctypes.byref(det)) > 20 << 20
    assert lib.rift2_detect_noalloc(fake, 4096, 4096, ctypes.byref(det), fake, fake, null) == _l.ERR_WORKSPACE
    assert lib.rift2_detect_workspace_size(2048, 2048, ctypes.byref(det)) <= 20 << 20
    try:
        import torch

        if torch.cuda.is_available():
            return
    except ImportError:
        pass
    # no device at all: nothing has been initialised
    assert lib.rift2_detect_noalloc(fake, 2048, 2048, ctypes.byref(det), fake, fake, null) == _l.ERR_NOT_INITIALIZED


def test_filter_batch_validates_on_the_host():
    _l, lib = _lib()
    pc = _l.PCParams()
    lib.rift2_default_params(ctypes.byref(pc), None, None, None)
    jobs = (_l.FilterJob * 9)()
    fake = 0x1000
    for j in jobs:
        j.img, j.mim, j.max_moment, j.workspace, j.workspace_bytes = fake, fake, fake, fake, 1 << 40
    null = ctypes.c_void_p(0)
    assert lib.rift2_filter_mim_batch(0, jobs, 0, 256, 256, 256, ctypes.byref(pc), null) == _l.ERR_INVALID_ARG
    assert lib.rift2_filter_mim_batch(9, jobs, 0, 256, 256, 256, ctypes.byref(pc), null) == _l.ERR_INVALID_ARG
    jobs[1].mim = 0
    assert lib.rift2_filter_mim_batch(2, jobs, 0, 256, 256, 256, ctypes.byref(pc), null) == _l.ERR_INVALID_ARG
    jobs[1].mim = fake
    jobs[1].workspace_bytes = 16
    assert lib.rift2_filter_mim_batch(2, jobs, 0, 256, 256, 256, ctypes.byref(pc), null) == _l.ERR_WORKSPACE
    assert lib.rift2_filter_mim_batch(2, jobs, 0, 250, 256, 256, ctypes.byref(pc), null) == _l.ERR_UNSUPPORTED
    # two jobs on one workspace (or overlapping ones) are refused before anything runs
    jobs[1].workspace_bytes = 1 << 40
    assert lib.rift2_filter_mim_batch(2, jobs, 0, 256, 256, 256, ctypes.byref(pc), null) == _l.ERR_INVALID_ARG
    need = lib.rift2_filter_workspace_size(256, 256, ctypes.byref(pc))
    jobs[1].workspace = fake + need - 256
    assert lib.rift2_filter_mim_batch(2, jobs, 0, 256, 256, 256, ctypes.byref(pc), null) == _l.ERR_INVALID_ARG
    try:
        import torch

        if torch.cuda.is_available():
            return
    except ImportError:
        pass
    # no device at all: disjoint workspaces pass the host checks and stop at the missing initialisation
    jobs[1].workspace = fake + need
    assert lib.rift2_filter_mim_batch(2, jobs, 0, 256, 256, 256, ctypes.byref(pc), null) == _l.ERR_NOT_INITIALIZED


def test_binding_refuses_tensor_layouts_the_library_cannot_read():
    """Outputs, tables and workspaces are dense blocks; an image may have pitched rows but a unit column
    stride.  Checked on host tensors: only strides are looked at."""
    torch = pytest.importorskip("torch")
    import paper_2303_00319_amd as r2

    a = torch.zeros((64, 96), dtype=torch.float32)
    assert r2._ptr(a).value == a.data_ptr() and r2._ptr(None).value is None
    for bad in (a.t(), a[:, :48], a[::2]):
        with pytest.raises(ValueError):
            r2._ptr(bad)
    crop = a[3:40, 5:70]
    assert r2._img_ptr(crop).value == crop.data_ptr()
    for bad in (a.t(), a[:, ::2], a.reshape(-1)):
        with pytest.raises(ValueError):
            r2._img_ptr(bad)


def test_mfma_calibration_validates_on_the_host():
    _l, lib = _lib()
    ms = ctypes.c_float(0.0)
    sink = ctypes.c_void_p(0x1000)
    for prec, w, it, reps, snk, out in ((0, 0, 10, 1, sink, ctypes.byref(ms)), (0, 5, 10, 1, sink, ctypes.byref(ms)),
                                        (1, 3, 0, 1, sink, ctypes.byref(ms)), (1, 3, 10, 0, sink, ctypes.byref(ms)),
                                        (0, 3, 10, 1, None, ctypes.byref(ms)), (0, 3, 10, 1, sink, None),
                                        (2, 3, 10, 1, sink, ctypes.byref(ms)), (-1, 3, 10, 1, sink, ctypes.byref(ms))):
        assert lib.rift2_debug_mfma_rate(prec, w, it, reps, snk, out, None) == _l.ERR_INVALID_ARG
