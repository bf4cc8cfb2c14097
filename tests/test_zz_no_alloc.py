"""rift2_detect_noalloc (detection on the library's own device scratch) against rift2_detect.

Two calls in a row through the C ABI, the second on a smaller map with a
smaller keypoint cap, each compared bit for bit with rift2_detect on a
workspace of its own; plus the host-side size limit.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _moment_map(r2, dev, seed, n):
    """A max-moment map of a synthetic scene of side n (the detector's real input)."""
    from synth.gen import make_scene

    img = make_scene(n, 200 * n * n // (1024 * 1024) + 20, 60 * n * n // (1024 * 1024) + 8, 255,
                     np.random.default_rng(seed)).astype(np.uint8)
    pc = r2.defaults()[0]
    return r2.filter_mim(torch.from_numpy(img).to(dev), pc)["M"]


def _both(r2, moment, max_keypoints):
    from paper_2303_00319_amd import _lib

    det = r2.defaults()[1]
    det.max_keypoints = max_keypoints
    dev = moment.device
    h, w = moment.shape
    ref_k = torch.empty((max_keypoints, 3), dtype=torch.int32, device=dev)
    ref_n = torch.empty((1,), dtype=torch.int32, device=dev)
    ws = torch.empty(r2.detect_workspace_bytes(h, w, det), dtype=torch.uint8, device=dev)
    r2.detect_into(moment, det, ref_k, ref_n, ws)
    got_k = torch.full((max_keypoints, 3), -7, dtype=torch.int32, device=dev)
    got_n = torch.full((1,), -7, dtype=torch.int32, device=dev)
    lib = _lib.load()
    st = lib.rift2_detect_noalloc(ctypes.c_void_p(moment.data_ptr()), h, w, ctypes.byref(det),
                                  ctypes.c_void_p(got_k.data_ptr()), ctypes.c_void_p(got_n.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.OK, lib.rift2_status_string(st)
    torch.cuda.synchronize()
    n = int(ref_n.item())
    assert int(got_n.item()) == n
    assert torch.equal(got_k[:n], ref_k[:n])
    return n


def test_detect_noalloc_equals_detect_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_00319_amd as r2

    r2.init(0)
    dev = torch.device("cuda:0")
    big = _moment_map(r2, dev, 11, 1024)
    small = _moment_map(r2, dev, 12, 512)
    print("[no-alloc detect] 1024^2, 5000 keypoints", flush=True)
    n1 = _both(r2, big, 5000)
    print(f"  {n1} keypoints equal; 512^2, 700 keypoints", flush=True)
    n2 = _both(r2, small, 700)
    print(f"  {n2} keypoints equal", flush=True)
    assert n1 > 1000 and n2 > 100


def test_detect_noalloc_rejects_sizes_beyond_its_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_00319_amd as r2
    from paper_2303_00319_amd import _lib

    r2.init(0)
    lib = _lib.load()
    det = r2.defaults()[1]
    det.max_keypoints = 50000
    fake = ctypes.c_void_p(0x1000)
    st = lib.rift2_detect_noalloc(fake, 4096, 4096, ctypes.byref(det), fake, fake, ctypes.c_void_p(0))
    assert st == _lib.ERR_WORKSPACE
