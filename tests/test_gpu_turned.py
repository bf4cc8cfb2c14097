"""GPU parity of the descriptor form whose sampling grid is turned by the dominant index
(RIFT2_DESC_TURNED) against the oracle (describe.describe_rotated).

The form is integer counting on exact fixed-point sample positions, so the bar
is bit-exact: rows, row order, keypoint indices and inverse norms.  An exactly
rotated pair then matches through the whole GPU pipeline, and the GPU's
outlier removal recovers the rotation.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle import filterbank, detect, describe, match, outliers as ol  # noqa: E402
from synth import make_pair  # noqa: E402
from synth.matches import sample_words  # noqa: E402


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_00319_amd as r2

    return r2, torch.device("cuda:0")


def _check(r2, dev, mim, kpts, tag, n_orient=6, byte_offset=0, patch=96, grid=6):
    """byte_offset > 0 places the MIM that many bytes into its device buffer (rows not 4-byte aligned)."""
    print(f"[turned parity] {tag} n={len(kpts)} N_o={n_orient} patch={patch} grid={grid}", flush=True)
    dp = r2.defaults()[2]
    dp.n_orient = n_orient
    dp.patch_size = patch
    dp.grid = grid
    dp.mode = r2.DESC_TURNED
    c_ref, k_ref, _ = describe.describe_rotated(mim, kpts,
                                                oracle.DescParams(patch_size=patch, grid=grid, n_orient=n_orient))
    kp = np.zeros((max(len(kpts), 1), 3), dtype=np.int32)
    kp[:len(kpts), :2] = kpts
    buf = torch.zeros(mim.size + byte_offset, dtype=torch.uint8, device=dev)
    buf[byte_offset:] = torch.from_numpy(mim.reshape(-1)).to(dev)
    mim_dev = buf[byte_offset:].view(mim.shape)
    assert mim_dev.data_ptr() % 4 == byte_offset % 4
    d, inv, dk, nd = r2.describe(mim_dev, torch.from_numpy(kp).to(dev),
                                 torch.tensor([len(kpts)], dtype=torch.int32, device=dev), dp)
    nd = int(nd.item())
    assert nd == len(c_ref), f"{tag}: {nd} vs {len(c_ref)} rows"
    assert np.array_equal(d[:nd].cpu().numpy().astype(np.uint16), c_ref), f"{tag}: counts differ"
    assert np.array_equal(dk[:nd].cpu().numpy(), k_ref), f"{tag}: keypoint index differs"
    assert np.array_equal(inv[:nd].cpu().numpy(), match.inv_norms(c_ref, np.float32)), f"{tag}: norms differ"
    return nd - len(kpts)


def test_turned_rows_bitexact():
    r2, dev = _gpu()
    a, _, _ = make_pair(0, 0)
    fm = filterbank.filter_mim(a, oracle.PCParams())
    kp, _ = detect.detect(fm["M"], oracle.DetectParams(max_keypoints=500), dtype=np.float32)
    _check(r2, dev, fm["mim"], kp, "c0 A")
    rng = np.random.default_rng(51)
    mim8 = rng.integers(0, 8, size=(300, 260)).astype(np.uint8)
    # anywhere in the image: turned samples leave it near the borders
    pts = np.stack([rng.integers(0, 260, 401), rng.integers(0, 300, 401)], 1).astype(np.int32)
    _check(r2, dev, mim8, pts, "random N_o=8, all positions", n_orient=8)
    mim2 = (rng.integers(0, 2, size=(200, 230)) * 3).astype(np.uint8)  # two values: many second rows
    pts = np.stack([rng.integers(30, 200, 333), rng.integers(30, 170, 333)], 1).astype(np.int32)
    assert _check(r2, dev, mim2, pts, "two-valued") > 100
    # the kernel copies each keypoint's MIM window with dword loads when every row starts 4-byte
    # aligned and byte by byte otherwise: an odd width, and a MIM starting one byte into its buffer
    mim3 = rng.integers(0, 6, size=(211, 257)).astype(np.uint8)
    pts = np.stack([rng.integers(0, 257, 301), rng.integers(0, 211, 301)], 1).astype(np.int32)
    _check(r2, dev, mim3, pts, "odd width, all positions")
    _check(r2, dev, mim8, np.stack([rng.integers(0, 260, 201), rng.integers(0, 300, 201)], 1).astype(np.int32),
           "N_o=8, MIM one byte into its buffer", n_orient=8, byte_offset=1)


def test_turned_rows_small_patch_build():
    """The 64-pixel patch, 4 x 4 grid build: keypoints anywhere, a MIM with a dominant value in most
    patches and a second row where two values balance (40 of 300)."""
    r2, dev = _gpu()
    rng = np.random.default_rng(29)
    h, w = 150, 230
    mixed = np.where(rng.random((h, w)) < np.linspace(0.0, 1.0, w)[None, :], 2, 4).astype(np.uint8)
    mixed[rng.random((h, w)) < 0.2] = 0
    pts = np.stack([rng.integers(0, w, 300), rng.integers(0, h, 300)], 1).astype(np.int32)
    assert 0 < _check(r2, dev, mixed, pts, "patch 64 mixed", patch=64, grid=4) < 300


def test_turned_pipeline_matches_a_rotated_pair_and_ransac_recovers_it():
    """Image B = A turned a quarter turn (MIM values move by N_o/2 exactly).  With the turned grid
    the pair matches; the GPU's RANSAC finds the quarter turn, and the ground-truth consensus counts
    as many correct matches as the oracle's own pipeline gives (within 5 %)."""
    r2, dev = _gpu()
    a, _, _ = make_pair(0, 0)
    b = np.ascontiguousarray(np.rot90(a))
    n = a.shape[0]
    pc, det, dp, mp = r2.defaults()
    det.max_keypoints = 500
    dp.mode = r2.DESC_TURNED
    words = torch.from_numpy(sample_words(61, 1024).view(np.int32).copy()).to(dev)
    pipe = r2.PairPipeline(n, n, pc, det, dp, mp, ransac_words=words)
    pipe.run(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
    torch.cuda.synchronize()
    f = r2.similarity_fields(pipe.ransac_result)
    # np.rot90: (x, y) -> (y, W - 1 - x), i.e. a = cos = 0, b = sin = -1, t = (0, W - 1)
    truth = (0.0, -1.0, 0.0, float(n - 1))
    assert f["status"] == 0 and f["n_inliers"] >= 50
    assert all(abs(u - v) < tol for u, v, tol in zip(f["model"], truth, (1e-3, 1e-3, 0.5, 0.5))), f["model"]
    gt = torch.tensor(truth, dtype=torch.float64, device=dev)
    res, _ = r2.consensus(gt, pipe.out, pipe.n_out, pipe.a.kpts, pipe.b.kpts, threshold=3.0)
    n_gpu = r2.consensus_fields(res)["n_inliers"]
    fa, fb, m = oracle.pipeline.match_pair(a, b, det=oracle.DetectParams(max_keypoints=500), turned=True)
    ref = ol.gt_metrics(truth, *ol.match_coords(fa["kpts"], fb["kpts"], m[0], m[1]))
    print(f"rot90 pair: gpu {int(pipe.n_out.item())} matches, {n_gpu} correct; oracle {len(m[0])} matches, "
          f"{ref['n_correct']} correct; ransac inliers {f['n_inliers']}", flush=True)
    assert n_gpu > 100 and abs(n_gpu - ref["n_correct"]) <= 0.05 * ref["n_correct"]
