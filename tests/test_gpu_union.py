"""GPU parity of RIFT's corner + edge detector union (rift2_detect_union) against the oracle.

FAST on each map is correctly rounded FP32 arithmetic, so given the same FP32
maximum- and minimum-moment maps the union must be bit-exact: positions,
order and score bits.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle import filterbank, detect  # noqa: E402
from synth import make_pair  # noqa: E402


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_00319_amd as r2

    return r2, torch.device("cuda:0")


def _check(r2, dev, e32, c32, k, tag, patch=96):
    print(f"[union parity] {tag} shape={e32.shape} K={k}", flush=True)
    det = r2.defaults()[1]
    det.max_keypoints = k
    det.patch_size = patch
    ref_pts, ref_sc = detect.detect_union(e32, c32, oracle.DetectParams(max_keypoints=k, patch_size=patch),
                                          dtype=np.float32)
    kp, n = r2.detect_union(torch.from_numpy(e32).to(dev), torch.from_numpy(c32).to(dev), det)
    n = int(n.item())
    got = kp[:n].cpu().numpy()
    assert n == len(ref_pts), f"{tag}: {n} vs {len(ref_pts)} keypoints"
    assert np.array_equal(got[:, :2], ref_pts), f"{tag}: positions differ"
    assert np.array_equal(got[:, 2].view(np.float32), np.asarray(ref_sc, np.float32)), f"{tag}: scores differ"
    return n


def test_union_bitexact_on_oracle_moment_maps():
    r2, dev = _gpu()
    a, _, _ = make_pair(0, 0)
    fm = filterbank.filter_mim(a, oracle.PCParams())
    e32, c32 = fm["M"].astype(np.float32), fm["m"].astype(np.float32)
    n = _check(r2, dev, e32, c32, 500, "c0 A")
    n_edge = len(detect.detect(e32, oracle.DetectParams(max_keypoints=10 ** 6), dtype=np.float32)[0])
    n_all = _check(r2, dev, e32, c32, 100000, "c0 A, every point")
    assert n == 500 and n_all > n_edge  # the corner map adds points
    _check(r2, dev, e32, c32, 37, "c0 A small K")


def test_union_random_maps_ties_and_special_cases():
    r2, dev = _gpu()
    rng = np.random.default_rng(31)
    e = (rng.integers(0, 6, size=(256, 256)) / 5.0).astype(np.float32)
    c = (rng.integers(0, 6, size=(256, 256)) / 5.0).astype(np.float32)
    c[64:192, 64:192] = e[64:192, 64:192]  # shared survivors
    _check(r2, dev, e, c, 300, "quantised")
    _check(r2, dev, e, c, 100000, "quantised, every point")
    g1 = rng.standard_normal((512, 256)).astype(np.float32)
    g2 = rng.standard_normal((512, 256)).astype(np.float32)
    _check(r2, dev, g1, g2, 3000, "gaussian, non-square", patch=32)
    _check(r2, dev, g1, np.full_like(g1, 2.5), 3000, "flat corner map", patch=32)
    _check(r2, dev, g1, g1.copy(), 3000, "same map twice", patch=32)


def test_union_pipeline_runs_and_describes_every_point():
    r2, dev = _gpu()
    a, b, _ = make_pair(0, 1)
    pc, det, dp, mp = r2.defaults()
    det.max_keypoints = 500
    pipe = r2.PairPipeline(256, 256, pc, det, dp, mp, union=True)
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    pipe.run(ta, tb)
    torch.cuda.synchronize()
    # the pipeline's detection equals the union of its own FP32 moment maps
    ref_pts, _ = detect.detect_union(pipe.a.M.cpu().numpy(), pipe.a.m.cpu().numpy(),
                                     oracle.DetectParams(max_keypoints=500), dtype=np.float32)
    nk = int(pipe.a.nk.item())
    assert nk == len(ref_pts) and np.array_equal(pipe.a.kpts[:nk, :2].cpu().numpy(), ref_pts)
    assert int(pipe.a.nd.item()) >= nk
