"""GPU parity of the outlier-removal stage (rift2_ransac, rift2_consensus) against the oracle.

Both sides evaluate every step as one IEEE double operation in the same
order and take the least-squares sums as exact integers, so the bar is
bit-exact: every hypothesis' consensus count, the chosen hypothesis, the
refined model's four doubles, the inlier mask and its size.  The one
floating-point sum (the inliers' squared residuals of rift2_consensus) is
added in a different order on each side and is compared to 1e-12 relative.

Inputs are planted match sets from synth.matches (a known similarity plus
unrelated wrong pairs), with the uniform sample words drawn there as well.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle import outliers as ol  # noqa: E402
from synth.matches import planted_matches, sample_words  # noqa: E402


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_00319_amd as r2

    return r2, torch.device("cuda:0")


def _dev_inputs(dev, ka, kb, m, words, cap=None, n=None):
    cap = max(1, len(m)) if cap is None else cap
    mt = torch.zeros((cap, 3), dtype=torch.int32)
    mt[: len(m)] = torch.from_numpy(np.asarray(m, np.int32).reshape(-1, 3))
    nt = torch.tensor([len(m) if n is None else n], dtype=torch.int32)
    w = torch.from_numpy(np.asarray(words, np.uint32).view(np.int32).reshape(-1, 2).copy())
    return (mt.to(dev), nt.to(dev), torch.from_numpy(np.asarray(ka, np.int32)).to(dev),
            torch.from_numpy(np.asarray(kb, np.int32)).to(dev), w.to(dev))


def _run_gpu(r2, dev, ka, kb, m, words, thr, refine, cap=None):
    mt, nt, kat, kbt, wt = _dev_inputs(dev, ka, kb, m, words, cap)
    result, mask, counts = r2.ransac(mt, nt, kat, kbt, wt, threshold=thr, refine=refine)
    torch.cuda.synchronize()
    return r2.similarity_fields(result), mask.cpu().numpy(), counts.cpu().numpy()


def _run_oracle(ka, kb, m, words, thr, refine):
    m = np.asarray(m).reshape(-1, 3)
    xa, ya, xb, yb = ol.match_coords(ka, kb, m[:, 0], m[:, 1])
    return ol.ransac(xa, ya, xb, yb, words, threshold=thr, refine=refine)


def _assert_same(gpu, ref, n, cap):
    fields, mask, counts = gpu
    assert fields["status"] == 0
    assert fields["n_matches"] == n
    assert np.array_equal(counts, ref["counts"]), np.nonzero(counts != ref["counts"])[0][:10]
    assert fields["best"] == ref["best"]
    if ref["model"] is None:
        assert fields["model"] == (0.0, 0.0, 0.0, 0.0)
    else:
        # bit-exact doubles
        assert np.array_equal(np.array(fields["model"]).view(np.int64), np.array(ref["model"]).view(np.int64)), \
            (fields["model"], ref["model"])
    assert np.array_equal(mask[:n].astype(bool), ref["mask"])
    assert not mask[n:cap].any()
    assert fields["n_inliers"] == ref["n_inliers"]


@pytest.mark.parametrize("seed,n_in,n_out,n_hyp,thr,refine,extra_cap", [
    (1, 30, 70, 64, 3.0, 2, 0),
    (2, 150, 250, 400, 3.0, 2, 13),
    (3, 500, 4500, 4096, 3.0, 2, 0),     # 5000 matches, 4096 hypotheses: the benchmarked shape
    (4, 2, 0, 5, 3.0, 1, 0),
    (5, 40, 600, 1000, 25.0, 0, 100),    # wide threshold: many partial consensus sets
    (6, 100, 157, 77, 1.0, 4, 1),        # threshold 1 px: the rounding of planted points decides
    (7, 1000, 9000, 2051, 3.0, 3, 300),  # ragged capacity, hypotheses not a multiple of 16
    (8, 3000, 57000, 256, 3.0, 16, 7),   # the most refits, each over 59 blocks of refit sums
    (9, 25, 20000, 300, 2.0, 5, 0),      # few inliers among many matches
])
def test_ransac_bitexact_on_planted_sets(seed, n_in, n_out, n_hyp, thr, refine, extra_cap):
    r2, dev = _gpu()
    ka, kb, m, truth, _ = planted_matches(seed, n_in, n_out, extra_kpts=37)
    words = sample_words(seed, n_hyp)
    n = len(m)
    print(f"ransac planted seed {seed}: N={n} H={n_hyp} thr={thr} refine={refine}", flush=True)
    gpu = _run_gpu(r2, dev, ka, kb, m, words, thr, refine, cap=n + extra_cap)
    ref = _run_oracle(ka, kb, m, words, thr, refine)
    _assert_same(gpu, ref, n, n + extra_cap)
    if thr == 3.0 and n_in >= 30 and n_hyp >= 64:
        assert ref["n_inliers"] >= n_in


def test_ransac_ties_go_to_the_lowest_hypothesis():
    r2, dev = _gpu()
    ka, kb, m, truth, _ = planted_matches(11, 60, 140)
    words = sample_words(11, 40)
    words = np.concatenate([words, words[::-1], words[5:9]])  # every count appears at least twice
    gpu = _run_gpu(r2, dev, ka, kb, m, words, 3.0, 2)
    ref = _run_oracle(ka, kb, m, words, 3.0, 2)
    _assert_same(gpu, ref, len(m), len(m))
    c = ref["counts"]
    assert (c == c.max()).sum() >= 2 and ref["best"] == int(np.argmax(c))


def test_ransac_degenerate_inputs():
    r2, dev = _gpu()
    words = sample_words(12, 33)
    ka = np.array([[5, 6, 0], [5, 6, 0], [5, 6, 0]], np.int32)
    kb = np.array([[1, 4, 0], [2, 5, 0], [3, 7, 0]], np.int32)
    for m in (np.zeros((0, 3), np.int32), np.array([[0, 1, 0]], np.int32),
              np.array([[0, 0, 0], [1, 1, 0], [2, 2, 0]], np.int32)):  # none, one, all A points equal
        print(f"ransac degenerate N={len(m)}", flush=True)
        gpu = _run_gpu(r2, dev, ka, kb, m, words, 3.0, 2, cap=8)
        ref = _run_oracle(ka, kb, m, words, 3.0, 2)
        _assert_same(gpu, ref, len(m), 8)
        assert gpu[0]["best"] == -1 and (gpu[2] == -1).all()


def test_ransac_rejects_invalid_match_lists_on_the_device():
    r2, dev = _gpu()
    ka, kb, m, _, _ = planted_matches(13, 20, 20)
    words = sample_words(13, 50)
    bad_index = m.copy()
    bad_index[7, 1] = len(kb) + 5  # keypoint index past the table
    bad_coord = ka.copy()
    bad_coord[m[3, 0], 0] = 9000  # coordinate past 2^13
    for ka_, m_ in ((ka, bad_index), (bad_coord, m)):
        fields, mask, counts = _run_gpu(r2, dev, ka_, kb, m_, words, 3.0, 2)
        assert fields["status"] == 1 and fields["best"] == -1 and fields["n_inliers"] == 0
        assert fields["n_matches"] == 0 and (counts == -1).all() and not mask.any()
    # a valid list afterwards gives the oracle's result again
    _assert_same(_run_gpu(r2, dev, ka, kb, m, words, 3.0, 2), _run_oracle(ka, kb, m, words, 3.0, 2), len(m), len(m))


@pytest.mark.parametrize("seed,n_in,n_out", [(21, 300, 700), (22, 5, 3000), (23, 0, 50)])
def test_consensus_of_ground_truth_equals_oracle_metrics(seed, n_in, n_out):
    r2, dev = _gpu()
    ka, kb, m, truth, gt = planted_matches(seed, n_in, n_out)
    model = ol.gt_model(gt["phi"], gt["t"], (gt["size"], gt["size"]))
    mt, nt, kat, kbt, _ = _dev_inputs(dev, ka, kb, m, np.zeros((1, 2), np.uint32), cap=len(m) + 9)
    md = torch.tensor(model, dtype=torch.float64, device=dev)
    res, mask = r2.consensus(md, mt, nt, kat, kbt, threshold=3.0)
    torch.cuda.synchronize()
    got = r2.consensus_fields(res)
    xa, ya, xb, yb = ol.match_coords(ka, kb, m[:, 0], m[:, 1])
    ref = ol.gt_metrics(model, xa, ya, xb, yb, threshold=3.0)
    mask = mask.cpu().numpy()
    assert got["status"] == 0 and got["n_inliers"] == ref["n_correct"]
    assert np.array_equal(mask[: len(m)].astype(bool), ref["correct"]) and not mask[len(m):].any()
    assert got["sum_sq"] == pytest.approx(ref["sum_sq"], rel=1e-12, abs=0.0)
    assert ref["n_correct"] == n_in  # every planted match is within 0.71 px, every wrong one beyond 10 px


def test_ransac_on_pipeline_matches_agrees_with_the_oracle_pipeline():
    """A shifted, intensity-inverted 256^2 pair through both pipelines: each
    side's RANSAC on its own matches recovers the (7, 4) shift, and the two
    inlier sets agree (the match sets themselves agree to Jaccard > 0.9)."""
    r2, dev = _gpu()
    import synth.gen as g
    from synth import make_pair

    a, _, _ = make_pair(0, 2)
    b = g._warp_bilinear(a.astype(np.float64), 0.0, 7.0, 4.0)
    b = np.rint(np.clip(255 * np.power(np.clip((255 - b) / 255, 0, 1), 0.5), 0, 255)).astype(np.uint8)
    fa, fb, mref = oracle.pipeline.match_pair(a, b, det=oracle.DetectParams(max_keypoints=500))
    pc, detp, dp, mp = r2.defaults()
    detp.max_keypoints = 500
    feats = []
    for img in (a, b):
        fm = r2.filter_mim(torch.from_numpy(img).to(dev), pc)
        kp, nk = r2.detect(fm["M"], detp)
        feats.append((kp, nk) + r2.describe(fm["mim"], kp, nk, dp))
    out, n = r2.match(*feats[0][2:6], *feats[1][2:6], mp)
    words = sample_words(31, 1024)
    wt = torch.from_numpy(words.view(np.int32).copy()).to(dev)
    res, mask, _ = r2.ransac(out, n, feats[0][0], feats[1][0], wt, threshold=3.0, refine=2)
    torch.cuda.synchronize()
    got = r2.similarity_fields(res)
    n = int(n.item())
    ref = ol.ransac(*ol.match_coords(fa["kpts"], fb["kpts"], mref[0], mref[1]), words, 3.0, 2)
    for model in (got["model"], ref["model"]):
        assert abs(model[0] - 1.0) < 1e-3 and abs(model[1]) < 1e-3
        assert abs(model[2] - 7.0) < 0.5 and abs(model[3] - 4.0) < 0.5
    ka, kb = feats[0][0].cpu().numpy(), feats[1][0].cpu().numpy()
    om = out[:n].cpu().numpy()
    mk = mask[:n].cpu().numpy().astype(bool)
    gpu_in = {(tuple(ka[i, :2]), tuple(kb[j, :2])) for (i, j), k in zip(om[:, :2], mk) if k}
    ref_in = {(tuple(fa["kpts"][i]), tuple(fb["kpts"][j])) for i, j, k in zip(mref[0], mref[1], ref["mask"]) if k}
    jac = len(gpu_in & ref_in) / max(1, len(gpu_in | ref_in))
    print(f"pipeline ransac: gpu {got['n_inliers']} inliers of {n}, oracle {ref['n_inliers']} of {len(mref[0])}, "
          f"Jaccard {jac:.4f}", flush=True)
    assert got["n_inliers"] > 100 and jac > 0.9
    assert math.isfinite(got["model"][2])
