"""Pins of the outlier-removal and ground-truth-metric oracle (oracle/outliers.py).

Each check rests on something other than the oracle's own formulas: complex
arithmetic for the similarity, numpy's least-squares solver, planted inlier
sets, a brute-force consensus count, the synthetic generator's warp, and the
metric definitions of Section 4 on hand-built residuals.
"""
import math

import numpy as np
import pytest

from oracle import outliers as ol


def _apply(model, p):
    a, b, tx, ty = model
    z = complex(p[0], p[1]) * complex(a, b) + complex(tx, ty)
    return z.real, z.imag


def test_minimal_fit_maps_both_points():
    rng = np.random.default_rng(1)
    for _ in range(200):
        p1, p2, q1, q2 = (tuple(int(v) for v in rng.integers(0, 1024, 2)) for _ in range(4))
        m = ol.fit_minimal(p1, q1, p2, q2)
        if p1 == p2:
            assert m is None
            continue
        for p, q in ((p1, q1), (p2, q2)):
            u, v = _apply(m, p)
            assert abs(u - q[0]) < 1e-9 and abs(v - q[1]) < 1e-9


def test_minimal_fit_recovers_known_similarity():
    phi, s = math.radians(37.0), 1.3
    truth = (s * math.cos(phi), s * math.sin(phi), 12.5, -40.25)
    p1, p2 = (100, 200), (640, 30)
    m = ol.fit_minimal(p1, _apply(truth, p1), p2, _apply(truth, p2))
    assert np.allclose(m, truth, rtol=0, atol=1e-12)


def test_lsq_equals_numpy_lstsq():
    rng = np.random.default_rng(2)
    for n in (2, 3, 17, 400):
        x, y, u, v = (rng.integers(0, 4096, n) for _ in range(4))
        m = ol.fit_lsq(x, y, u, v)
        # rows [x, -y, 1, 0] -> u and [y, x, 0, 1] -> v
        A = np.zeros((2 * n, 4))
        A[0::2] = np.stack([x, -y, np.ones(n), np.zeros(n)], 1)
        A[1::2] = np.stack([y, x, np.zeros(n), np.ones(n)], 1)
        rhs = np.empty(2 * n)
        rhs[0::2], rhs[1::2] = u, v
        ref = np.linalg.lstsq(A, rhs, rcond=None)[0]
        assert np.allclose(m, ref, rtol=1e-9, atol=1e-6), (n, m, ref)


def test_lsq_degenerate():
    assert ol.fit_lsq([5], [6], [7], [8]) is None
    assert ol.fit_lsq([5, 5, 5], [6, 6, 6], [1, 2, 3], [4, 5, 6]) is None


def test_residual_known_distances():
    ident = (1.0, 0.0, 0.0, 0.0)
    r2 = ol.residual_sq(ident, [0, 10, 7], [0, 20, 7], [3, 10, 7], [4, 20, 7])
    assert list(r2) == [25.0, 0.0, 0.0]
    # rotation by 90 degrees: (1, 0) -> (0, 1)
    r2 = ol.residual_sq((0.0, 1.0, 0.0, 0.0), [1], [0], [0], [1])
    assert r2[0] == 0.0


def test_sample_indices_bounds():
    assert ol.sample_indices([0], 7)[0] == 0
    assert ol.sample_indices([2 ** 32 - 1], 7)[0] == 6
    w = np.random.default_rng(3).integers(0, 2 ** 32, 100000, dtype=np.uint64)
    idx = ol.sample_indices(w, 13)
    assert idx.min() == 0 and idx.max() == 12
    counts = np.bincount(idx, minlength=13)
    assert counts.min() > 0.9 * len(w) / 13


def _planted(rng, n_in, n_out, truth, size=1024):
    pa = rng.integers(0, size, (n_in + n_out, 2))
    pb = np.empty_like(pa)
    for i, p in enumerate(pa):
        u, v = _apply(truth, p)
        pb[i] = (int(round(u)), int(round(v)))  # rounding error <= 0.71 px
    out = rng.permutation(n_in + n_out)[:n_out]
    for i in out:
        while True:
            q = rng.integers(0, size, 2)
            u, v = _apply(truth, pa[i])
            if math.hypot(q[0] - u, q[1] - v) > 10.0:
                break
        pb[i] = q
    inlier = np.ones(n_in + n_out, bool)
    inlier[out] = False
    return pa[:, 0], pa[:, 1], pb[:, 0], pb[:, 1], inlier


def test_ransac_finds_planted_inliers():
    rng = np.random.default_rng(4)
    phi = math.radians(-71.0)
    truth = (math.cos(phi), math.sin(phi), 300.0, -120.0)
    xa, ya, xb, yb, inlier = _planted(rng, 150, 250, truth)
    words = rng.integers(0, 2 ** 32, (400, 2), dtype=np.uint64).astype(np.uint32)
    res = ol.ransac(xa, ya, xb, yb, words, threshold=3.0, refine=2)
    assert np.array_equal(res["mask"], inlier)
    assert res["n_inliers"] == 150
    # points rounded to integers: rotation to ~1e-4, translation to a fraction of a pixel
    assert np.allclose(res["model"][:2], truth[:2], atol=1e-3)
    assert np.allclose(res["model"][2:], truth[2:], atol=0.2)


def test_ransac_counts_equal_brute_force():
    rng = np.random.default_rng(5)
    n = 120
    xa, ya, xb, yb = (rng.integers(0, 512, n) for _ in range(4))
    words = rng.integers(0, 2 ** 32, (60, 2), dtype=np.uint64).astype(np.uint32)
    res = ol.ransac(xa, ya, xb, yb, words, threshold=25.0, refine=0)
    for h, (w0, w1) in enumerate(words):
        i0, i1 = (int(w0) * n) >> 32, (int(w1) * n) >> 32
        za = [complex(x, y) for x, y in zip(xa, ya)]
        zb = [complex(x, y) for x, y in zip(xb, yb)]
        if za[i0] == za[i1]:
            assert res["counts"][h] == -1
            continue
        k = (zb[i1] - zb[i0]) / (za[i1] - za[i0])
        t = zb[i0] - k * za[i0]
        c = sum(abs(k * p + t - q) < 25.0 for p, q in zip(za, zb))
        assert res["counts"][h] == c, h
    assert res["best"] == int(np.argmax(res["counts"]))


def test_ransac_picks_the_only_clean_sample():
    rng = np.random.default_rng(6)
    truth = (1.0, 0.0, 40.0, 25.0)
    xa, ya, xb, yb, inlier = _planted(rng, 30, 70, truth)
    n = len(xa)
    ins, outs = np.nonzero(inlier)[0], np.nonzero(~inlier)[0]

    def word(i):  # a word whose index is i: floor(u n / 2^32) = i
        return (i * 2 ** 32 + n - 1) // n

    words = np.array([(word(outs[k]), word(outs[k + 1])) for k in range(0, 20, 2)], dtype=np.uint64)
    words = np.insert(words, 7, (word(ins[3]), word(ins[11])), axis=0).astype(np.uint32)
    assert list(ol.sample_indices(words[7], n)) == [ins[3], ins[11]]
    res = ol.ransac(xa, ya, xb, yb, words, threshold=3.0, refine=1)
    assert res["best"] == 7
    assert np.array_equal(res["mask"], inlier)
    # the same clean sample again at a later index: a tie, the lower index wins
    words2 = np.insert(words, 9, words[7], axis=0)
    res = ol.ransac(xa, ya, xb, yb, words2, threshold=3.0, refine=1)
    assert res["counts"][9] == res["counts"][7] and res["best"] == 7


def test_ransac_degenerate_inputs():
    w = np.zeros((5, 2), np.uint32)
    for n in (0, 1):
        res = ol.ransac(np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n), w)
        assert res["best"] == -1 and res["model"] is None and res["n_inliers"] == 0
    res = ol.ransac([3, 3, 3], [4, 4, 4], [1, 2, 3], [5, 6, 7], np.arange(10, dtype=np.uint32).reshape(5, 2) * 10 ** 8)
    assert res["best"] == -1 and list(res["counts"]) == [-1] * 5


def test_gt_model_matches_generator_warp():
    import synth.gen as g

    n = 128
    for phi, tx, ty in ((0.0, 5.0, -3.0), (math.radians(90.0), 0.0, 0.0), (math.radians(33.0), -7.5, 12.25)):
        m = ol.gt_model(phi, (tx, ty), (n, n))
        for px, py in ((40, 50), (64, 60), (80, 90)):
            img = np.zeros((n, n))
            img[py, px] = 1000.0
            b = g._warp_bilinear(img, phi, tx, ty)
            qy, qx = np.unravel_index(np.argmax(b), b.shape)
            u, v = _apply(m, (px, py))
            assert abs(qx - u) <= 0.5 + 1e-9 and abs(qy - v) <= 0.5 + 1e-9, (phi, px, py, qx, qy, u, v)


def test_gt_metrics_definitions():
    ident = (1.0, 0.0, 0.0, 0.0)
    # residuals 0, 1, 2.9, 3 (not correct: strictly below 3), 10
    xa = np.zeros(5, np.int64)
    ya = np.zeros(5, np.int64)
    xb = np.array([0.0, 1.0, 2.9, 3.0, 10.0])
    yb = np.zeros(5)
    m = ol.gt_metrics(ident, xa, ya, xb, yb)
    assert m["n_correct"] == 3 and list(m["correct"]) == [True, True, True, False, False]
    assert m["success"] is False and m["rmse"] == 20.0
    k = 12
    m = ol.gt_metrics(ident, np.zeros(k), np.zeros(k), np.full(k, 2.0), np.zeros(k))
    assert m["n_correct"] == k and m["success"] is True and m["rmse"] == pytest.approx(2.0)
