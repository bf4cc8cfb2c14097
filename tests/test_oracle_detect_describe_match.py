"""Pins of the oracle's FAST detector, dominant-index descriptor and matcher.

Pins: hand-built corner / edge maps, pure-Python brute force on tiny inputs,
full sorts, the paper's worked histogram example (tests/golden), count
invariants and the exact 90 degree grid law of the descriptor.
"""
import json
import os

import numpy as np
import pytest

from oracle import DetectParams, DescParams, MatchParams
from oracle import detect as dt
from oracle import describe as ds
from oracle import match as mt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- detection

def test_single_bright_pixel_is_a_corner_and_edge_is_not():
    d = np.zeros((21, 21))
    d[10, 10] = 1.0
    sc = dt.fast_scores(d)
    assert sc[10, 10] == 1.0
    assert (dt.nms(sc, 0.001)).sum() == 1
    e = np.zeros((24, 24))
    e[:, 12:] = 1.0
    sc = dt.fast_scores(e)
    assert np.all(sc[3:-3, 3:-3] <= 0.0)


def test_corner_of_a_square_is_detected():
    d = np.zeros((32, 32))
    d[10:, 10:] = 1.0   # the pixel (10, 10) sees 5 bright circle pixels, 11 dark
    sc = dt.fast_scores(d)
    assert sc[10, 10] > 0.5
    assert sc[20, 20] <= 0.0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_fast_scores_match_bruteforce(dtype):
    rng = np.random.default_rng(10)
    d = rng.uniform(0, 1, size=(17, 19)).astype(dtype)
    sc = dt.fast_scores(d)
    assert sc.dtype == dtype
    for y in range(17):
        for x in range(19):
            if 3 <= y < 14 and 3 <= x < 16:
                assert sc[y, x] == dt.fast_score_bruteforce(d, y, x)
            else:
                assert sc[y, x] == 0


def _nms_bruteforce(score, t):
    h, w = score.shape
    keep = np.zeros_like(score, dtype=bool)
    for y in range(h):
        for x in range(w):
            if not score[y, x] > t:
                continue
            ok = True
            for yy in range(max(0, y - 1), min(h, y + 2)):
                for xx in range(max(0, x - 1), min(w, x + 2)):
                    if (yy, xx) == (y, x) or not score[yy, xx] > t:
                        continue
                    if score[yy, xx] > score[y, x] or (score[yy, xx] == score[y, x] and yy * w + xx < y * w + x):
                        ok = False
            keep[y, x] = ok
    return keep


def test_nms_matches_bruteforce_with_ties():
    rng = np.random.default_rng(11)
    s = rng.integers(0, 4, size=(15, 13)).astype(np.float32) / 4.0  # many exact ties
    assert np.array_equal(dt.nms(s, 0.1), _nms_bruteforce(s, 0.1))


def test_top_k_is_a_full_sort_prefix():
    rng = np.random.default_rng(12)
    h, w = 40, 30
    s = rng.integers(1, 50, size=(h, w)).astype(np.float32) / 50.0
    keep = rng.uniform(size=(h, w)) < 0.3
    pts, sc = dt.top_k(s, keep, 25)
    items = sorted(((-float(s[y, x]), y * w + x) for y in range(h) for x in range(w) if keep[y, x]))[:25]
    assert [(int(p[1]) * w + int(p[0])) for p in pts] == [r for _, r in items]
    assert np.array_equal(sc, np.array([-v for v, _ in items], dtype=np.float32))


def test_border_mask_keeps_exactly_full_patches():
    m = dt.border_mask(200, 180, 96)
    ys, xs = np.nonzero(m)
    assert ys.min() == 48 and ys.max() == 200 - 48 and xs.min() == 48 and xs.max() == 180 - 48


def test_flat_map_has_no_keypoints():
    pts, sc = dt.detect(np.full((128, 128), 3.0), DetectParams(max_keypoints=10))
    assert pts.shape == (0, 2)


# ---------------------------------------------------------------- description

def _union_by_sets(d_edge, d_corner, p, dtype):
    """The union from two separate single-map detections (every survivor, K unbounded): a dict
    keyed by pixel keeps the larger score, then one sort by (score desc, raster asc)."""
    big = DetectParams(fast_threshold=p.fast_threshold, max_keypoints=10 ** 9, patch_size=p.patch_size)
    best = {}
    for d in (d_edge, d_corner):
        pts, sc = dt.detect(d, big, dtype=dtype)
        for (x, y), s in zip(pts.tolist(), sc.tolist()):
            best[(x, y)] = max(best.get((x, y), -1.0), s)
    w = np.shape(d_edge)[1]
    order = sorted(best, key=lambda q: (-best[q], q[1] * w + q[0]))[: p.max_keypoints]
    return order, [best[q] for q in order]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_union_detector_equals_merged_single_map_detections(dtype):
    rng = np.random.default_rng(21)
    for k in (7, 60, 10 ** 6):
        e = np.round(rng.uniform(0, 1, size=(120, 140)) * 16)  # coarse values: tied scores everywhere
        c = np.round(rng.uniform(0, 1, size=(120, 140)) * 16)
        c[40:80, 50:90] = e[40:80, 50:90]  # both maps agree here: shared pixels
        p = DetectParams(max_keypoints=k, patch_size=20)
        pts, sc = dt.detect_union(e, c, p, dtype=dtype)
        ref_pts, ref_sc = _union_by_sets(e, c, p, dtype)
        assert [tuple(q) for q in pts.tolist()] == ref_pts
        assert np.array_equal(np.asarray(sc, dtype), np.asarray(ref_sc, dtype))
        shared = set(map(tuple, dt.detect(e, p, dtype)[0].tolist())) & set(map(tuple, dt.detect(c, p, dtype)[0].tolist()))
        assert len(pts) == min(k, len(set(ref_pts)))
    assert shared  # the agreeing region yields pixels kept on both maps


def test_union_detector_special_cases():
    rng = np.random.default_rng(22)
    e = rng.uniform(0, 1, size=(100, 100))
    c = rng.uniform(0, 1, size=(100, 100))
    p = DetectParams(max_keypoints=300, patch_size=20)
    # a flat corner map adds nothing
    pe, se = dt.detect(e, p)
    pu, su = dt.detect_union(e, np.full_like(e, 3.0), p)
    assert np.array_equal(pe, pu) and np.array_equal(se, su)
    # the union does not depend on which map is which
    a = dt.detect_union(e, c, p)
    b = dt.detect_union(c, e, p)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # a map with itself is the single-map detection
    pu, su = dt.detect_union(e, e, p)
    assert np.array_equal(pe, pu) and np.array_equal(se, su)


def test_paper_worked_histogram_example():
    g = json.load(open(os.path.join(GOLDEN, "paper_histogram_example.json")))
    p = DescParams(patch_size=36, grid=6, n_orient=g["n_orient"])
    h1 = np.array(g["hist_initial_layer_1"])
    h2 = np.array(g["hist_initial_layer_2"])
    assert h1.sum() == g["patch_pixels"] == 36 * 36
    s1, s21, two1 = ds.dominant(h1, p)
    s2, s22, two2 = ds.dominant(h2, p)
    assert s1 + 1 == g["dominant_index_one_based_layer_1"]
    assert s2 + 1 == g["dominant_index_one_based_layer_2"]
    assert list(ds.recode_histogram(h1, s1)) == g["recoded_hist"]
    assert list(ds.recode_histogram(h2, s2)) == g["recoded_hist"]
    assert two1 == g["second_descriptor"] and two2 == g["second_descriptor"]
    # Eq. 2 with the second layer as the initial one (s = 2, one-based): 2 -> 1, 4 -> 3
    for before, after in g["pointwise_layer1_to_layer2_one_based"]:
        assert ds.recode_mim(np.array([before]), 2, 6)[0] == after
    # Eq. 2 (one-based values, one-based s) equals the 0-based cyclic shift used by recode_histogram
    for s in range(1, 7):
        for v in range(1, 7):
            assert ds.recode_mim(np.array([v]), s, 6)[0] - 1 == (v - s) % 6


def test_paper_example_as_a_real_patch_descriptor():
    """Build a 36x36 MIM patch with the example's histogram; relabelling the
    initial layer (MIM - 1 mod N_o) leaves the descriptor unchanged."""
    g = json.load(open(os.path.join(GOLDEN, "paper_histogram_example.json")))
    p = DescParams(patch_size=36, grid=6, n_orient=6)
    rng = np.random.default_rng(13)
    vals = np.repeat(np.arange(6), g["hist_initial_layer_1"])
    rng.shuffle(vals)
    mim = np.zeros((60, 60), dtype=np.uint8)
    mim[12:48, 12:48] = vals.reshape(36, 36)
    kp = np.array([[30, 30]])
    c1, _, sh1 = ds.describe(mim, kp, p)
    mim2 = ((mim.astype(int) - 1) % 6).astype(np.uint8)
    c2, _, sh2 = ds.describe(mim2, kp, p)
    assert c1.shape == (1, 216)
    assert np.array_equal(c1, c2)
    assert sh1[0] == 2 and sh2[0] == 1
    assert list(c1.reshape(36, 6).sum(axis=0)) == g["recoded_hist"]


def test_counts_sum_to_patch_and_cells():
    rng = np.random.default_rng(14)
    mim = rng.integers(0, 6, size=(200, 210)).astype(np.uint8)
    kp = np.array([[60, 70], [100, 150], [48, 48], [162, 152]])
    c, kpi, sh = ds.describe(mim, kp, DescParams())
    assert np.all(c.astype(int).sum(axis=1) == 96 * 96)
    assert np.all(c.reshape(-1, 36, 6).astype(int).sum(axis=2) == 256)
    assert list(kpi[:4]) == [0, 1, 2, 3]


def test_second_descriptor_rule_is_exact_at_80_percent():
    p = DescParams()
    assert ds.dominant(np.array([0, 500, 400, 0, 0, 0]), p) == (1, 2, True)     # exactly 0.8
    assert ds.dominant(np.array([0, 500, 399, 0, 0, 0]), p) == (1, 2, False)
    assert ds.dominant(np.array([7, 3, 7, 0, 0, 0]), p) == (0, 2, True)         # tie -> lowest index


def test_descriptor_rot90_grid_law():
    """For a keypoint (x, y) of f, the descriptor of rot90(f) taken at
    (x', y') = (y, W - x) is the original with its cell grid rotated:
    desc'[ci][cj][b] = desc[cj][G-1-ci][b] (MIM values shifted by N_o/2)."""
    rng = np.random.default_rng(15)
    n = 160
    mim = rng.integers(0, 6, size=(n, n))
    mim[mim == 5] = 2  # make histograms uneven so dominant indices are untied
    mim = mim.astype(np.uint8)
    rmim = ((np.rot90(mim).astype(int) + 3) % 6).astype(np.uint8)
    p = DescParams()
    checked = 0
    for (x, y) in [(60, 70), (80, 80), (100, 64), (70, 100)]:
        c, _, _ = ds.describe(mim, np.array([[x, y]]), p)
        hist = c[0].reshape(36, 6).sum(axis=0)
        if np.sort(hist)[-1] == np.sort(hist)[-2]:
            continue
        cr, _, _ = ds.describe(rmim, np.array([[y, n - x]]), p)
        a = c[0].reshape(6, 6, 6)
        b = cr[0].reshape(6, 6, 6)
        for ci in range(6):
            for cj in range(6):
                assert np.array_equal(b[ci, cj], a[cj, 5 - ci])
        checked += 1
    assert checked >= 3


def test_ring_rows_reproduce_the_paper_example():
    """Section 3's example: the ring's second MIM (initial layer 2) has the
    histogram printed in the paper, and RIFT2's recoded histogram is the ring
    member whose initial layer is the dominant index."""
    g = json.load(open(os.path.join(GOLDEN, "paper_histogram_example.json")))
    p = DescParams(patch_size=36, grid=6, n_orient=6)
    rng = np.random.default_rng(16)
    vals = np.repeat(np.arange(6), g["hist_initial_layer_1"])
    rng.shuffle(vals)
    mim = np.zeros((60, 60), dtype=np.uint8)
    mim[12:48, 12:48] = vals.reshape(36, 36)
    kp = np.array([[30, 30]])
    ring, kpi, om = ds.describe_ring(mim, kp, p)
    assert ring.shape == (6, 216) and list(kpi) == [0] * 6 and list(om) == list(range(6))
    hists = ring.reshape(6, 36, 6).astype(int).sum(axis=1)
    assert list(hists[0]) == g["hist_initial_layer_1"]
    assert list(hists[1]) == g["hist_initial_layer_2"]
    # relabelling the MIM directly (layer 2 first: value v -> v - 1 mod 6) gives ring row 1
    plain2, _, _ = ds.describe_plain(((mim.astype(int) - 1) % 6).astype(np.uint8), kp, p)
    assert np.array_equal(plain2[0], ring[1])
    rift2, _, sh = ds.describe(mim, kp, p)
    assert sh[0] == g["dominant_index_one_based_layer_1"] - 1
    assert np.array_equal(rift2[0], ring[sh[0]])
    assert list(hists[sh[0]]) == g["recoded_hist"]


def test_ring_contains_every_rift2_row_and_sums_to_the_patch():
    rng = np.random.default_rng(17)
    mim = rng.integers(0, 6, size=(200, 210)).astype(np.uint8)
    kp = np.array([[60, 70], [100, 150], [48, 48], [162, 152]])
    ring, kpi, om = ds.describe_ring(mim, kp, DescParams())
    plain, pk, _ = ds.describe_plain(mim, kp, DescParams())
    rift2, rk, sh = ds.describe(mim, kp, DescParams())
    assert ring.shape == (24, 216) and list(kpi) == [k for k in range(4) for _ in range(6)]
    assert np.array_equal(plain, ring[0::6]) and list(pk) == [0, 1, 2, 3]
    assert np.all(ring.astype(int).sum(axis=1) == 96 * 96)
    for row, k, s in zip(rift2, rk, sh):
        assert np.array_equal(row, ring[6 * k + s])
    # each ring row is a per-cell cyclic permutation of the plain row
    for k in range(4):
        cells = plain[k].reshape(36, 6).astype(int)
        for w in range(6):
            assert np.array_equal(ring[6 * k + w].reshape(36, 6), np.roll(cells, -w, axis=1))


def test_ring_rows_follow_a_rot90_rotation():
    """Under an exact 90-degree rotation the MIM values shift by N_o/2, so the
    rotated image's plain descriptor is the original ring row N_o/2 with the
    cell grid rotated (the ring absorbs the value shift, not the grid)."""
    rng = np.random.default_rng(18)
    n = 160
    mim = rng.integers(0, 6, size=(n, n)).astype(np.uint8)
    rmim = ((np.rot90(mim).astype(int) + 3) % 6).astype(np.uint8)
    p = DescParams()
    for (x, y) in [(60, 70), (80, 80), (100, 64)]:
        ring, _, _ = ds.describe_ring(mim, np.array([[x, y]]), p)
        pr, _, _ = ds.describe_plain(rmim, np.array([[y, n - x]]), p)
        a = ring[3].reshape(6, 6, 6)
        b = pr[0].reshape(6, 6, 6)
        for ci in range(6):
            for cj in range(6):
                assert np.array_equal(b[ci, cj], a[cj, 5 - ci])


# ---------------------------------------------------------------- matching

def _random_descriptors(rng, n_kp, d=216, dup=0.3):
    base = rng.integers(0, 40, size=(n_kp, d))
    rows = [base]
    kp = list(range(n_kp))
    extra = [i for i in range(n_kp) if rng.uniform() < dup]
    if extra:
        rows.append(np.roll(base[extra], 6, axis=1))
        kp += extra
    return np.concatenate(rows).astype(np.uint16), np.array(kp, dtype=np.int32)


def test_match_equals_pure_python_bruteforce():
    rng = np.random.default_rng(16)
    ca, ka = _random_descriptors(rng, 25, d=24)
    cb, kb = _random_descriptors(rng, 30, d=24)
    # plant near-duplicates so that some rows pass the ratio test
    cb[:10] = ca[:10] + rng.integers(0, 2, size=(10, 24))
    got = mt.match(ca, ka, cb, kb, MatchParams())
    ref = mt.match_bruteforce(ca, ka, cb, kb, MatchParams())
    assert list(got[0]) == ref[0] and list(got[1]) == ref[1]
    assert np.allclose(got[2], ref[2], rtol=1e-12, atol=1e-15)
    assert len(ref[0]) >= 5


def test_mutual_match_equals_bruteforce_and_is_a_subset():
    """Mutual mode against the pure-Python brute force (reverse nearest neighbour over all A rows),
    at several chunk sizes of the vectorised oracle; its matches are a subset of the plain mode's."""
    rng = np.random.default_rng(26)
    for trial in range(4):
        ca, ka = _random_descriptors(rng, 30, d=24)
        cb, kb = _random_descriptors(rng, 28, d=24)
        cb[:12] = ca[:12] + rng.integers(0, 2, size=(12, 24))
        # a B row that is the nearest of two A keypoints' rows: only one of them can be mutual
        cb[12] = ca[13]
        ca[14] = ca[13] + rng.integers(0, 2, size=24)
        pm = MatchParams(mutual=True)
        ref = mt.match_bruteforce(ca, ka, cb, kb, pm)
        for chunk in (7, 2048):
            got = mt.match(ca, ka, cb, kb, pm, chunk=chunk)
            assert list(got[0]) == ref[0] and list(got[1]) == ref[1]
            assert np.allclose(got[2], ref[2], rtol=1e-12, atol=1e-15)
        plain = mt.match(ca, ka, cb, kb, MatchParams())
        pairs = set(zip(plain[0].tolist(), plain[1].tolist()))
        assert set(zip(ref[0], ref[1])) <= pairs
        assert len(ref[0]) >= 3


def test_mutual_mode_rejects_a_one_sided_nearest_neighbour():
    """Hand-built: B's only row is nearest to both A rows, and the ratio test passes for both
    (no second B keypoint exists... so a second B keypoint far away); the mutual check keeps only
    the A keypoint that B's row itself picks."""
    e = np.eye(8, dtype=np.uint16) * 10
    ca = np.stack([e[0] + e[1] // 10, e[0] + 2 * (e[2] // 10)])  # A0 closer to B0 than A1 is
    cb = np.stack([e[0], e[5]])
    ka = np.array([0, 1])
    kb = np.array([0, 1])
    plain = mt.match(ca, ka, cb, kb, MatchParams())
    mutual = mt.match(ca, ka, cb, kb, MatchParams(mutual=True))
    assert list(plain[0]) == [0, 1] and list(plain[1]) == [0, 0]
    assert list(mutual[0]) == [0] and list(mutual[1]) == [0]


def test_match_float32_agrees_with_float64_away_from_ties():
    rng = np.random.default_rng(17)
    ca, ka = _random_descriptors(rng, 200)
    cb, kb = _random_descriptors(rng, 180)
    cb[:50] = ca[:50]
    a64 = mt.match(ca, ka, cb, kb, dtype=np.float64)
    a32 = mt.match(ca, ka, cb, kb, dtype=np.float32)
    assert list(a64[0]) == list(a32[0]) and list(a64[1]) == list(a32[1])


def test_exact_dots_are_exact():
    rng = np.random.default_rng(18)
    c = rng.integers(0, 257, size=(6, 216))
    d64 = c.astype(np.float64) @ c.astype(np.float64).T
    d_int = c.astype(np.int64) @ c.astype(np.int64).T
    assert np.array_equal(d64.astype(np.int64), d_int)


def test_ring_matching_equals_bruteforce_and_recovers_rotated_values():
    """Template rows against reference ring rows: the matcher equals pure-Python
    brute force, and a template whose MIM values are shifted by omega (a
    rotation by omega pi / N_o in the value sense) finds its reference keypoint
    through ring row omega."""
    rng = np.random.default_rng(19)
    n_kp, cells, no = 20, 4, 6
    base = rng.integers(0, 30, size=(n_kp, cells, no))
    ring = np.stack([np.roll(base[k], -w, axis=1).ravel() for k in range(n_kp) for w in range(no)]).astype(np.uint16)
    kr = np.repeat(np.arange(n_kp), no).astype(np.int32)
    shift = rng.integers(0, no, size=n_kp)
    tmpl = np.stack([np.roll(base[k], -shift[k], axis=1).ravel() for k in range(n_kp)])
    tmpl = (tmpl + rng.integers(0, 2, size=tmpl.shape)).astype(np.uint16)
    kt = np.arange(n_kp, dtype=np.int32)
    got = mt.match(tmpl, kt, ring, kr, MatchParams())
    ref = mt.match_bruteforce(tmpl, kt, ring, kr, MatchParams())
    assert list(got[0]) == ref[0] and list(got[1]) == ref[1]
    assert len(ref[0]) >= 15 and all(a == b for a, b in zip(ref[0], ref[1]))


# ---------------------------------------------------------------- grid turned by the dominant index

def test_turned_grid_without_turn_is_the_axis_aligned_descriptor():
    """When every dominant index is 0 the grid is not turned, and each row equals the axis-aligned
    descriptor's row."""
    rng = np.random.default_rng(23)
    mim = rng.integers(0, 6, size=(220, 240))
    mim[rng.uniform(size=mim.shape) < 0.6] = 0  # value 0 dominates every patch, no second peak
    mim = mim.astype(np.uint8)
    kp = np.array([[60, 70], [120, 110], [48, 48], [192, 172], [100, 150]])
    c, k, sh = ds.describe_rotated(mim, kp, DescParams())
    c0, k0, sh0 = ds.describe(mim, kp, DescParams())
    assert list(sh) == [0] * 5 and list(sh0) == [0] * 5
    assert np.array_equal(c, c0) and np.array_equal(k, k0)


def test_turned_grid_follows_rot90_up_to_a_half_turn():
    """rot90 turns the image a quarter turn counter-clockwise and raises MIM values by N_o/2; the
    keypoint (x, y) moves to (y, W - x) (the grid's centre is the pixel corner).  Its rows are then
    identical, or -- when s + N_o/2 wraps past N_o, the direction being known only modulo pi -- the
    same with the cell grid turned by pi."""
    rng = np.random.default_rng(24)
    n, no = 260, 6
    mim = rng.integers(0, 6, size=(n, n))
    mim[mim == 5] = 2
    mim[(mim == 4) & (rng.uniform(size=mim.shape) < 0.5)] = 1  # uneven histograms: untied peaks
    corner = mim[140:, 140:]
    corner[rng.uniform(size=corner.shape) < 0.3] = 4  # a region whose dominant index wraps
    mim = mim.astype(np.uint8)
    rmim = ((np.rot90(mim).astype(int) + no // 2) % no).astype(np.uint8)
    p = DescParams()
    seen = {False: 0, True: 0}
    for x, y in [(100, 110), (130, 100), (150, 100), (110, 125), (200, 200), (190, 210), (215, 185)]:
        hist = ds.disc_histogram(mim, x, y, p)
        top = np.sort(hist)[::-1]
        if top[0] == top[1] or top[1] == top[2]:
            continue
        c, k, sh = ds.describe_rotated(mim, np.array([[x, y]]), p)
        cr, kr, shr = ds.describe_rotated(rmim, np.array([[y, n - x]]), p)
        assert len(c) == len(cr) and list(shr) == [(s + no // 2) % no for s in sh]
        for row, rrow, s in zip(c, cr, sh):
            wrap = s + no // 2 >= no
            a = row.reshape(6, 6, no)
            b = rrow.reshape(6, 6, no)
            assert np.array_equal(b, a[::-1, ::-1] if wrap else a)
            seen[wrap] += 1
    assert seen[False] >= 1 and seen[True] >= 1


def test_turned_grid_counts_and_rotation_table():
    rng = np.random.default_rng(25)
    mim = rng.integers(0, 6, size=(300, 280)).astype(np.uint8)
    kp = np.array([[140, 150], [100, 200], [50, 50], [260, 250]])
    c, k, sh = ds.describe_rotated(mim, kp, DescParams())
    sums = c.astype(int).sum(axis=1)
    for row, kk in enumerate(k):
        x, y = kp[kk]
        interior = min(x, y, 280 - 1 - x, 300 - 1 - y) >= 68  # the turned square reaches P / sqrt(2)
        assert sums[row] == 96 * 96 if interior else sums[row] <= 96 * 96
    assert sums.min() < 96 * 96  # a corner keypoint loses samples outside the image
    for no in (6, 8):
        t = ds.rotation_table(no)
        assert t[0] == (65536, 0) and t[no // 2] == (0, 65536)
        for cq, sq in t:
            assert abs(cq * cq + sq * sq - 65536 ** 2) < 2 * 65536
