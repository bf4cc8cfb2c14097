"""FAST keypoints on the moment map (Section 2.1; Table 1 settings).

Steps, in the paper's order of detection:
1. normalise the detection map to [0, 1]: Dn = (D - min D) / (max D - min D);
2. FAST segment test on the 16-pixel Bresenham circle of radius 3: a pixel is
   a corner at threshold t when 9 contiguous circle pixels are all brighter
   than p + t or all darker than p - t.  Its score is the largest such t:
   max(max_j min(arc_j) - p, p - min_j max(arc_j)); corner iff score > t
   (t = 0.001, Table 1);
3. 3x3 non-maximum suppression among corners (ties: lower raster index wins);
4. keep points whose full P x P patch lies in the image (P = 96);
5. the K strongest (K = 5000, Table 1) by (score desc, raster asc).

`dtype` selects the arithmetic: float64 for the end-to-end oracle, float32
for the stage that the GPU must reproduce bit for bit (normalisation by a
correctly rounded division, scores by one rounded subtraction).
"""
from __future__ import annotations

import numpy as np

from .params import DetectParams

__all__ = ["CIRCLE", "normalise", "fast_scores", "nms", "border_mask", "top_k", "detect",
           "fast_score_bruteforce", "detect_union"]

# (dx, dy) around the circle, clockwise starting straight above the centre.
CIRCLE = [(0, -3), (1, -3), (2, -2), (3, -1), (3, 0), (3, 1), (2, 2), (1, 3),
          (0, 3), (-1, 3), (-2, 2), (-3, 1), (-3, 0), (-3, -1), (-2, -2), (-1, -3)]
ARC = 9


def normalise(d: np.ndarray, dtype=np.float64):
    """(D - min) / (max - min) in `dtype`; None when the map is flat."""
    d = np.asarray(d, dtype=dtype)
    lo = d.min()
    hi = d.max()
    if not hi > lo:
        return None
    rng = dtype(hi - lo)
    return ((d - lo) / rng).astype(dtype)


def fast_scores(dn: np.ndarray) -> np.ndarray:
    """FAST-9 score at every pixel with a full circle (0 elsewhere)."""
    h, w = dn.shape
    dt = dn.dtype
    score = np.zeros((h, w), dtype=dt)
    if h < 7 or w < 7:
        return score
    core = dn[3:h - 3, 3:w - 3]
    ring = [dn[3 + dy:h - 3 + dy, 3 + dx:w - 3 + dx] for dx, dy in CIRCLE]
    best_lo = None
    best_hi = None
    for j in range(16):
        arc = [ring[(j + i) % 16] for i in range(ARC)]
        lo = arc[0]
        hi = arc[0]
        for a in arc[1:]:
            lo = np.minimum(lo, a)
            hi = np.maximum(hi, a)
        best_lo = lo if best_lo is None else np.maximum(best_lo, lo)
        best_hi = hi if best_hi is None else np.minimum(best_hi, hi)
    bright = (best_lo - core).astype(dt)
    dark = (core - best_hi).astype(dt)
    score[3:h - 3, 3:w - 3] = np.maximum(bright, dark)
    return score


def fast_score_bruteforce(dn: np.ndarray, y: int, x: int) -> float:
    """Largest t for which pixel (y, x) passes the segment test (pure Python)."""
    p = dn[y, x]
    vals = [dn[y + dy, x + dx] for dx, dy in CIRCLE]
    best = None
    for j in range(16):
        arc = [vals[(j + i) % 16] for i in range(ARC)]
        for cand in (min(arc) - p, p - max(arc)):
            cand = dn.dtype.type(cand)
            best = cand if best is None or cand > best else best
    return best


def nms(score: np.ndarray, t: float) -> np.ndarray:
    """Boolean map of corners (score > t) that beat every corner in their 3x3 neighbourhood."""
    h, w = score.shape
    corner = score > t
    keep = corner.copy()
    pad_s = np.full((h + 2, w + 2), -np.inf, dtype=np.float64)
    pad_s[1:-1, 1:-1] = np.where(corner, score, -np.inf)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            nb = pad_s[1 + dy:h + 1 + dy, 1 + dx:w + 1 + dx]
            # the neighbour's raster index is smaller iff it lies earlier in scan order
            nb_earlier = (dy < 0) or (dy == 0 and dx < 0)
            if nb_earlier:
                keep &= score.astype(np.float64) > nb
            else:
                keep &= score.astype(np.float64) >= nb
    return keep


def border_mask(h: int, w: int, patch: int) -> np.ndarray:
    """Pixels whose patch rows/cols [c - P/2, c + P/2 - 1] stay in the image."""
    half = patch // 2
    m = np.zeros((h, w), dtype=bool)
    m[half:h - half + 1, half:w - half + 1] = True
    return m


def top_k(score: np.ndarray, keep: np.ndarray, k: int):
    """K best kept points by (score desc, raster asc) -> int32 (n, 2) [x, y] and scores."""
    h, w = score.shape
    ys, xs = np.nonzero(keep)
    sc = score[ys, xs]
    raster = ys.astype(np.int64) * w + xs
    order = np.lexsort((raster, -sc.astype(np.float64)))[:k]
    pts = np.stack([xs[order], ys[order]], axis=1).astype(np.int32)
    return pts, sc[order]


def detect(d: np.ndarray, p: DetectParams = DetectParams(), dtype=np.float64):
    """Keypoints (x, y) int32 (n, 2) and their scores, strongest first."""
    dn = normalise(d, dtype)
    if dn is None:
        return np.zeros((0, 2), np.int32), np.zeros((0,), dtype)
    sc = fast_scores(dn)
    keep = nms(sc, p.fast_threshold) & border_mask(*dn.shape, p.patch_size)
    return top_k(sc, keep, p.max_keypoints)


def detect_union(d_edge: np.ndarray, d_corner: np.ndarray, p: DetectParams = DetectParams(), dtype=np.float64):
    """RIFT's detector (Section 2.1): FAST on the maximum-moment map (edge features) and on the
    minimum-moment map (corners), steps 1-4 on each map separately, then the union of the two point
    sets -- a pixel found on both keeps the larger score -- and step 5 on the union."""
    h, w = np.shape(d_edge)
    score = np.zeros((h, w), dtype=dtype)
    keep = np.zeros((h, w), dtype=bool)
    border = border_mask(h, w, p.patch_size)
    for d in (d_edge, d_corner):
        dn = normalise(d, dtype)
        if dn is None:
            continue
        sc = fast_scores(dn)
        k = nms(sc, p.fast_threshold) & border
        score = np.where(k & keep, np.maximum(score, sc), np.where(k, sc, score)).astype(dtype)
        keep |= k
    return top_k(score, keep, p.max_keypoints)
