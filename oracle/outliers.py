"""Outlier removal and ground-truth match metrics (test infrastructure only).

The workflow of Fig. 1 ends with a RANSAC-like filter of the putative
matches (Section 1 names RANSAC, Fischler and Bolles 1981, and its variants).
The evaluation of Section 4 instead extracts correct matches with the
ground-truth transformation: a match is correct when its residual is below
3 pixels, a pair is matched successfully when it has at least 10 correct
matches, and the RMSE is taken over the correct matches (20 pixels for a
failed pair).

Transform model: the similarity x' = a x - b y + tx, y' = b x + a y + ty, the
class of the synthetic pairs' ground truth (rotation about the image centre
plus a translation).

RANSAC, as Fischler and Bolles define it:
  1. draw a minimal sample (two matches) per hypothesis and fit the model to
     it exactly;
  2. score the hypothesis by its consensus set: the matches whose squared
     residual is below tau^2;
  3. keep the hypothesis with the largest consensus set (lowest hypothesis
     index on ties);
  4. refit the model to its consensus set by least squares and recompute the
     consensus set, a fixed number of times.

Conventions the GPU path follows by specification (it shares no code with
this module):
  * the random draws are inputs: hypothesis h uses the two uniform 32-bit
    words words[h] and maps each to the match index floor(u * N / 2^32);
  * every floating-point step is one IEEE double operation, in the order
    written here (Python floats and numpy float64 never fuse a multiply and an
    add);
  * keypoint coordinates are integers, so the least-squares sums are exact
    integer sums and their order does not matter.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["sample_indices", "fit_minimal", "fit_lsq", "residual_sq", "ransac", "gt_model", "gt_metrics",
           "match_coords"]


def sample_indices(words, n):
    """Match indices of the sample words: floor(u * n / 2^32) for every uint32 word u."""
    w = np.asarray(words, dtype=np.uint64)
    return ((w * np.uint64(n)) >> np.uint64(32)).astype(np.int64)


def fit_minimal(p1, q1, p2, q2):
    """The similarity that maps p1 -> q1 and p2 -> q2 (exact fit to a minimal sample).

    With d = p2 - p1 and e = q2 - q1 (as complex numbers), (a + ib) = e / d and
    t = q1 - (a + ib) p1.  Returns None when p1 = p2 (no unique transform).
    """
    dx, dy = p2[0] - p1[0], p2[1] - p1[1]
    du, dv = q2[0] - q1[0], q2[1] - q1[1]
    den = dx * dx + dy * dy
    if den == 0:
        return None
    a = float(dx * du + dy * dv) / float(den)
    b = float(dx * dv - dy * du) / float(den)
    x1, y1 = float(p1[0]), float(p1[1])
    tx = float(q1[0]) - (a * x1 - b * y1)
    ty = float(q1[1]) - (b * x1 + a * y1)
    return (a, b, tx, ty)


def residual_sq(model, x, y, u, v):
    """Squared distance between the model's image of (x, y) and (u, v), elementwise in float64."""
    a, b, tx, ty = (np.float64(c) for c in model)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    ex = ((a * x - b * y) + tx) - u
    ey = ((b * x + a * y) + ty) - v
    return ex * ex + ey * ey


def fit_lsq(x, y, u, v):
    """Least-squares similarity of integer correspondences (x, y) -> (u, v).

    Minimising sum |(a + ib) z + t - w|^2 over z = x + iy, w = u + iv gives
    (a + ib) = sum conj(z - zbar)(w - wbar) / sum |z - zbar|^2 and
    t = wbar - (a + ib) zbar.  The sums are taken as exact integers
    (n-scaled to stay integral); returns None for fewer than two distinct
    points.
    """
    x = [int(t) for t in x]
    y = [int(t) for t in y]
    u = [int(t) for t in u]
    v = [int(t) for t in v]
    n = len(x)
    if n < 2:
        return None
    sx, sy, su, sv = sum(x), sum(y), sum(u), sum(v)
    sxx_yy = sum(p * p + q * q for p, q in zip(x, y))
    sxu_yv = sum(p * r + q * s for p, q, r, s in zip(x, y, u, v))
    sxv_yu = sum(p * s - q * r for p, q, r, s in zip(x, y, u, v))
    den = n * sxx_yy - (sx * sx + sy * sy)
    if den == 0:
        return None
    num_a = n * sxu_yv - (sx * su + sy * sv)
    num_b = n * sxv_yu - (sx * sv - sy * su)
    a = float(num_a) / float(den)
    b = float(num_b) / float(den)
    fx, fy, fn = float(sx), float(sy), float(n)
    tx = (float(su) - (a * fx - b * fy)) / fn
    ty = (float(sv) - (b * fx + a * fy)) / fn
    return (a, b, tx, ty)


def match_coords(kpts_a, kpts_b, kp_a, kp_b):
    """Integer coordinates (xa, ya, xb, yb) of matches given as keypoint indices; kpts rows are (x, y, ...)."""
    ka = np.asarray(kpts_a)[np.asarray(kp_a, dtype=np.int64)]
    kb = np.asarray(kpts_b)[np.asarray(kp_b, dtype=np.int64)]
    return (ka[:, 0].astype(np.int64), ka[:, 1].astype(np.int64), kb[:, 0].astype(np.int64),
            kb[:, 1].astype(np.int64))


def ransac(xa, ya, xb, yb, words, threshold=3.0, refine=2):
    """RANSAC over the similarity model (steps 1-4 of the module docstring).

    xa, ya, xb, yb: integer coordinates of the N matches (A point -> B point).
    words: (H, 2) uint32 sample words.  Returns a dict with
      counts  (H,) consensus-set sizes, -1 for a hypothesis without a model;
      best    index of the chosen hypothesis (-1 if none);
      model   (a, b, tx, ty) after refinement, or None;
      mask    (N,) bool consensus set of the final model;
      n_inliers.
    """
    xa, ya, xb, yb = (np.asarray(c, dtype=np.int64) for c in (xa, ya, xb, yb))
    words = np.asarray(words, dtype=np.uint32).reshape(-1, 2)
    n, h_count = len(xa), len(words)
    tau2 = float(threshold) * float(threshold)
    counts = np.full((h_count,), -1, dtype=np.int64)
    empty = {"counts": counts, "best": -1, "model": None, "mask": np.zeros((n,), bool), "n_inliers": 0}
    if n < 2:
        return empty
    idx = sample_indices(words, n)
    best, best_count, best_model = -1, -1, None
    for h in range(h_count):
        i0, i1 = int(idx[h, 0]), int(idx[h, 1])
        m = fit_minimal((xa[i0], ya[i0]), (xb[i0], yb[i0]), (xa[i1], ya[i1]), (xb[i1], yb[i1]))
        if m is None:
            continue
        c = int(np.count_nonzero(residual_sq(m, xa, ya, xb, yb) < tau2))
        counts[h] = c
        if c > best_count:
            best, best_count, best_model = h, c, m
    if best < 0:
        return empty
    model = best_model
    mask = residual_sq(model, xa, ya, xb, yb) < tau2
    for _ in range(refine):
        m = fit_lsq(xa[mask], ya[mask], xb[mask], yb[mask])
        if m is None:
            break
        model = m
        mask = residual_sq(model, xa, ya, xb, yb) < tau2
    return {"counts": counts, "best": best, "model": model, "mask": mask, "n_inliers": int(np.count_nonzero(mask))}


def gt_model(phi, t, size):
    """Similarity of the synthetic pairs' ground truth p_B = R(phi)(p_A - c) + c + t, c the image centre."""
    h, w = size
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    a, b = math.cos(phi), math.sin(phi)
    tx = (cx + float(t[0])) - (a * cx - b * cy)
    ty = (cy + float(t[1])) - (b * cx + a * cy)
    return (a, b, tx, ty)


def gt_metrics(model, xa, ya, xb, yb, threshold=3.0, min_correct=10, rmse_cap=20.0):
    """Section 4 metrics of one pair: correct matches (residual < threshold), their RMSE, success.

    Returns n_correct, sum of the correct matches' squared residuals, rmse
    (rmse_cap for a failed pair) and success (n_correct >= min_correct).
    """
    r2 = residual_sq(model, xa, ya, xb, yb)
    correct = r2 < float(threshold) * float(threshold)
    n = int(np.count_nonzero(correct))
    ssq = float(np.sum(r2[correct])) if n else 0.0
    ok = n >= min_correct
    rmse = math.sqrt(ssq / n) if ok else float(rmse_cap)
    return {"n_correct": n, "sum_sq": ssq, "rmse": rmse, "success": ok, "correct": correct}
