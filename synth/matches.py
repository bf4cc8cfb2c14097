"""Synthetic putative-match sets for the outlier-removal stage.

A match set is what the matcher hands on: two keypoint tables (rows x, y,
score) and a list of (keypoint in A, keypoint in B) pairs.  Here a fraction of
the pairs are planted as correct -- B's point is A's point moved by a known
rotation about the image centre plus a translation, rounded to the pixel grid
as a detector would report it -- and the rest pair A points with unrelated B
points, as wrong matches do.  The uniform 32-bit words that a RANSAC run
consumes are drawn here too, so both implementations receive the same draws.
Every draw comes from numpy PCG64 streams of one seed.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["planted_matches", "sample_words"]


def _rng(seed: int, salt: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, salt])))


def sample_words(seed: int, n_hyp: int) -> np.ndarray:
    """(n_hyp, 2) uniform uint32 words."""
    return _rng(seed, 1).integers(0, 2 ** 32, (n_hyp, 2), dtype=np.uint64).astype(np.uint32)


def planted_matches(seed: int, n_in: int, n_out: int, size: int = 1024, phi: float | None = None,
                    t: tuple | None = None, extra_kpts: int = 0, dup_a: int = 0):
    """A planted match set.

    Returns kpts_a, kpts_b (int32 [K, 3]: x, y, score bits = 0), matches
    (int32 [n_in + n_out, 3]: kp_a, kp_b, 0), truth (bool [N], planted as
    correct) and gt = {"phi", "t", "size"}.  Keypoint tables hold the matched
    points in shuffled rows plus `extra_kpts` unmatched rows each.  `dup_a`
    wrong matches reuse the A point of another match (coincident samples).
    """
    rng = _rng(seed, 0)
    if phi is None:
        phi = float(rng.uniform(0.0, 2.0 * math.pi))
    if t is None:
        t = (float(rng.uniform(-64, 64)), float(rng.uniform(-64, 64)))
    n = n_in + n_out
    c = (size - 1) / 2.0
    ca, sa = math.cos(phi), math.sin(phi)

    def warp(p):
        dx, dy = p[0] - c, p[1] - c
        return (ca * dx - sa * dy + c + t[0], sa * dx + ca * dy + c + t[1])

    pa = np.empty((n, 2), np.int64)
    pb = np.empty((n, 2), np.int64)
    truth = np.zeros(n, bool)
    order = rng.permutation(n)
    for k in range(n):
        planted = k < n_in
        while True:
            p = rng.integers(0, size, 2)
            if planted:
                u, v = warp(p)
                q = np.array([int(round(u)), int(round(v))])
                if 0 <= q[0] < size and 0 <= q[1] < size:
                    break
            else:
                q = rng.integers(0, size, 2)
                u, v = warp(p)
                if math.hypot(q[0] - u, q[1] - v) > 10.0:
                    break
        pa[order[k]] = p
        pb[order[k]] = q
        truth[order[k]] = planted
    if dup_a:
        wrong = np.nonzero(~truth)[0]
        for i in wrong[:dup_a]:
            pa[i] = pa[(i + 1) % n]
    ka_rows = rng.permutation(n + extra_kpts)
    kb_rows = rng.permutation(n + extra_kpts)
    kpts_a = np.zeros((n + extra_kpts, 3), np.int32)
    kpts_b = np.zeros((n + extra_kpts, 3), np.int32)
    kpts_a[:, :2] = rng.integers(0, size, (n + extra_kpts, 2))
    kpts_b[:, :2] = rng.integers(0, size, (n + extra_kpts, 2))
    kpts_a[ka_rows[:n], :2] = pa
    kpts_b[kb_rows[:n], :2] = pb
    matches = np.zeros((n, 3), np.int32)
    matches[:, 0] = ka_rows[:n]
    matches[:, 1] = kb_rows[:n]
    return kpts_a, kpts_b, matches, truth, {"phi": phi, "t": t, "size": size}
