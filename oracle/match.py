"""Brute-force nearest-neighbour descriptor matching (Section 4, Experiments).

The paper matches every method by brute force with the nearest feature
distance.  Readings where it is silent:
* distance = Euclidean distance of the L2-normalised count vectors,
  d^2(i, j) = 2 - 2 <c_i, c_j> / (|c_i| |c_j|), with the dot product exact
  (integer counts);
* j1 = nearest B row (ties -> lowest row); j2 = nearest B row that belongs to a
  different B keypoint than j1 (a keypoint has at most two rows);
* accept row i iff d^2(i, j1) < r^2 d^2(i, j2) with r = 0.9; no j2 -> reject;
* mutual mode (off by default; a mutual nearest-neighbour check as a stricter
  form of the nearest-distance rule): row i with nearest B row j1 is kept
  only if the nearest A row of j1 (the smallest argmin over all A rows of the
  same d^2 matrix, ties -> lowest row) belongs to row i's A keypoint;
* each A keypoint keeps its accepted row with the smallest d^2 (ties -> lower
  row); the result is sorted by A keypoint.

`dtype=np.float32` evaluates the distance exactly as the GPU does:
ia = fl(1 / fl(sqrt(|c|^2))), t = fl(fl(dot * ia_i) * ib_j), d^2 = fl(2 - 2 t),
test d1^2 < fl(r^2 * d2^2).
"""
from __future__ import annotations

import numpy as np

from .params import MatchParams

__all__ = ["inv_norms", "distances", "match", "match_bruteforce"]


def inv_norms(counts: np.ndarray, dtype=np.float64) -> np.ndarray:
    n2 = (counts.astype(np.int64) ** 2).sum(axis=1)
    if dtype == np.float32:
        return (np.float32(1.0) / np.sqrt(n2.astype(np.float32))).astype(np.float32)
    return 1.0 / np.sqrt(n2.astype(np.float64))


def distances(ca: np.ndarray, cb: np.ndarray, dtype=np.float64) -> np.ndarray:
    """Squared distances (n_a, n_b) of normalised count vectors in `dtype`."""
    dots = ca.astype(np.float64) @ cb.astype(np.float64).T  # exact: integers < 2^53
    ia = inv_norms(ca, dtype)
    ib = inv_norms(cb, dtype)
    if dtype == np.float32:
        t = (dots.astype(np.float32) * ia[:, None]).astype(np.float32)
        t = (t * ib[None, :]).astype(np.float32)
        return (np.float32(2.0) - np.float32(2.0) * t).astype(np.float32)
    return 2.0 - 2.0 * dots * ia[:, None] * ib[None, :]


def _row_decisions(d2: np.ndarray, kp_b: np.ndarray, ratio_sq, dtype):
    """Per A row: (j1, d1, accepted) from a block of squared distances."""
    n_a, n_b = d2.shape
    j1 = np.argmin(d2, axis=1)
    d1 = d2[np.arange(n_a), j1]
    same = kp_b[None, :] == kp_b[j1][:, None]
    masked = np.where(same, np.inf, d2.astype(np.float64)).astype(d2.dtype)
    j2 = np.argmin(masked, axis=1)
    d2nd = masked[np.arange(n_a), j2]
    has2 = np.isfinite(d2nd)
    thr = (dtype(ratio_sq) * d2nd).astype(dtype)
    acc = has2 & (d1 < thr)
    return j1, d1, acc


def match(ca, kp_a, cb, kp_b, p: MatchParams = MatchParams(), dtype=np.float64, chunk: int = 2048):
    """Matches as (kp_a int32, kp_b int32, d2) sorted by kp_a."""
    ca = np.asarray(ca)
    cb = np.asarray(cb)
    kp_a = np.asarray(kp_a, dtype=np.int64)
    kp_b = np.asarray(kp_b, dtype=np.int64)
    n_a = ca.shape[0]
    if n_a == 0 or cb.shape[0] == 0:
        z = np.zeros((0,), np.int32)
        return z, z.copy(), np.zeros((0,), dtype)
    j1s, d1s, accs = [], [], []
    n_b = cb.shape[0]
    col_d = np.full(n_b, np.inf)   # reverse nearest neighbour: column minimum of d^2
    col_i = np.full(n_b, -1, dtype=np.int64)
    for r0 in range(0, n_a, chunk):
        d2 = distances(ca[r0:r0 + chunk], cb, dtype)
        j1, d1, acc = _row_decisions(d2, kp_b, p.ratio_sq, dtype)
        j1s.append(j1)
        d1s.append(d1)
        accs.append(acc)
        if p.mutual:
            ci = np.argmin(d2, axis=0)  # first occurrence: lowest row of this chunk
            cd = d2[ci, np.arange(n_b)].astype(np.float64)
            upd = cd < col_d  # chunks ascend, so ties keep the earlier (lower) row
            col_d = np.where(upd, cd, col_d)
            col_i = np.where(upd, ci + r0, col_i)
    j1 = np.concatenate(j1s)
    d1 = np.concatenate(d1s)
    acc = np.concatenate(accs)
    if p.mutual:
        acc = acc & (kp_a[col_i[j1]] == kp_a)
    best = {}
    for i in range(n_a):
        if not acc[i]:
            continue
        k = int(kp_a[i])
        cur = best.get(k)
        if cur is None or d1[i] < d1[cur]:
            best[k] = i
    keys = sorted(best)
    out_a = np.array(keys, dtype=np.int32)
    out_b = np.array([kp_b[j1[best[k]]] for k in keys], dtype=np.int32)
    out_d = np.array([d1[best[k]] for k in keys], dtype=dtype)
    return out_a, out_b, out_d


def match_bruteforce(ca, kp_a, cb, kp_b, p: MatchParams = MatchParams()):
    """Pure-Python FP64 reference of `match` for tiny inputs (exact integer dots)."""
    import math

    def norm(c):
        return math.sqrt(sum(int(v) * int(v) for v in c))

    na = [norm(c) for c in ca]
    nb = [norm(c) for c in cb]
    rows = []
    for i, c in enumerate(ca):
        ds = []
        for j, e in enumerate(cb):
            dot = sum(int(u) * int(v) for u, v in zip(c, e))
            ds.append(2.0 - 2.0 * dot / (na[i] * nb[j]))
        j1 = min(range(len(ds)), key=lambda j: (ds[j], j))
        others = [j for j in range(len(ds)) if kp_b[j] != kp_b[j1]]
        if not others:
            rows.append(None)
            continue
        j2 = min(others, key=lambda j: (ds[j], j))
        ok = ds[j1] < p.ratio_sq * ds[j2]
        if ok and p.mutual:
            back = []
            for i2, c2 in enumerate(ca):
                dot = sum(int(u) * int(v) for u, v in zip(c2, cb[j1]))
                back.append((2.0 - 2.0 * dot / (na[i2] * nb[j1]), i2))
            ok = int(kp_a[min(back)[1]]) == int(kp_a[i])
        rows.append((j1, ds[j1]) if ok else None)
    best = {}
    for i, r in enumerate(rows):
        if r is None:
            continue
        k = int(kp_a[i])
        if k not in best or r[1] < best[k][1]:
            best[k] = (r[0], r[1])
    keys = sorted(best)
    return ([k for k in keys], [int(kp_b[best[k][0]]) for k in keys], [best[k][1] for k in keys])
