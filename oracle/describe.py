"""Dominant-index rotation-invariant MIM descriptor (Sections 2.2 and 3).

For each keypoint (x, y):
1. take the P x P MIM patch, rows y - P/2 .. y + P/2 - 1 and the same for
   columns (P = 96, Table 1);
2. split it into G x G cells (G = 6, Section 2.2) and count, per cell, how
   many pixels carry each MIM value b in 0..N_o-1 -> h[cy][cx][b];
3. the patch histogram Hist[b] = sum over cells; its peak gives the dominant
   index s (Eq. 1; ties -> lowest index);
4. recode every MIM value relative to s (Eq. 2, which in 0-based form is
   MIM_n = (MIM - s) mod N_o); the recoded cell histograms are the
   descriptor, desc[cy][cx][b] = h[cy][cx][(b + s) mod N_o], laid out
   (cy, cx, b) row-major, D = G*G*N_o values;
5. if the second-highest bin s2 (lowest index among ties, s2 != s) reaches
   the dominant ratio of the peak (0.8, Table 1; tested exactly as
   5 Hist[s2] >= 4 Hist[s]) a second descriptor is built with s2 (Section 3,
   last paragraph).

Descriptor values are integer counts; distances use the L2-normalised vector.
Row order: all primary rows in keypoint order, then all secondary rows in
keypoint order.

RIFT's convolution-sequence ring (Section 2.3), the method RIFT2 replaces, is
here as the baseline variant: the template image gets one plain descriptor
per keypoint (the MIM as computed, initial layer 1), the reference image gets
N_o descriptors per keypoint, one per choice of initial layer omega of the
ring.  Taking layer omega as the first relabels every MIM value v as
(v - omega) mod N_o (Section 3's analysis of the ring), so bin b of ring row
omega counts the pixels whose original value is (b + omega) mod N_o.
"""
from __future__ import annotations

import numpy as np

from .params import DescParams

__all__ = ["cell_histograms", "dominant", "recode_histogram", "recode_mim", "describe", "ring_histogram",
           "describe_plain", "describe_ring", "rotation_table", "disc_histogram", "rotated_cell_histograms",
           "describe_rotated"]


def cell_histograms(mim: np.ndarray, x: int, y: int, p: DescParams) -> np.ndarray:
    """h[cy, cx, b] counts of the P x P patch centred (in the [-P/2, P/2) sense) on (x, y)."""
    half = p.patch_size // 2
    patch = mim[y - half:y + half, x - half:x + half].astype(np.int64)
    if patch.shape != (p.patch_size, p.patch_size):
        raise ValueError("patch leaves the image")
    cell = p.patch_size // p.grid
    cy = (np.arange(p.patch_size) // cell)[:, None]
    cx = (np.arange(p.patch_size) // cell)[None, :]
    idx = (cy * p.grid + cx) * p.n_orient + patch
    h = np.bincount(idx.ravel(), minlength=p.grid * p.grid * p.n_orient)
    return h.reshape(p.grid, p.grid, p.n_orient)


def dominant(hist: np.ndarray, p: DescParams):
    """(s, s2, has_second) of a patch histogram (Eq. 1 plus the 80 % rule)."""
    hist = np.asarray(hist, dtype=np.int64)
    s = int(np.argmax(hist))
    rest = hist.copy()
    rest[s] = -1
    s2 = int(np.argmax(rest))
    has2 = p.dominant_den * int(hist[s2]) >= p.dominant_num * int(hist[s])
    return s, s2, bool(has2)


def recode_mim(values: np.ndarray, s: int, n_orient: int) -> np.ndarray:
    """Eq. 2 in the paper's 1-based form: v - s + 1 if v >= s else v + N_o - s + 1."""
    v = np.asarray(values, dtype=np.int64)
    return np.where(v >= s, v - s + 1, v + n_orient - s + 1)


def recode_histogram(h: np.ndarray, s: int) -> np.ndarray:
    """Bins b of the recoded histogram take the count of original bin (b + s) mod N_o."""
    n = h.shape[-1]
    return h[..., (np.arange(n) + s) % n]


def describe(mim: np.ndarray, kpts: np.ndarray, p: DescParams = DescParams()):
    """Descriptors of keypoints `kpts` (n, 2) [x, y] on a 0-based MIM.

    Returns (counts uint16 (rows, D), kp_index int32 (rows,), shift int32 (rows,)).
    """
    prim = []
    sec = []
    for i, (x, y) in enumerate(np.asarray(kpts, dtype=np.int64)):
        h = cell_histograms(mim, int(x), int(y), p)
        hist = h.sum(axis=(0, 1))
        s, s2, has2 = dominant(hist, p)
        prim.append((i, s, recode_histogram(h, s).ravel()))
        if has2:
            sec.append((i, s2, recode_histogram(h, s2).ravel()))
    rows = prim + sec
    d = p.grid * p.grid * p.n_orient
    if not rows:
        return np.zeros((0, d), np.uint16), np.zeros((0,), np.int32), np.zeros((0,), np.int32)
    counts = np.stack([r[2] for r in rows]).astype(np.uint16)
    kp = np.array([r[0] for r in rows], dtype=np.int32)
    sh = np.array([r[1] for r in rows], dtype=np.int32)
    return counts, kp, sh


def ring_histogram(h: np.ndarray, omega: int) -> np.ndarray:
    """Cell histograms of the MIM rebuilt with layer omega (0-based) as the ring's initial layer.

    Every MIM value v becomes (v - omega) mod N_o (Section 3: starting the ring
    one layer later lowers every index by one, cyclically), so new bin b counts
    the pixels whose value was (b + omega) mod N_o.
    """
    n = h.shape[-1]
    out = np.zeros_like(h)
    for v in range(n):
        out[..., (v - omega) % n] += h[..., v]
    return out


def _rows(mim, kpts, p, shifts):
    rows, kp, sh = [], [], []
    for i, (x, y) in enumerate(np.asarray(kpts, dtype=np.int64)):
        h = cell_histograms(mim, int(x), int(y), p)
        for omega in shifts:
            rows.append(ring_histogram(h, omega).ravel())
            kp.append(i)
            sh.append(omega)
    d = p.grid * p.grid * p.n_orient
    if not rows:
        return np.zeros((0, d), np.uint16), np.zeros((0,), np.int32), np.zeros((0,), np.int32)
    return np.stack(rows).astype(np.uint16), np.array(kp, np.int32), np.array(sh, np.int32)


def describe_plain(mim: np.ndarray, kpts: np.ndarray, p: DescParams = DescParams()):
    """RIFT's template descriptors (Sections 2.2-2.3): one row per keypoint, the cell histograms of the
    MIM as computed, no dominant-index normalisation.  Returns (counts, kp_index, shift = 0)."""
    return _rows(mim, kpts, p, [0])


def describe_ring(mim: np.ndarray, kpts: np.ndarray, p: DescParams = DescParams()):
    """RIFT's reference descriptors (Section 2.3): N_o rows per keypoint, row k N_o + omega built from
    the MIM with layer omega as the ring's initial layer.  Returns (counts, kp_index, omega)."""
    return _rows(mim, kpts, p, list(range(p.n_orient)))


# ---------------------------------------------------------------- sampling grid turned by the dominant index
#
# Section 3 takes the dominant index as SIFT takes its dominant orientation.
# SIFT also turns its sampling grid by that orientation; this variant does the
# same, since index s stands for the filter direction s pi / N_o:
#   * the dominant index comes from the MIM values inside the disc of diameter
#     P around the keypoint (a support that a rotation maps onto itself);
#   * sample (i, j) of the P x P grid (column i, row j) sits at offset
#     (u, v) = (i - P/2 + 1/2, j - P/2 + 1/2) from the corner point
#     (x - 1/2, y - 1/2) shared by the keypoint pixel and its upper-left
#     neighbours, so that with no turn the grid is exactly the axis-aligned
#     patch of `cell_histograms`;
#   * the offset is turned counter-clockwise on screen (y grows downwards) by
#     theta = s pi / N_o: (u cos + v sin, -u sin + v cos), and the nearest
#     pixel is read.  The turn uses 16-bit fixed-point cos / sin values, so
#     the pixel choice is exact integer arithmetic:
#       X = x + floor((c U + s V) / 2^17),  Y = y + floor((-s U + c V) / 2^17)
#     with U = 2i - P + 1, V = 2j - P + 1 and (c, s) the table entry;
#   * samples that fall outside the image are not counted;
#   * the sampled values are recoded by s (Eq. 2) and counted per cell;
#   * the second peak (80 % rule) gives a second row with its own turn.
# Angles are only known modulo pi (an index is a direction, not a heading),
# so a pair rotated by more than a half turn relative to the grid sees its
# descriptors with the cell grid turned by pi.


def rotation_table(n_orient: int):
    """[(cos_q, sin_q)] for theta = k pi / N_o, k = 0..N_o-1, as round(2^16 cos), round(2^16 sin)."""
    import math

    return [(int(round(math.cos(k * math.pi / n_orient) * 65536.0)),
             int(round(math.sin(k * math.pi / n_orient) * 65536.0))) for k in range(n_orient)]


def disc_histogram(mim: np.ndarray, x: int, y: int, p: DescParams) -> np.ndarray:
    """Counts of the MIM values of the pixels x + i - P/2, y + j - P/2 whose sample offsets (U, V) =
    (2i - P + 1, 2j - P + 1) satisfy U^2 + V^2 <= P^2 (the disc of diameter P), inside the image."""
    h, w = mim.shape
    P = p.patch_size
    idx = np.arange(P)
    U = 2 * idx - P + 1
    inside = (U[None, :] ** 2 + U[:, None] ** 2) <= P * P
    ys = y + idx - P // 2
    xs = x + idx - P // 2
    ok = inside & ((ys >= 0) & (ys < h))[:, None] & ((xs >= 0) & (xs < w))[None, :]
    vals = mim[np.clip(ys, 0, h - 1)[:, None], np.clip(xs, 0, w - 1)[None, :]].astype(np.int64)
    return np.bincount(vals[ok], minlength=p.n_orient)[: p.n_orient]


def rotated_cell_histograms(mim: np.ndarray, x: int, y: int, s: int, p: DescParams) -> np.ndarray:
    """h[cy, cx, b]: samples of the grid turned by s pi / N_o whose MIM value recodes (Eq. 2) to b."""
    h, w = mim.shape
    P, G, n = p.patch_size, p.grid, p.n_orient
    c, sn = rotation_table(n)[s]
    idx = np.arange(P)
    U = (2 * idx - P + 1)[None, :]  # column i
    V = (2 * idx - P + 1)[:, None]  # row j
    X = x + ((c * U + sn * V) >> 17)
    Y = y + ((-sn * U + c * V) >> 17)
    ok = (X >= 0) & (X < w) & (Y >= 0) & (Y < h)
    vals = mim[np.clip(Y, 0, h - 1), np.clip(X, 0, w - 1)].astype(np.int64)
    b = (vals - s) % n
    cell = (idx[:, None] * G // P) * G + (idx[None, :] * G // P)
    flat = (cell * n + b)[ok]
    return np.bincount(flat, minlength=G * G * n).reshape(G, G, n)


def describe_rotated(mim: np.ndarray, kpts: np.ndarray, p: DescParams = DescParams()):
    """Dominant-index descriptors on a grid turned by the dominant index (see above).

    Same row order and outputs as `describe`: (counts, kp_index, shift)."""
    prim, sec = [], []
    for i, (x, y) in enumerate(np.asarray(kpts, dtype=np.int64)):
        hist = disc_histogram(mim, int(x), int(y), p)
        s, s2, has2 = dominant(hist, p)
        prim.append((i, s, rotated_cell_histograms(mim, int(x), int(y), s, p).ravel()))
        if has2:
            sec.append((i, s2, rotated_cell_histograms(mim, int(x), int(y), s2, p).ravel()))
    rows = prim + sec
    d = p.grid * p.grid * p.n_orient
    if not rows:
        return np.zeros((0, d), np.uint16), np.zeros((0,), np.int32), np.zeros((0,), np.int32)
    counts = np.stack([r[2] for r in rows]).astype(np.uint16)
    return counts, np.array([r[0] for r in rows], np.int32), np.array([r[1] for r in rows], np.int32)
