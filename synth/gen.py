"""Synthetic image-pair generator.

The paper evaluates on 100 SAR-optical and 100 infrared-optical pairs, each with
a ground-truth rotation + translation, whose images suffer from nonlinear
radiation distortion (Section 4, Experiments).  Those datasets are not
available, so pairs are synthesised:

* scene A: sum of random Gaussian blobs plus random filled rotated rectangles
  and thick line segments, min-max scaled to [0, V] and rounded;
* image B: A warped by a similarity transform (rotation about the image
  centre + translation, bilinear, zero outside), remapped by a nonlinear
  intensity curve (inversion + gamma for the small case, a random monotone or
  inverted 8-knot piecewise-linear curve otherwise) and multiplied by i.i.d.
  Gamma(L, 1/L) speckle (mean 1), then clipped and rounded.

Every random draw comes from numpy PCG64 streams spawned from one seed, so a
(config, index) pair is byte-identical across runs and machines.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = ["CONFIGS", "PairConfig", "make_pair", "make_shifted_pair", "make_scene", "serving_sizes", "keypoint_cap",
           "gt_similarity"]


@dataclass(frozen=True)
class PairConfig:
    size: int
    dtype: type
    vmax: int
    n_blob: int
    n_shape: int
    angle_deg: float | None  # None -> uniform in [0, 360)
    max_shift: float
    remap: str  # "invert_gamma" or "pwl8"
    looks: float
    n_scales: int
    n_orient: int
    max_keypoints: int


# Workload definitions (sizes, value ranges, counts) for the five standard cases.
CONFIGS = {
    0: PairConfig(256, np.uint8, 255, 40, 15, 30.0, 0.0, "invert_gamma", 4.0, 4, 6, 500),
    1: PairConfig(1024, np.uint8, 255, 200, 60, None, 64.0, "pwl8", 4.0, 4, 6, 5000),
    2: PairConfig(2048, np.uint8, 255, 200, 60, None, 64.0, "pwl8", 4.0, 4, 6, 20000),
    3: PairConfig(1024, np.uint8, 255, 200, 60, None, 64.0, "pwl8", 4.0, 4, 6, 2097),
    4: PairConfig(4096, np.uint16, 4095, 800, 240, None, 64.0, "pwl8", 1.0, 5, 8, 50000),
}

SEED_STRIDE = 1_000_003


def serving_sizes():
    """Square sizes drawn by the mixed-size serving workload."""
    return (512, 768, 1024, 1536, 2048)


def keypoint_cap(h: int, w: int) -> int:
    """Serving keypoint budget: 2e-3 of the pixel count."""
    return int(2 * h * w // 1000)


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]


def _add_blobs(canvas: np.ndarray, rng: np.random.Generator, n: int) -> None:
    h, w = canvas.shape
    for _ in range(n):
        cx = rng.uniform(0, w)
        cy = rng.uniform(0, h)
        sig = rng.uniform(3.0, 20.0)
        amp = rng.uniform(-1.0, 1.0)
        rad = int(math.ceil(4 * sig))
        x0, x1 = max(0, int(cx) - rad), min(w, int(cx) + rad + 1)
        y0, y1 = max(0, int(cy) - rad), min(h, int(cy) + rad + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        xs = np.arange(x0, x1, dtype=np.float64) - cx
        ys = np.arange(y0, y1, dtype=np.float64) - cy
        g = np.exp(-(ys[:, None] ** 2 + xs[None, :] ** 2) / (2 * sig * sig))
        canvas[y0:y1, x0:x1] += amp * g


def _add_shapes(canvas: np.ndarray, rng: np.random.Generator, n: int) -> None:
    h, w = canvas.shape
    for _ in range(n):
        if rng.uniform() < 0.5:
            # filled rotated rectangle
            cx, cy = rng.uniform(0, w), rng.uniform(0, h)
            a = rng.uniform(4.0, min(h, w) / 8.0)
            b = rng.uniform(4.0, min(h, w) / 8.0)
            ang = rng.uniform(0.0, math.pi)
            amp = rng.uniform(-1.0, 1.0)
            rad = int(math.ceil(math.hypot(a, b))) + 1
            x0, x1 = max(0, int(cx) - rad), min(w, int(cx) + rad + 1)
            y0, y1 = max(0, int(cy) - rad), min(h, int(cy) + rad + 1)
            if x0 >= x1 or y0 >= y1:
                continue
            xs = np.arange(x0, x1, dtype=np.float64) - cx
            ys = np.arange(y0, y1, dtype=np.float64) - cy
            X, Y = np.meshgrid(xs, ys)
            c, s = math.cos(ang), math.sin(ang)
            pu = c * X + s * Y
            pv = -s * X + c * Y
            inside = (np.abs(pu) <= a) & (np.abs(pv) <= b)
            canvas[y0:y1, x0:x1] += amp * inside
        else:
            # thick line segment
            xa, ya = rng.uniform(0, w), rng.uniform(0, h)
            xb, yb = rng.uniform(0, w), rng.uniform(0, h)
            hw = rng.uniform(0.5, 2.0)
            amp = rng.uniform(-1.0, 1.0)
            x0 = max(0, int(min(xa, xb) - hw) - 1)
            x1 = min(w, int(max(xa, xb) + hw) + 2)
            y0 = max(0, int(min(ya, yb) - hw) - 1)
            y1 = min(h, int(max(ya, yb) + hw) + 2)
            if x0 >= x1 or y0 >= y1:
                continue
            xs = np.arange(x0, x1, dtype=np.float64)
            ys = np.arange(y0, y1, dtype=np.float64)
            X, Y = np.meshgrid(xs, ys)
            dx, dy = xb - xa, yb - ya
            L2 = dx * dx + dy * dy
            if L2 == 0.0:
                tpar = np.zeros_like(X)
            else:
                tpar = np.clip(((X - xa) * dx + (Y - ya) * dy) / L2, 0.0, 1.0)
            dist = np.hypot(X - (xa + tpar * dx), Y - (ya + tpar * dy))
            canvas[y0:y1, x0:x1] += amp * (dist <= hw)


def make_scene(size: int, n_blob: int, n_shape: int, vmax: int, rng: np.random.Generator) -> np.ndarray:
    """Scene A as float64 values already rounded to integers in [0, vmax]."""
    canvas = np.zeros((size, size), dtype=np.float64)
    _add_blobs(canvas, rng, n_blob)
    _add_shapes(canvas, rng, n_shape)
    lo, hi = canvas.min(), canvas.max()
    if hi > lo:
        canvas = (canvas - lo) / (hi - lo) * vmax
    else:
        canvas = np.zeros_like(canvas)
    return np.rint(canvas)


def _warp_bilinear(img: np.ndarray, phi: float, tx: float, ty: float) -> np.ndarray:
    """B(p) = A(R(-phi)(p - c - t) + c) with zero outside A."""
    h, w = img.shape
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    px, py = xs - cx - tx, ys - cy - ty
    c, s = math.cos(phi), math.sin(phi)
    ax = c * px + s * py + cx
    ay = -s * px + c * py + cy
    x0 = np.floor(ax).astype(np.int64)
    y0 = np.floor(ay).astype(np.int64)
    fx, fy = ax - x0, ay - y0
    pad = np.zeros((h + 2, w + 2), dtype=np.float64)
    pad[1:-1, 1:-1] = img

    def at(yy, xx):
        ok = (yy >= -1) & (yy <= h) & (xx >= -1) & (xx <= w)
        yy = np.clip(yy, -1, h) + 1
        xx = np.clip(xx, -1, w) + 1
        return np.where(ok, pad[yy, xx], 0.0)

    return ((1 - fy) * ((1 - fx) * at(y0, x0) + fx * at(y0, x0 + 1))
            + fy * ((1 - fx) * at(y0 + 1, x0) + fx * at(y0 + 1, x0 + 1)))


def _remap(img: np.ndarray, kind: str, vmax: int, rng: np.random.Generator) -> np.ndarray:
    if kind == "invert_gamma":
        return vmax * np.power(np.clip((vmax - img) / vmax, 0.0, 1.0), 0.5)
    knots_x = vmax * np.arange(8) / 7.0
    inner = np.sort(rng.uniform(0.0, vmax, size=6))
    knots_y = np.concatenate([[0.0], inner, [float(vmax)]])
    if rng.uniform() < 0.5:
        knots_y = vmax - knots_y
    return np.interp(img, knots_x, knots_y)


def make_pair(config: int, index: int, size: int | None = None):
    """Return (A, B, gt) for workload `config`, pair `index`.

    `size` overrides the image side (mixed-size serving); blob and shape
    counts then scale with the image area relative to the config's size.
    gt = {"phi": radians, "t": (tx, ty), "size": (H, W)}; p_B = R(phi)(p_A - c) + c + t.
    """
    cfg = CONFIGS[config]
    n = cfg.size if size is None else int(size)
    scale = (n * n) / float(cfg.size * cfg.size)
    n_blob = max(10, int(round(cfg.n_blob * scale)))
    n_shape = max(4, int(round(cfg.n_shape * scale)))
    scene_rng, warp_rng, noise_rng = _streams(SEED_STRIDE * config + index)
    a = make_scene(n, n_blob, n_shape, cfg.vmax, scene_rng)
    if cfg.angle_deg is None:
        phi = math.radians(warp_rng.uniform(0.0, 360.0))
    else:
        phi = math.radians(cfg.angle_deg)
    tx = warp_rng.uniform(-cfg.max_shift, cfg.max_shift) if cfg.max_shift > 0 else 0.0
    ty = warp_rng.uniform(-cfg.max_shift, cfg.max_shift) if cfg.max_shift > 0 else 0.0
    b = _warp_bilinear(a, phi, tx, ty)
    b = _remap(b, cfg.remap, cfg.vmax, noise_rng)
    b = b * noise_rng.gamma(shape=cfg.looks, scale=1.0 / cfg.looks, size=b.shape)
    b = np.rint(np.clip(b, 0, cfg.vmax))
    gt = {"phi": phi, "t": (tx, ty), "size": (n, n)}
    return a.astype(cfg.dtype), b.astype(cfg.dtype), gt


def make_shifted_pair(config: int, index: int, size: int | None = None, shift=(5.0, -3.0)):
    """Return (A, B, gt): A is pair `index`'s scene of workload `config`; B is A translated by `shift`
    (bilinear, zero outside), inverted and gamma-0.5 remapped, with no rotation and no speckle.

    The workloads' own pairs (arbitrary rotations, 1- or 4-look speckle) leave almost no descriptor
    rows through the ratio test, so a match-set comparison on them is empty; this pair keeps
    thousands of matches at the same size and keypoint count."""
    cfg = CONFIGS[config]
    n = cfg.size if size is None else int(size)
    scale = (n * n) / float(cfg.size * cfg.size)
    n_blob = max(10, int(round(cfg.n_blob * scale)))
    n_shape = max(4, int(round(cfg.n_shape * scale)))
    scene_rng, _, noise_rng = _streams(SEED_STRIDE * config + index)
    a = make_scene(n, n_blob, n_shape, cfg.vmax, scene_rng)
    b = _warp_bilinear(a, 0.0, float(shift[0]), float(shift[1]))
    b = np.rint(np.clip(_remap(b, "invert_gamma", cfg.vmax, noise_rng), 0, cfg.vmax))
    gt = {"phi": 0.0, "t": (float(shift[0]), float(shift[1])), "size": (n, n)}
    return a.astype(cfg.dtype), b.astype(cfg.dtype), gt


def gt_similarity(gt) -> tuple:
    """The pair's warp p_B = R(phi)(p_A - c) + c + t as (a, b, tx, ty) with u = a x - b y + tx,
    v = b x + a y + ty (c the image centre)."""
    h, w = gt["size"]
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    a, b = math.cos(gt["phi"]), math.sin(gt["phi"])
    return (a, b, cx + gt["t"][0] - (a * cx - b * cy), cy + gt["t"][1] - (b * cx + a * cy))
