"""End-to-end oracle for one image pair (Fig. 1 workflow: detection, description, matching)."""
from __future__ import annotations

import numpy as np

from .params import PCParams, DetectParams, DescParams, MatchParams
from . import filterbank, detect, describe, match

__all__ = ["image_features", "match_pair", "ring_match_pair"]


def image_features(img, pc=PCParams(), det=DetectParams(), desc=None, dtype=np.float64, keep_amp=False,
                   turned=False):
    """Filter/MIM, keypoints on the max moment map and descriptors of one image (turned=True: the
    sampling grid turned by the dominant index, describe.describe_rotated)."""
    if desc is None:
        desc = DescParams(patch_size=det.patch_size, n_orient=pc.n_orient)
    fm = filterbank.filter_mim(img, pc, keep_amp=keep_amp)
    kpts, scores = detect.detect(fm["M"], det, dtype=dtype)
    counts, kp, shift = (describe.describe_rotated if turned else describe.describe)(fm["mim"], kpts, desc)
    return {"fm": fm, "kpts": kpts, "scores": scores, "desc": counts, "desc_kp": kp, "shift": shift}


def match_pair(img_a, img_b, pc=PCParams(), det=DetectParams(), mp=MatchParams(), dtype=np.float64, turned=False):
    fa = image_features(img_a, pc, det, dtype=dtype, turned=turned)
    fb = image_features(img_b, pc, det, dtype=dtype, turned=turned)
    m = match.match(fa["desc"], fa["desc_kp"], fb["desc"], fb["desc_kp"], mp, dtype=dtype)
    return fa, fb, m


def ring_match_pair(img_t, img_r, pc=PCParams(), det=DetectParams(), mp=MatchParams(), dtype=np.float64):
    """RIFT's ring form of one pair (Section 2.3), the baseline RIFT2 replaces: the template's plain
    descriptors are matched against the N_o ring descriptors of every reference keypoint.
    Returns (template features, reference features, matches (kp_t, kp_r, d2))."""
    desc = DescParams(patch_size=det.patch_size, n_orient=pc.n_orient)
    feats = []
    for img, form in ((img_t, describe.describe_plain), (img_r, describe.describe_ring)):
        fm = filterbank.filter_mim(img, pc)
        kpts, scores = detect.detect(fm["M"], det, dtype=dtype)
        counts, kp, shift = form(fm["mim"], kpts, desc)
        feats.append({"fm": fm, "kpts": kpts, "scores": scores, "desc": counts, "desc_kp": kp, "shift": shift})
    ft, fr = feats
    m = match.match(ft["desc"], ft["desc_kp"], fr["desc"], fr["desc_kp"], mp, dtype=dtype)
    return ft, fr, m
