"""Parameter records of the oracle.

Paper values: N_o = 6 orientations (Section 2.3), patch 96, FAST threshold
0.001, dominant ratio 0.8, 5000 keypoints (Table 1), 6x6 grid (Section 2.2).
The log-Gabor and phase-congruency constants are not printed in the paper; the
defaults are the usual ones of the log-Gabor phase-congruency literature the
paper builds on (minimum wavelength 3, scale factor 2.1, sigma_onf 0.55,
angular spread (pi/N_o)/1.2, Butterworth low-pass 0.45 / order 15, k = 2,
cutoff 0.5, g = 10, eps 1e-4).
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class PCParams:
    n_scales: int = 4
    n_orient: int = 6
    min_wavelength: float = 3.0
    mult: float = 2.1
    sigma_onf: float = 0.55
    dtheta_on_sigma: float = 1.2
    lp_cutoff: float = 0.45
    lp_order: int = 15
    k: float = 2.0
    cutoff: float = 0.5
    g: float = 10.0
    eps: float = 1e-4


@dataclass(frozen=True)
class DetectParams:
    fast_threshold: float = 0.001
    max_keypoints: int = 5000
    patch_size: int = 96


@dataclass(frozen=True)
class DescParams:
    patch_size: int = 96
    grid: int = 6
    n_orient: int = 6
    # second descriptor iff den * h2 >= num * h1 (ratio num/den = 0.8)
    dominant_num: int = 4
    dominant_den: int = 5


@dataclass(frozen=True)
class MatchParams:
    # accept iff d1^2 < ratio_sq * d2^2 (ratio 0.9)
    ratio_sq: float = 0.81
    # also require the accepted row's nearest B row to have this A keypoint's row as its own nearest
    mutual: bool = False
