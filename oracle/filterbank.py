"""Log-Gabor filter bank, maximum index map and phase-congruency moments (FP64).

Paper passages followed (the paper names these steps but prints no formulas):
* Section 2.2 (Feature Description): the log-Gabor convolution sequence, the
  per-orientation amplitude sums A_o(x), the multi-channel map {A_o^w} and
  the maximum index map MIM(x) = argmax_w A_o^w(x).
* Section 2.1 (Feature Detection): a one-dimensional phase congruency per
  orientation of the log-Gabor convolutions, then the variation of the
  moment with orientation giving the maximum moment M (edges) and the
  minimum moment m (corners).

Readings where the paper is silent (each listed in the design notes):
* convolution is circular (the DFT's own periodicity), input values unscaled;
* filter on exact DFT bins, frequency v = k~/H, u = l~/W with
  k~ = k - H [k >= ceil(H/2)], polar angle theta = atan2(-v, u); the filter is
  zero at DC and on the Nyquist row/column so the bank maps onto itself
  under a 90 degree rotation;
* even/odd responses e = Re EO, o = Im EO of the one-sided filter;
* MIM ties go to the lowest orientation, stored 0-based (paper 1-based);
* phase congruency is the noise-compensated energy model with the noise
  threshold T_o from the median of the smallest-scale amplitude.
"""
from __future__ import annotations

import math

import numpy as np

from .params import PCParams

__all__ = [
    "frequency_grid", "radial_factor", "lowpass_factor", "angular_factor", "log_gabor",
    "spectrum", "responses", "noise_threshold", "phase_congruency", "moments", "filter_mim",
]


def frequency_grid(h: int, w: int):
    """Signed bin frequencies (v rows, u columns) in cycles/pixel."""
    k = np.arange(h)
    l = np.arange(w)
    kt = np.where(k >= (h + 1) // 2, k - h, k)
    lt = np.where(l >= (w + 1) // 2, l - w, l)
    v = (kt / h)[:, None] * np.ones((1, w))
    u = np.ones((h, 1)) * (lt / w)[None, :]
    nyq = np.zeros((h, w), dtype=bool)
    if h % 2 == 0:
        nyq |= (kt == -h // 2)[:, None]
    if w % 2 == 0:
        nyq |= (lt == -w // 2)[None, :]
    return v, u, nyq


def radial_factor(r: np.ndarray, s: int, p: PCParams) -> np.ndarray:
    """Log-Gaussian radial profile of scale s, centre frequency 1/(lambda_min mult^s)."""
    f0 = 1.0 / (p.min_wavelength * p.mult ** s)
    with np.errstate(divide="ignore"):
        lr = np.log(r / f0)
    out = np.exp(-(lr * lr) / (2.0 * math.log(p.sigma_onf) ** 2))
    return np.where(r > 0, out, 0.0)


def lowpass_factor(r: np.ndarray, p: PCParams) -> np.ndarray:
    """Butterworth low-pass 1 / (1 + (r / cutoff)^(2 n))."""
    return 1.0 / (1.0 + (r / p.lp_cutoff) ** (2 * p.lp_order))


def angular_factor(theta: np.ndarray, o: int, p: PCParams) -> np.ndarray:
    """Gaussian angular spread about theta_o = o pi / N_o (one-sided)."""
    th_o = o * math.pi / p.n_orient
    ds = np.sin(theta) * math.cos(th_o) - np.cos(theta) * math.sin(th_o)
    dc = np.cos(theta) * math.cos(th_o) + np.sin(theta) * math.sin(th_o)
    dth = np.abs(np.arctan2(ds, dc))
    sig = (math.pi / p.n_orient) / p.dtheta_on_sigma
    return np.exp(-(dth * dth) / (2.0 * sig * sig))


def log_gabor(h: int, w: int, s: int, o: int, p: PCParams) -> np.ndarray:
    """Real frequency response G_{s,o}(k, l) on the H x W DFT grid."""
    v, u, nyq = frequency_grid(h, w)
    r = np.sqrt(u * u + v * v)
    theta = np.arctan2(-v, u)
    g = radial_factor(r, s, p) * lowpass_factor(r, p) * angular_factor(theta, o, p)
    g[0, 0] = 0.0
    g[nyq] = 0.0
    return g


def spectrum(img: np.ndarray) -> np.ndarray:
    """2-D DFT of the raw pixel values (no rescaling)."""
    return np.fft.fft2(np.asarray(img, dtype=np.float64))


def responses(spec: np.ndarray, o: int, p: PCParams) -> list:
    """Complex responses EO_{s,o} = IDFT(F G_{s,o}), s = 0..N_s-1 (circular convolution)."""
    h, w = spec.shape
    return [np.fft.ifft2(spec * log_gabor(h, w, s, o, p)) for s in range(p.n_scales)]


def noise_threshold(a0: np.ndarray, p: PCParams) -> float:
    """Noise energy threshold T_o from the smallest-scale amplitude a0 of one orientation.

    Rayleigh model: tau = median(a0)/sqrt(ln 4); the expected total amplitude
    over the geometric series of scales is tau (1 - mult^-N_s)/(1 - mult^-1);
    T = mean + k * sigma of the noise energy distribution.
    """
    tau = float(np.median(a0)) / math.sqrt(math.log(4.0))
    total = tau * (1.0 - (1.0 / p.mult) ** p.n_scales) / (1.0 - 1.0 / p.mult)
    mean = total * math.sqrt(math.pi / 2.0)
    sigma = total * math.sqrt((4.0 - math.pi) / 2.0)
    return mean + p.k * sigma


def phase_congruency(eo: list, t_o: float, p: PCParams):
    """Noise-compensated phase congruency of one orientation from its N_s complex responses.

    Returns (pc, sum_amp).  Energy is measured along the mean phase
    direction: En = sum_s (e_s phi_e + o_s phi_o - |e_s phi_o - o_s phi_e|),
    weighted by a sigmoid of the frequency spread.
    """
    e = [z.real for z in eo]
    od = [z.imag for z in eo]
    amp = [np.abs(z) for z in eo]
    s_e = sum(e)
    s_o = sum(od)
    s_a = sum(amp)
    max_a = amp[0].copy()
    for a in amp[1:]:
        max_a = np.maximum(max_a, a)
    xe = np.sqrt(s_e * s_e + s_o * s_o) + p.eps
    ph_e = s_e / xe
    ph_o = s_o / xe
    energy = np.zeros_like(s_e)
    for es, os_ in zip(e, od):
        energy += es * ph_e + os_ * ph_o - np.abs(es * ph_o - os_ * ph_e)
    spread = (s_a / (max_a + p.eps) - 1.0) / (p.n_scales - 1)
    weight = 1.0 / (1.0 + np.exp(p.g * (p.cutoff - spread)))
    pc = weight * np.maximum(energy - t_o, 0.0) / (s_a + p.eps)
    return pc, s_a


def moments(pcs: list, n_orient: int):
    """Max and min moment of phase congruency over orientation theta_o = o pi / N_o."""
    a = np.zeros_like(pcs[0])
    b = np.zeros_like(pcs[0])
    c = np.zeros_like(pcs[0])
    for o, pc in enumerate(pcs):
        th = o * math.pi / n_orient
        pcc = pc * math.cos(th)
        pcs_ = pc * math.sin(th)
        a += pcc * pcc
        b += 2.0 * pcc * pcs_
        c += pcs_ * pcs_
    root = np.sqrt(b * b + (a - c) * (a - c))
    return 0.5 * (a + c + root), 0.5 * (a + c - root)


def filter_mim(img: np.ndarray, p: PCParams = PCParams(), keep_amp: bool = True):
    """Whole filter/MIM stage on one image.

    Returns dict with
      amp  (N_o, H, W) float64  -- A_o = sum_s |EO_{s,o}|  (if keep_amp)
      mim  (H, W) uint8         -- first argmax_o A_o, 0-based
      M, m (H, W) float64       -- max / min moment of phase congruency
      T    (N_o,) float64       -- noise thresholds
    """
    spec = spectrum(img)
    h, w = spec.shape
    best = np.full((h, w), -np.inf)
    mim = np.zeros((h, w), dtype=np.uint8)
    amps = []
    pcs = []
    ts = []
    for o in range(p.n_orient):
        eo = responses(spec, o, p)
        t_o = noise_threshold(np.abs(eo[0]), p)
        pc, s_a = phase_congruency(eo, t_o, p)
        upd = s_a > best
        best = np.where(upd, s_a, best)
        mim[upd] = o
        pcs.append(pc)
        ts.append(t_o)
        if keep_amp:
            amps.append(s_a)
    big_m, small_m = moments(pcs, p.n_orient)
    out = {"mim": mim, "M": big_m, "m": small_m, "T": np.array(ts)}
    if keep_amp:
        out["amp"] = np.stack(amps)
    return out
