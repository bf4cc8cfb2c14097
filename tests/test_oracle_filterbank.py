"""Pins of the oracle's filter bank, MIM, noise threshold, phase congruency and moments.

Each test checks the oracle against something other than its own code:
definitions written out (the DFT sum, circular convolution), closed forms
of special inputs (plane waves, constant images), exact symmetries of the
bank (90 degree rotation) and brute-force order statistics.
"""
import math

import numpy as np
import pytest

from oracle import PCParams
from oracle import filterbank as fb


def naive_dft2(f, sign=-1):
    h, w = f.shape
    ky = np.exp(sign * 2j * np.pi * np.outer(np.arange(h), np.arange(h)) / h)
    kx = np.exp(sign * 2j * np.pi * np.outer(np.arange(w), np.arange(w)) / w)
    return ky @ f @ kx.T


@pytest.mark.parametrize("shape", [(12, 12), (16, 12), (18, 18), (9, 10)])
def test_spectrum_is_the_dft_sum(shape):
    rng = np.random.default_rng(1)
    f = rng.integers(0, 256, size=shape).astype(np.float64)
    ref = np.zeros(shape, dtype=complex)
    h, w = shape
    for k in range(h):
        for l in range(w):
            acc = 0j
            for y in range(h):
                for x in range(w):
                    acc += f[y, x] * complex(math.cos(-2 * math.pi * (k * y / h + l * x / w)),
                                             math.sin(-2 * math.pi * (k * y / h + l * x / w)))
            ref[k, l] = acc
    got = fb.spectrum(f)
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", [(12, 12), (18, 12), (16, 16)])
def test_responses_equal_direct_circular_convolution(shape):
    """Filtering in the frequency domain == circular convolution with h = IDFT(G)."""
    p = PCParams()
    h, w = shape
    rng = np.random.default_rng(2)
    f = rng.uniform(0, 255, size=shape)
    for o in (0, 2, 5):
        eo = fb.responses(fb.spectrum(f), o, p)
        for s in (0, 1, 3):
            g = fb.log_gabor(h, w, s, o, p)
            kern = naive_dft2(g, sign=+1) / (h * w)
            direct = np.zeros(shape, dtype=complex)
            for y in range(h):
                for x in range(w):
                    acc = 0j
                    for yy in range(h):
                        for xx in range(w):
                            acc += f[yy, xx] * kern[(y - yy) % h, (x - xx) % w]
                    direct[y, x] = acc
            scale = max(np.max(np.abs(direct)), 1e-300)
            assert np.max(np.abs(eo[s] - direct)) <= 1e-10 * scale


def test_filter_closed_form_values():
    p = PCParams(min_wavelength=4.0, mult=2.0)
    n = 64
    lp = lambda r: 1.0 / (1.0 + (r / p.lp_cutoff) ** (2 * p.lp_order))
    for s in range(3):
        f0 = 1.0 / (4.0 * 2 ** s)
        m = int(round(n * f0))
        # theta = 0 (o = 0): bin (k = 0, l = m)
        g0 = fb.log_gabor(n, n, s, 0, p)
        assert g0[0, m] == pytest.approx(lp(f0), rel=1e-12)
        # theta = pi/2 (o = N_o/2): u = 0, v = -f0 -> k = n - m
        g3 = fb.log_gabor(n, n, s, p.n_orient // 2, p)
        assert g3[n - m, 0] == pytest.approx(lp(f0), rel=1e-12)
        # DC and both Nyquist lines are zero
        assert g0[0, 0] == 0.0 and np.all(g0[n // 2, :] == 0.0) and np.all(g0[:, n // 2] == 0.0)
    # radial half-power points: exp(-1/2) at r = f0 * sigma_onf^{+-1}
    f0 = 1.0 / p.min_wavelength
    for r in (f0 * p.sigma_onf, f0 / p.sigma_onf):
        assert fb.radial_factor(np.array([r]), 0, p)[0] == pytest.approx(math.exp(-0.5), rel=1e-12)
    # angular factor exp(-1/2) at one sigma from theta_o, and 1 on theta_o
    sig = (math.pi / p.n_orient) / p.dtheta_on_sigma
    th1 = math.pi / p.n_orient
    assert fb.angular_factor(np.array([th1 + sig]), 1, p)[0] == pytest.approx(math.exp(-0.5), rel=1e-12)
    assert fb.angular_factor(np.array([th1]), 1, p)[0] == pytest.approx(1.0, rel=1e-15)
    # one-sidedness: the opposite direction is suppressed by exp(-pi^2 / (2 sig^2))
    assert fb.angular_factor(np.array([th1 + math.pi]), 1, p)[0] == pytest.approx(
        math.exp(-math.pi ** 2 / (2 * sig * sig)), rel=1e-9)


def test_bank_is_closed_under_90_degree_rotation():
    """G_{s,o+N_o/2}(R k) = G_{s,o}(k) and G_{s,o-N_o/2}(R k) = G_{s,o}(-k) on the grid."""
    p = PCParams()
    n = 48
    q = p.n_orient // 2
    kk, ll = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    kt = np.where(kk >= n // 2, kk - n, kk)
    lt = np.where(ll >= n // 2, ll - n, ll)
    # rotation by +90 degrees of theta: (u, v) -> (v, -u), i.e. l~' = k~, k~' = -l~
    rk = (-lt) % n
    rl = kt % n
    nk = (-kt) % n
    nl = (-lt) % n
    for s in range(p.n_scales):
        for o in range(p.n_orient):
            g = fb.log_gabor(n, n, s, o, p)
            gr = fb.log_gabor(n, n, s, (o + q) % p.n_orient, p)
            if o + q < p.n_orient:
                assert np.allclose(gr[rk, rl], g, rtol=1e-12, atol=1e-300)
            else:
                assert np.allclose(gr[rk, rl], g[nk, nl], rtol=1e-12, atol=1e-300)


def test_plane_wave_responses_and_mim():
    """A cosine has two spectral lines, so EO = (G(k0) e^{i phi} + G(-k0) e^{-i phi}) / 2."""
    p = PCParams()
    n = 64
    ys, xs = np.mgrid[0:n, 0:n].astype(np.float64)
    # wave vectors with direction exactly theta_0 = 0 and theta_3 = pi/2 (N_o = 6)
    for (k0, l0, expect_o) in [(0, 6, 0), (n - 6, 0, 3), (0, 11, 0), (n - 9, 0, 3)]:
        kt0 = k0 - n if k0 >= n // 2 else k0
        phase = 2 * np.pi * (l0 * xs / n + kt0 * ys / n)
        f = np.cos(phase)
        spec = fb.spectrum(f)
        fm = fb.filter_mim(f, p)
        for o in range(p.n_orient):
            eo = fb.responses(spec, o, p)
            for s in range(p.n_scales):
                g = fb.log_gabor(n, n, s, o, p)
                gp = g[k0 % n, l0 % n]
                gm = g[(-k0) % n, (-l0) % n]
                ref = 0.5 * (gp * np.exp(1j * phase) + gm * np.exp(-1j * phase))
                assert np.max(np.abs(eo[s] - ref)) < 1e-12
        assert np.all(fm["mim"] == expect_o)


def test_plane_wave_phase_congruency_closed_form():
    """Aligned orientation of a plane wave: all scales share one phase, so
    En = S^2/(S+eps) with S = sum_s A_s, and the noise median is the constant A_0."""
    p = PCParams()
    n = 64
    ys, xs = np.mgrid[0:n, 0:n].astype(np.float64)
    l0 = 7
    f = np.cos(2 * np.pi * l0 * xs / n)
    spec = fb.spectrum(f)
    eo = fb.responses(spec, 0, p)
    amps = [0.5 * fb.log_gabor(n, n, s, 0, p)[0, l0] for s in range(p.n_scales)]
    S = sum(amps)
    tau = amps[0] / math.sqrt(math.log(4))
    tot = tau * (1 - p.mult ** -p.n_scales) / (1 - 1 / p.mult)
    T = tot * math.sqrt(math.pi / 2) + p.k * tot * math.sqrt((4 - math.pi) / 2)
    assert fb.noise_threshold(np.abs(eo[0]), p) == pytest.approx(T, rel=1e-9)
    spread = (S / (max(amps) + p.eps) - 1) / (p.n_scales - 1)
    wgt = 1 / (1 + math.exp(p.g * (p.cutoff - spread)))
    expect = wgt * max(S * S / (S + p.eps) - T, 0.0) / (S + p.eps)
    pc, s_a = fb.phase_congruency(eo, T, p)
    assert np.allclose(s_a, S, rtol=1e-9)
    assert np.allclose(pc, expect, rtol=1e-8, atol=1e-12)
    assert expect > 0.1


def test_constant_image_gives_zero_everything():
    p = PCParams()
    for val in (0.0, 77.0):
        fm = fb.filter_mim(np.full((32, 32), val), p)
        assert np.max(np.abs(fm["amp"])) < 1e-9
        assert np.max(np.abs(fm["M"])) < 1e-18
        assert np.all(fm["mim"] == 0)


def test_moment_closed_forms():
    p = PCParams()
    rng = np.random.default_rng(3)
    pval = rng.uniform(0, 1, size=(5, 5))
    for o in range(p.n_orient):
        pcs = [np.zeros_like(pval) for _ in range(p.n_orient)]
        pcs[o] = pval
        big, small = fb.moments(pcs, p.n_orient)
        assert np.allclose(big, pval ** 2, rtol=1e-12, atol=1e-15)
        assert np.allclose(small, 0.0, atol=1e-15)
    big, small = fb.moments([pval] * p.n_orient, p.n_orient)
    assert np.allclose(big, p.n_orient / 2 * pval ** 2, rtol=1e-12)
    assert np.allclose(small, p.n_orient / 2 * pval ** 2, rtol=1e-12)


def test_median_threshold_is_the_exact_order_statistic():
    p = PCParams()
    rng = np.random.default_rng(4)
    for n in (10, 11, 64):
        a = rng.uniform(0, 3, size=n)
        srt = sorted(a.tolist())
        med = srt[n // 2] if n % 2 else 0.5 * (srt[n // 2 - 1] + srt[n // 2])
        tau = med / math.sqrt(math.log(4))
        tot = tau * (1 - p.mult ** -p.n_scales) / (1 - 1 / p.mult)
        T = tot * (math.sqrt(math.pi / 2) + p.k * math.sqrt((4 - math.pi) / 2))
        assert fb.noise_threshold(a, p) == pytest.approx(T, rel=1e-13)


def test_rot90_equivariance_of_amplitudes_mim_and_moments():
    """rot90 of the image rotates every map and shifts orientation by N_o/2."""
    p = PCParams()
    rng = np.random.default_rng(5)
    n = 64
    f = rng.uniform(0, 255, size=(n, n))
    f = np.real(np.fft.ifft2(np.fft.fft2(f) * np.exp(-((np.fft.fftfreq(n)[:, None] ** 2 +
                                                        np.fft.fftfreq(n)[None, :] ** 2) / 0.02))))
    a = fb.filter_mim(f, p)
    b = fb.filter_mim(np.rot90(f).copy(), p)
    q = p.n_orient // 2
    for o in range(p.n_orient):
        ref = np.rot90(a["amp"][(o + q) % p.n_orient])
        assert np.max(np.abs(b["amp"][o] - ref)) <= 1e-9 * np.max(ref)
    assert np.max(np.abs(b["M"] - np.rot90(a["M"]))) <= 1e-9 * np.max(a["M"])
    assert np.allclose(b["T"], a["T"][(np.arange(p.n_orient) + q) % p.n_orient], rtol=1e-9)
    exp_mim = (np.rot90(a["mim"]).astype(int) + q) % p.n_orient
    diff = b["mim"] != exp_mim
    # any disagreement must be a near-tie of the top two amplitude sums
    srt = np.sort(b["amp"], axis=0)
    gap = (srt[-1] - srt[-2]) / np.maximum(srt[-1], 1e-300)
    assert np.all(gap[diff] < 1e-9)
    assert diff.mean() < 1e-3


def test_noise_threshold_against_sampled_rayleigh_noise():
    """Monte Carlo pin of the noise model, independent of the formula's constants.

    Pure noise gives smallest-scale amplitudes that are Rayleigh distributed,
    and each coarser scale's noise amplitude shrinks by 1/mult.  Taking the
    scales' noise amplitudes as one common Rayleigh draw u scaled per scale,
    the total noise amplitude is sum_s sigma mult^-s u, and the threshold must
    be its mean plus k standard deviations.  Both statistics are taken from
    numpy's Rayleigh sampler, so a wrong median-to-sigma factor, a wrong
    geometric sum or wrong Rayleigh moments all fail here.
    """
    p = PCParams()
    rng = np.random.default_rng(11)
    sigma = 0.37
    u = rng.rayleigh(scale=1.0, size=2_000_000)
    a0 = sigma * u
    total = sum(sigma * p.mult ** (-s) * u for s in range(p.n_scales))
    want = total.mean() + p.k * total.std()
    got = fb.noise_threshold(a0, p)
    assert got == pytest.approx(want, rel=3e-3)
    # the threshold scales linearly with the noise level
    assert fb.noise_threshold(4.0 * a0, p) == pytest.approx(4.0 * got, rel=1e-12)
