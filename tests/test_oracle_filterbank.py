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
    # the whole stage takes its orientation-0 threshold from the smallest scale's amplitude
    assert fb.filter_mim(f, p)["T"][0] == pytest.approx(T, rel=1e-9)
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


# ---------------------------------------------------------------- phase congruency, pinned to the
# published energy model (Section 2.1 names a one-dimensional phase congruency per orientation; the
# model is the noise-compensated energy form of the log-Gabor phase-congruency literature): each
# scale's response z_s = A_s e^{i phi_s} contributes A_s (cos(phi_s - phibar) - |sin(phi_s - phibar)|),
# phibar = arg sum_s z_s, and the sum is weighted by a logistic of the normalised frequency spread.
# The oracle evaluates the same energy in rectangular form (e, o, phi_e, phi_o); the polar form below
# is the definition, so a sign flip or swapped component in the deviation term fails here.

def _polar_energy(zs, eps):
    z = sum(zs)
    bar = np.angle(z)
    en = sum(np.abs(q) * (np.cos(np.angle(q) - bar) - np.abs(np.sin(np.angle(q) - bar))) for q in zs)
    return en * np.abs(z) / (np.abs(z) + eps)


def _logit(w):
    return np.log(w / (1.0 - w))


@pytest.mark.parametrize("n_scales,amps,spread", [
    (4, (1.0, 0.5, 0.5, 0.5), 0.5),      # sum/max = 2.5 -> (2.5 - 1)/3: the sigmoid's midpoint
    (4, (2.0, 0.0, 0.0, 0.0), 0.0),      # one active scale: no spread
    (4, (0.7, 0.7, 0.7, 0.7), 1.0),      # flat over the scales: full spread
    (5, (1.0, 0.25, 0.25, 0.25, 0.25), 0.25),
    (5, (0.3, 0.3, 0.3, 0.3, 0.3), 1.0),
])
def test_spread_weight_is_a_logistic_of_the_normalised_spread(n_scales, amps, spread):
    """With every scale in phase and no noise threshold the energy equals sum_s A_s, so PC is the
    weight itself; its logit must be g (spread - cutoff) with spread normalised to [0, 1]
    (0 for one active scale, 1 for equal amplitudes).  Dropping the (N_s - 1) normalisation, moving
    the cutoff or changing the gain fails."""
    p = PCParams(n_scales=n_scales, eps=0.0)
    phase = 0.3
    zs = [np.array([a * np.exp(1j * phase)]) for a in amps]
    pc, s_a = fb.phase_congruency(zs, 0.0, p)
    assert s_a[0] == pytest.approx(sum(amps), rel=1e-15)
    assert _logit(pc[0]) == pytest.approx(p.g * (spread - p.cutoff), abs=1e-9)
    if spread == p.cutoff:
        assert pc[0] == pytest.approx(0.5, abs=1e-15)


def test_phase_congruency_energy_matches_the_polar_definition():
    """Random per-scale phases and amplitudes at the spread cutoff (weight exactly 1/2, eps = 0):
    PC = max(En - T, 0) / (2 sum A) with En from the polar definition."""
    p = PCParams(eps=0.0)
    rng = np.random.default_rng(21)
    n = 4000
    amps = np.array([1.0, 0.5, 0.5, 0.5])
    scale = rng.uniform(0.1, 50.0, size=n)
    phases = [rng.uniform(-np.pi, np.pi, size=n) for _ in range(p.n_scales)]
    # half the pixels nearly in phase (large energy), half random
    for s in range(1, p.n_scales):
        phases[s][: n // 2] = phases[0][: n // 2] + rng.normal(0.0, 0.2, size=n // 2)
    zs = [amps[s] * scale * np.exp(1j * phases[s]) for s in range(p.n_scales)]
    for t in (0.0, 3.0):
        pc, s_a = fb.phase_congruency(zs, t, p)
        en = _polar_energy(zs, 0.0)
        want = 0.5 * np.maximum(en - t, 0.0) / s_a
        assert np.allclose(pc, want, rtol=1e-12, atol=1e-14)
        assert np.count_nonzero(want) > n // 3  # the deviation term is exercised where En > T


def test_phase_congruency_deviation_term_has_its_sign():
    """Two equal responses a half-angle delta either side of their mean phase: the energy is
    2 A (cos delta - |sin delta|) (times |Z| / (|Z| + eps)), which is negative past 45 degrees."""
    p = PCParams(n_scales=2, eps=1e-4)
    for delta, a in ((0.1, 5.0), (0.5, 2.0), (np.pi / 4, 3.0), (1.2, 1.0)):
        bar = 0.7
        zs = [np.array([a * np.exp(1j * (bar + delta))]), np.array([a * np.exp(1j * (bar - delta))])]
        zmag = 2 * a * np.cos(delta)
        en = 2 * a * (np.cos(delta) - abs(np.sin(delta))) * zmag / (zmag + p.eps)
        # equal amplitudes over two scales: spread 1 (up to eps), weight of the logistic at 1
        sp = (2 * a / (a + p.eps) - 1.0)
        w = 1.0 / (1.0 + np.exp(p.g * (p.cutoff - sp)))
        pc, _ = fb.phase_congruency(zs, 0.0, p)
        assert pc[0] == pytest.approx(w * max(en, 0.0) / (2 * a + p.eps), rel=1e-12, abs=1e-15)
        if delta > np.pi / 4:
            assert pc[0] == 0.0


def test_two_spectral_lines_phase_congruency_closed_form():
    """f = cos(2 pi l1 x / n) + cos(2 pi l2 x / n + psi): along orientation 0 every scale's response is
    (G_s(l1) e^{i theta1} + G_s(l2) e^{i theta2}) / 2 (the mirrored lines fall where the one-sided
    angular factor is below 1e-11), so the scales' phases differ pixel by pixel.  The oracle's PC of
    orientation 0 must equal the polar-form PC of these closed-form responses."""
    p = PCParams()
    n = 64
    l1, l2, psi = 5, 13, 1.1
    xs = np.mgrid[0:n, 0:n][1].astype(np.float64)
    th1 = 2 * np.pi * l1 * xs / n
    th2 = 2 * np.pi * l2 * xs / n + psi
    f = np.cos(th1) + np.cos(th2)
    eo = fb.responses(fb.spectrum(f), 0, p)
    zs = []
    for s in range(p.n_scales):
        g = fb.log_gabor(n, n, s, 0, p)
        zs.append(0.5 * (g[0, l1] * np.exp(1j * th1) + g[0, l2] * np.exp(1j * th2)))
        assert np.max(np.abs(eo[s] - zs[-1])) < 1e-10
    amps = [np.abs(z) for z in zs]
    t = fb.noise_threshold(amps[0], p)
    # the exact order statistic of the closed-form amplitudes (library median as the primitive)
    med = float(np.median(amps[0]))
    tot = med / math.sqrt(math.log(4)) * (1 - p.mult ** -p.n_scales) / (1 - 1 / p.mult)
    assert t == pytest.approx(tot * (math.sqrt(math.pi / 2) + p.k * math.sqrt((4 - math.pi) / 2)), rel=1e-12)
    sa = sum(amps)
    mx = np.maximum.reduce(amps)
    sp = (sa / (mx + p.eps) - 1.0) / (p.n_scales - 1)
    w = 1.0 / (1.0 + np.exp(p.g * (p.cutoff - sp)))
    want = w * np.maximum(_polar_energy(zs, p.eps) - t, 0.0) / (sa + p.eps)
    pc, _ = fb.phase_congruency(eo, t, p)
    assert np.max(np.abs(pc - want)) < 1e-9
    # the scales really disagree in phase somewhere, and PC is positive somewhere
    dev = np.abs(np.angle(zs[0] * np.conj(zs[2])))
    assert dev.max() > 1.0 and (want > 0.05).any()


def test_lowpass_is_a_butterworth_of_the_stated_order():
    """1/2 at the cutoff, 1 at DC, and an asymptotic log-log slope of -2 n (n = lp_order)."""
    for order in (15, 7):
        p = PCParams(lp_order=order)
        assert fb.lowpass_factor(np.array([p.lp_cutoff]), p)[0] == pytest.approx(0.5, abs=1e-15)
        assert fb.lowpass_factor(np.array([0.0]), p)[0] == 1.0
        r1, r2 = 4.0 * p.lp_cutoff, 8.0 * p.lp_cutoff
        l1, l2 = fb.lowpass_factor(np.array([r1, r2]), p)
        slope = (math.log(l2) - math.log(l1)) / (math.log(r2) - math.log(r1))
        assert slope == pytest.approx(-2.0 * order, rel=1e-6)
