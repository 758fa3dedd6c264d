"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests re-types an oracle formula and compares it with itself:
each one checks a limit, a special value, an identity between two different
computations, a brute-force evaluation, or a literature constant.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


# ---------------------------------------------------------------------------
# Eq. (2): special values and limits of the printed closed form
# ---------------------------------------------------------------------------
def test_psd_equals_one_at_knee():
    # At f = f0 the three constant-ish terms sum to 0.16 + 0.52 + 0.32 = 1 and the
    # seismic wall contributes 4.49^-56 ~ 3e-37.
    c = _golden("paper_constants.json")
    assert c["psd_f0_hz"] == O.PSD_F0
    assert O.psd_initial_ligo(150.0) == pytest.approx(1.0, abs=1e-15)


def test_psd_log_slopes_pin_exponents():
    def slope(f, h=1e-4):
        return (math.log(O.psd_initial_ligo(f * (1 + h))) - math.log(O.psd_initial_ligo(f * (1 - h)))) / (
            math.log1p(h) - math.log1p(-h))
    # Far below the knee the seismic wall (exponent -56) dominates by ~76 decades.
    assert slope(1.0) == pytest.approx(-56.0, rel=1e-7)
    # Far above the knee the shot-noise term (exponent +2) dominates.
    assert slope(1.5e7) == pytest.approx(2.0, abs=1e-8)


def test_psd_high_frequency_coefficients():
    x = 1.0e6
    S = O.psd_initial_ligo(150.0 * x)
    assert S / x ** 2 == pytest.approx(0.32, rel=1e-11)
    x = 1.0e3
    S = O.psd_initial_ligo(150.0 * x)
    # S - 0.32 x^2 -> 0.52 (the mid term has decayed as x^-4.52 to ~2e-15).
    assert S - 0.32 * x * x == pytest.approx(0.52, abs=2e-9)


def test_psd_thermal_term_from_knee_value():
    # Knowing S(f0)=1, the constant 0.52 and the x^2 coefficient 0.32 fixes the
    # coefficient of the x^-4.52 term at 0.16; check that slope near 100 Hz
    # matches the mixture implied by those weights (no seismic contribution).
    f = 100.0
    x = f / 150.0
    mid = 0.16 * x ** -4.52
    hi = 0.32 * x * x
    expected = (-4.52 * mid + 2.0 * hi) / (mid + 0.52 + hi)
    h = 1e-5
    got = (math.log(O.psd_initial_ligo(f * (1 + h))) - math.log(O.psd_initial_ligo(f * (1 - h)))) / (
        math.log1p(h) - math.log1p(-h))
    assert got == pytest.approx(expected, rel=1e-6)


def test_psd_fp64_accuracy_against_40_digits():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    for f in [30.0, 40.0, 57.3, 150.0, 1024.0, 2047.9]:
        x = mp.mpf(f) / 150
        ref = (mp.mpf("4.49") * x) ** -56 + mp.mpf("0.16") * x ** mp.mpf("-4.52") + mp.mpf("0.52") + mp.mpf("0.32") * x ** 2
        assert abs(O.psd_initial_ligo(f) - float(ref)) <= 8e-15 * float(ref)


def test_psd_bins_band_and_inf_outside():
    n, fs = 1 << 12, 512.0
    S = O.psd_bins(n, fs, 40.0)
    k_lo = O.band_lo(n, fs, 40.0)
    assert k_lo == math.ceil(40.0 * n / fs)
    assert np.all(np.isinf(S[:k_lo])) and np.isinf(S[n // 2])
    assert np.all(np.isfinite(S[k_lo: n // 2]))


# ---------------------------------------------------------------------------
# Band edges and constants
# ---------------------------------------------------------------------------
def test_tsun_from_nominal_solar_mass_parameter():
    lit = _golden("literature_values.json")
    assert O.T_SUN == pytest.approx(lit["gm_sun_nominal_m3_s2"] / lit["speed_of_light_m_s"] ** 3, rel=1e-12)


def test_f_isco_textbook_scaling():
    lit = _golden("literature_values.json")
    assert O.f_isco(1.0) == pytest.approx(lit["f_isco_hz_times_msun"], abs=lit["f_isco_hz_times_msun_tol"])
    assert O.f_isco(2.8) * 2.8 == pytest.approx(O.f_isco(1.0), rel=1e-13)


def test_band_edges_paper_set_up():
    c = _golden("paper_constants.json")
    n = c["segment_points"]
    fs = c["sample_rate_hz"]
    assert n / fs == c["segment_seconds"]
    # 40 Hz x 256 s is an exact bin.
    mc, eta = synth.mc_eta(1.4, 1.4)
    k_lo, k_hi = O.band(n, fs, c["f_low_hz"], float(mc), float(eta))
    assert k_lo == 10240
    assert k_hi == math.floor(O.f_isco(2.8) * 256.0)
    assert 401900 < k_hi < 402100
    # Light templates are cut at Nyquist - 1 bin.
    mc, eta = synth.mc_eta(1.0, 1.0)
    assert O.band(n, fs, 40.0, float(mc), float(eta))[1] == n // 2 - 1
    with pytest.raises(ValueError):
        O.band(1 << 10, 256.0, 40.0, *map(float, synth.mc_eta(100.0, 100.0)))


# ---------------------------------------------------------------------------
# SPA phase: stationary-phase time/frequency relation and Newtonian limit
# ---------------------------------------------------------------------------
def _chirp_time_2pn(f, mc, eta):
    """Time to coalescence from frequency f at 2PN, typed from the literature
    (Sathyaprakash & Dhurandhar; Blanchet, Iyer, Will & Wiseman)."""
    M = mc * eta ** -0.6 * 4.925490947641267e-6
    v = (math.pi * M * f) ** (1.0 / 3.0)
    t2 = 743.0 / 252.0 + 11.0 * eta / 3.0
    t3 = -32.0 * math.pi / 5.0
    t4 = 3058673.0 / 508032.0 + 5429.0 * eta / 504.0 + 617.0 * eta ** 2 / 72.0
    return 5.0 * M / (256.0 * eta * v ** 8) * (1.0 + t2 * v ** 2 + t3 * v ** 3 + t4 * v ** 4)


@pytest.mark.parametrize("m1,m2", [(1.4, 1.4), (1.0, 3.0), (10.0, 1.2), (17.5, 17.5), (33.0, 1.5)])
@pytest.mark.parametrize("f", [40.0, 75.0, 200.0])
def test_spa_phase_derivative_is_minus_chirp_time(m1, m2, f):
    mc, eta = map(float, synth.mc_eta(m1, m2))
    h = 1e-20 * f
    dpsi = float(np.imag(O.spa_phase(f + 1j * h, mc, eta))) / h  # complex-step derivative
    assert dpsi / (2 * math.pi) == pytest.approx(-_chirp_time_2pn(f, mc, eta), rel=1e-12)


def test_spa_tc_shifts_derivative():
    mc, eta = map(float, synth.mc_eta(1.4, 1.4))
    f, tc = 55.0, 17.25
    h = 1e-20 * f
    d0 = float(np.imag(O.spa_phase(f + 1j * h, mc, eta))) / h
    d1 = float(np.imag(O.spa_phase(f + 1j * h, mc, eta, tc=tc))) / h
    assert (d1 - d0) / (2 * math.pi) == pytest.approx(tc, rel=1e-12)


def test_spa_newtonian_limit_depends_on_chirp_mass_only():
    lit = _golden("literature_values.json")
    for (m1, m2) in [(1.4, 1.4), (2.0, 1.0), (30.0, 4.0)]:
        mc, eta = map(float, synth.mc_eta(m1, m2))
        f = 1e-7
        psi = O.spa_phase(f, mc, eta) + math.pi / 4
        newt = 3.0 / 128.0 * (math.pi * mc * O.T_SUN * f) ** (-5.0 / 3.0)
        assert psi / newt == pytest.approx(1.0, rel=2e-5)
    mc, eta = map(float, synth.mc_eta(1.4, 1.4))
    tau0 = 5.0 / 256.0 * (math.pi * 40.0) ** (-8.0 / 3.0) * (mc * O.T_SUN) ** (-5.0 / 3.0)
    assert tau0 == pytest.approx(lit["newtonian_chirp_time_bns_40hz_s"], abs=lit["newtonian_chirp_time_tol_s"])


def test_template_time_domain_ends_at_tc():
    # The sign convention h = a e^{-i Psi} with Psi containing +2 pi f t_c puts the
    # chirp before t_c: inverse-transform a template with t_c in the middle.
    n, fs = 1 << 15, 2048.0
    T = n / fs
    mc, eta = map(float, synth.mc_eta(5.0, 5.0))
    tc = T / 2
    h = O.spa_template(n, fs, 40.0, mc, eta, tc=tc)
    ht = np.fft.irfft(h, n)
    t = np.arange(n) / fs
    before = np.sum(ht[(t > tc - 4.0) & (t < tc)] ** 2)
    after = np.sum(ht[(t > tc + 0.05) & (t < tc + 4.05)] ** 2)
    assert after < 1e-3 * before


def test_template_amplitude_and_band():
    n, fs = 1 << 16, 2048.0
    mc, eta = map(float, synth.mc_eta(2.0, 2.0))
    h = O.spa_template(n, fs, 40.0, mc, eta)
    k_lo, k_hi = O.band(n, fs, 40.0, mc, eta)
    f = O.freqs(n, fs)
    assert np.all(h[:k_lo] == 0) and np.all(h[k_hi + 1:] == 0)
    np.testing.assert_allclose(np.abs(h[k_lo:k_hi + 1]), f[k_lo:k_hi + 1] ** (-7.0 / 6.0), rtol=1e-14)


def _newtonian_chirp_time(f, mc):
    """Newtonian time to coalescence from GW frequency f (quadrupole inspiral):
    5/256 (pi f)^(-8/3) (G M_c / c^3)^(-5/3).  Accepts complex f."""
    return 5.0 / 256.0 * (np.pi * f) ** (-8.0 / 3.0) * (mc * 4.925490947641267e-6) ** (-5.0 / 3.0)


@pytest.mark.parametrize("m1,m2", [(1.4, 1.4), (3.0, 1.0), (20.0, 5.0)])
def test_spa_amplitude_from_stationary_phase_relation(m1, m2):
    """Stationary phase: a quadrupole chirp of amplitude ~ f^(2/3) that sweeps through f
    at the rate set by the chirp time has |h(f)|^2 proportional to f^(4/3) |d tau/df|.
    The oracle's amplitude must make that ratio constant over the band."""
    mc, _ = map(float, synth.mc_eta(m1, m2))
    f = np.geomspace(40.0, 1000.0, 41)
    h = 1e-20 * f
    dtau = np.imag(_newtonian_chirp_time(f + 1j * h, mc)) / h  # complex-step derivative
    ratio = O.spa_amplitude(f) ** 2 / (f ** (4.0 / 3.0) * np.abs(dtau))
    assert np.max(np.abs(ratio / ratio[0] - 1.0)) < 1e-12


def _time_domain_chirp_spectrum(m1, m2, fs, n, f_start, f_stop):
    """One-sided spectrum dt * DFT of a Newtonian chirp built in the time domain:
    frequency f(t) from inverting the chirp time, phase by summing 2 pi f dt,
    amplitude (pi M_c f)^(2/3), with raised-cosine tapers at both ends."""
    mc, _ = map(float, synth.mc_eta(m1, m2))
    Mc = mc * 4.925490947641267e-6
    tau_start = float(_newtonian_chirp_time(f_start, mc))
    tau_stop = float(_newtonian_chirp_time(f_stop, mc))
    dt = 1.0 / fs
    tau = tau_start + 1.0 - np.arange(n) * dt
    on = (tau > tau_stop) & (tau <= tau_start)
    f = np.zeros(n)
    f[on] = (5.0 / (256.0 * tau[on])) ** (3.0 / 8.0) * Mc ** (-5.0 / 8.0) / math.pi
    phase = np.cumsum(2.0 * math.pi * f) * dt
    amp = np.where(on, (math.pi * Mc * f) ** (2.0 / 3.0), 0.0)
    w = np.ones(n)
    i0 = int(np.argmax(on))
    i1 = n - 1 - int(np.argmax(on[::-1]))
    l0, l1 = int(2.0 * fs), int(0.02 * fs)
    w[i0:i0 + l0] = 0.5 - 0.5 * np.cos(np.pi * np.arange(l0) / l0)
    w[i1 - l1 + 1:i1 + 1] = 0.5 + 0.5 * np.cos(np.pi * np.arange(l1) / l1)
    return np.fft.rfftfreq(n, dt), np.fft.rfft(amp * np.cos(phase) * w) * dt


@pytest.mark.parametrize("m1,m2", [(1.4, 1.4), (3.0, 1.0)])
def test_spa_amplitude_matches_time_domain_chirp(m1, m2):
    """Brute force: the spectrum of a time-domain Newtonian chirp (64 s at 4096 Hz,
    30-700 Hz) has the oracle's amplitude shape between 50 and 400 Hz: |H| / a(f)
    is flat to about 1% and its log-log slope vanishes."""
    fq, H = _time_domain_chirp_spectrum(m1, m2, 4096.0, 1 << 18, 30.0, 700.0)
    sel = (fq > 50.0) & (fq < 400.0)
    r = np.abs(H[sel]) / O.spa_amplitude(fq[sel])
    assert r.max() / r.min() < 1.03
    slope = np.polyfit(np.log(fq[sel]), np.log(r), 1)[0]
    assert abs(slope) < 5e-3


# ---------------------------------------------------------------------------
# Quadrature pair and z = x + i y
# ---------------------------------------------------------------------------
def _real_filter(h, stilde, Sn, n, df):
    """Real matched-filter output of template h: two-sided integral of
    conj(h) s / S e^{2 pi i f t} over a Hermitian spectrum (via irfft)."""
    inv = np.where(np.isfinite(Sn), 1.0 / Sn, 0.0)
    q = 2.0 * df * np.conj(h) * stilde * inv  # weight of each positive-frequency bin
    q[0] = 0
    q[n // 2] = 0
    # irfft(Q) * n = Q_0 + 2 Re sum_{k>0} Q_k e^{+2 pi i jk/N} (for zero DC/Nyquist)
    return np.fft.irfft(q, n) * n


def _noise_segment(n, fs, seed, injection=None):
    g = O.grid(n, fs)
    Sn = O.psd_bins(n, fs, 40.0)
    k_lo = O.band_lo(n, fs, 40.0)
    rng = np.random.Generator(np.random.PCG64(seed))
    s = synth.coloured_noise(Sn[k_lo: n // 2], g["df"], k_lo, n // 2 + 1, rng, dtype=np.complex128)
    if injection is not None:
        mc, eta, snr, j0, phi0 = injection
        h = O.spa_template(n, fs, 40.0, mc, eta)
        sig = math.sqrt(O.sigma_sq(h, Sn, g["df"]))
        s = synth.inject(s, h, snr / sig, phi0, j0, n)
    return s, Sn, g


def test_quadrature_pair_orthogonal():
    n, fs = 1 << 14, 1024.0
    mc, eta = map(float, synth.mc_eta(1.4, 1.4))
    g = O.grid(n, fs)
    Sn = O.psd_bins(n, fs, 40.0)
    hc = O.spa_template(n, fs, 40.0, mc, eta)
    hs = O.quadrature_partner(hc)
    inv = np.where(np.isfinite(Sn), 1.0 / Sn, 0.0)
    inner = 4 * g["df"] * np.real(np.sum(hc * np.conj(hs) * inv))
    norm = O.sigma_sq(hc, Sn, g["df"])
    assert abs(inner) < 1e-14 * norm
    assert O.sigma_sq(hs, Sn, g["df"]) == pytest.approx(norm, rel=1e-14)


def test_phase_offset_half_pi_gives_quadrature_partner():
    # Sec. 1.1: the alpha = 0 and alpha = pi/2 templates are h_c and h_s with
    # h_c = -i h_s, i.e. the pi/2-offset template is i h_c.
    n, fs = 1 << 13, 1024.0
    mc, eta = map(float, synth.mc_eta(1.2, 2.2))
    hc = O.spa_template(n, fs, 40.0, mc, eta, phic=0.0)
    hs = O.spa_template(n, fs, 40.0, mc, eta, phic=math.pi / 2)
    np.testing.assert_allclose(hc, -1j * hs, atol=1e-15 * np.max(np.abs(hc)))


def test_z_is_x_plus_iy_from_two_real_filters():
    n, fs = 1 << 14, 1024.0
    mc, eta = map(float, synth.mc_eta(1.4, 1.4))
    s, Sn, g = _noise_segment(n, fs, 11, injection=(mc, eta, 12.0, 1234, 0.7))
    hc = O.spa_template(n, fs, 40.0, mc, eta)
    hs = O.quadrature_partner(hc)
    z = O.filter_z(s, Sn, hc, n, g["df"])
    x = _real_filter(hc, s, Sn, n, g["df"])
    y = _real_filter(hs, s, Sn, n, g["df"])
    scale = np.max(np.abs(z))
    np.testing.assert_allclose(z.real, x, atol=1e-12 * scale)
    np.testing.assert_allclose(z.imag, y, atol=1e-12 * scale)
    # The printed conjugate placement is the time reversal of the same series.
    zl = O.filter_z_literal(s, Sn, hc, n, g["df"])
    rev = (-np.arange(n)) % n
    np.testing.assert_allclose(zl, np.conj(z[rev]), atol=1e-12 * scale)


# ---------------------------------------------------------------------------
# FFT convention: brute force, Parseval, impulse
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [8, 64, 512])
def test_inverse_dft_matches_naive(n):
    rng = np.random.default_rng(n)
    q = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    got = O.inverse_dft(q)
    ref = O.naive_dft(q, +1)
    # naive DFT brute force: explicit double loop for the smallest size
    if n == 8:
        brute = np.array([sum(q[k] * complex(math.cos(2 * math.pi * j * k / n), math.sin(2 * math.pi * j * k / n))
                              for k in range(n)) for j in range(n)])
        np.testing.assert_allclose(ref, brute, atol=1e-12)
    np.testing.assert_allclose(got, ref, atol=1e-12 * n)


def test_parseval_and_impulse():
    n = 1 << 12
    rng = np.random.default_rng(3)
    q = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    z = O.inverse_dft(q)
    assert np.sum(np.abs(z) ** 2) == pytest.approx(n * np.sum(np.abs(q) ** 2), rel=1e-12)
    k0 = 37
    d = np.zeros(n, complex)
    d[k0] = 1.0
    j = np.arange(n)
    np.testing.assert_allclose(O.inverse_dft(d), np.exp(2j * np.pi * j * k0 / n), atol=1e-12)


# ---------------------------------------------------------------------------
# Eq. (4): Riemann sum against adaptive quadrature of the continuous integral
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,fs,m", [(1 << 16, 2048.0, 1.4), (1 << 20, 4096.0, 1.4), (1 << 20, 4096.0, 10.0)])
def test_sigma_against_quadrature(n, fs, m):
    integrate = pytest.importorskip("scipy.integrate")
    mc, eta = map(float, synth.mc_eta(m, m))
    g = O.grid(n, fs)
    Sn = O.psd_bins(n, fs, 40.0)
    h = O.spa_template(n, fs, 40.0, mc, eta)
    k_lo, k_hi = O.band(n, fs, 40.0, mc, eta)
    s2 = O.sigma_sq(h, Sn, g["df"])

    def integrand(f):
        return 4.0 * f ** (-7.0 / 3.0) / O.psd_initial_ligo(f)
    f_lo, f_hi = k_lo * g["df"], k_hi * g["df"]
    val, _ = integrate.quad(integrand, f_lo, f_hi, limit=400, epsabs=0, epsrel=1e-13)
    # Trapezoid end corrections turn the bin sum into an O(df^2) estimate.
    trap = s2 - 0.5 * g["df"] * (integrand(f_lo) + integrand(f_hi))
    assert trap == pytest.approx(val, rel=1e-7)


# ---------------------------------------------------------------------------
# Eq. (1)-(3) end to end: noiseless injection, Cauchy-Schwarz, noise statistics
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("j0,phi0", [(0, 0.0), (4321, 1.1), (65535, 5.9)])
def test_noiseless_injection_recovers_snr(j0, phi0):
    n, fs = 1 << 16, 2048.0
    mc, eta = map(float, synth.mc_eta(1.4, 1.4))
    g = O.grid(n, fs)
    Sn = O.psd_bins(n, fs, 40.0)
    h = O.spa_template(n, fs, 40.0, mc, eta)
    sig = math.sqrt(O.sigma_sq(h, Sn, g["df"]))
    s = synth.inject(np.zeros(n // 2 + 1, complex), h, 10.0 / sig, phi0, j0, n)
    out = O.filter_unit(n, fs, 40.0, mc, eta, s, Sn, threshold=9.99, return_series=True)
    assert out["j"] == j0
    assert out["rho"] == pytest.approx(10.0, rel=1e-12)
    assert np.all(out["series"] <= 10.0 * (1 + 1e-12))
    assert out["n_above"] >= 1
    zl = O.filter_z_literal(s, Sn, h, n, g["df"])
    assert int(np.argmax(np.abs(zl))) == (n - j0) % n


def test_noise_only_rho_squared_mean_is_two():
    n, fs = 1 << 14, 1024.0
    mc, eta = map(float, synth.mc_eta(1.4, 1.4))
    vals = []
    for seed in range(12):
        s, Sn, g = _noise_segment(n, fs, 1000 + seed)
        out = O.filter_unit(n, fs, 40.0, mc, eta, s, Sn, return_series=True)
        vals.append(np.mean(out["series"] ** 2))
    assert np.mean(vals) == pytest.approx(2.0, rel=0.03)


def test_peak_tie_break_and_window():
    rho = np.array([0.0, 3.0, 1.0, 3.0, 2.0, 3.0])
    assert O.peak(rho) == (3.0, 1, 0)
    assert O.peak(rho, threshold=2.0) == (3.0, 1, 4)
    assert O.peak(rho, j_begin=2, j_end=5) == (3.0, 3, 0)


def test_bank_mirror_pairs_identical():
    n, fs = 1 << 14, 1024.0
    s, Sn, g = _noise_segment(n, fs, 5)
    a = synth.mc_eta(1.0, 3.0)
    b = synth.mc_eta(3.0, 1.0)
    assert a[0] == b[0] and a[1] == b[1]
    oa = O.filter_unit(n, fs, 40.0, float(a[0]), float(a[1]), s, Sn)
    ob = O.filter_unit(n, fs, 40.0, float(b[0]), float(b[1]), s, Sn)
    assert oa == ob


# ---------------------------------------------------------------------------
# Gradient of rho^2
# ---------------------------------------------------------------------------
def _grad_case(noise=True):
    n, fs = 1 << 14, 1024.0
    mc, eta = map(float, synth.mc_eta(1.6, 1.3))
    j0 = 5000
    if noise:
        s, Sn, g = _noise_segment(n, fs, 21, injection=(mc, eta, 15.0, j0, 0.4))
    else:
        g = O.grid(n, fs)
        Sn = O.psd_bins(n, fs, 40.0)
        h = O.spa_template(n, fs, 40.0, mc, eta)
        sig = math.sqrt(O.sigma_sq(h, Sn, g["df"]))
        s = synth.inject(np.zeros(n // 2 + 1, complex), h, 15.0 / sig, 0.4, j0, n)
    k_lo, k_hi = O.band(n, fs, 40.0, mc, eta)
    return n, fs, mc, eta, j0 * g["dt"], s, Sn, k_lo, k_hi


def test_gradient_matches_finite_differences():
    n, fs, mc, eta, t0, s, Sn, k_lo, k_hi = _grad_case()
    theta = (mc * 1.0003, eta * 0.999, t0 + 2e-4)
    F, Z, grad = O.snr_sq(theta, s, Sn, n, fs, k_lo, k_hi, with_grad=True)
    fd = O.snr_sq_fd_grad(theta, s, Sn, n, fs, k_lo, k_hi)
    D = np.array([theta[0] * 1e-3, 1e-3, 1e-4])
    assert np.linalg.norm(D * (grad - fd)) <= 1e-5 * np.linalg.norm(D * fd) + 1e-9 * F
    np.testing.assert_allclose(grad, fd, rtol=1e-4)


def test_gradient_vanishes_at_noiseless_injection():
    n, fs, mc, eta, t0, s, Sn, k_lo, k_hi = _grad_case(noise=False)
    F, Z, grad = O.snr_sq((mc, eta, t0), s, Sn, n, fs, k_lo, k_hi, with_grad=True)
    assert F == pytest.approx(225.0, rel=1e-12)
    D = np.array([mc * 1e-3, 1e-3, 1e-4])
    assert np.linalg.norm(D * grad) < 1e-8 * F
    # A displaced point has a clearly non-zero gradient that points back.
    F2, _, g2 = O.snr_sq((mc, eta, t0 + 3e-4), s, Sn, n, fs, k_lo, k_hi, with_grad=True)
    assert F2 < F and g2[2] < 0


def test_snr_sq_equals_filter_output_at_sample_time():
    n, fs, mc, eta, t0, s, Sn, k_lo, k_hi = _grad_case()
    g = O.grid(n, fs)
    h = O.spa_template(n, fs, 40.0, mc, eta)
    z = O.filter_z(s, Sn, h, n, g["df"])
    sig2 = O.sigma_sq(h, Sn, g["df"])
    j = 4097
    F, Z, _ = O.snr_sq((mc, eta, j * g["dt"]), s, Sn, n, fs, k_lo, k_hi)
    assert Z == pytest.approx(complex(z[j]), rel=1e-10)
    assert F == pytest.approx(abs(z[j]) ** 2 / sig2, rel=1e-10)


def test_template_metric_predicts_the_quadratic_falloff():
    """Noiseless injection: 1 - F(theta*+delta)/F* = delta^T g delta + O(delta^3),
    checked against direct evaluations of F along several directions."""
    n, fs, mc, eta, t0, s, Sn, k_lo, k_hi = _grad_case(noise=False)
    g = O.template_metric((mc, eta, t0), Sn, n, fs, k_lo, k_hi)
    assert np.all(np.linalg.eigvalsh(g) > 0)
    Fs = O.snr_sq((mc, eta, t0), s, Sn, n, fs, k_lo, k_hi)[0]
    scales = np.array([mc * 2e-5, 2e-5, 2e-6])
    for direction in ([1, 0, 0], [0, 1, 0], [0, 0, 1], [1, -1, 0], [1, 1, 1]):
        dlt = np.array(direction, float) * scales
        F = O.snr_sq((mc + dlt[0], eta + dlt[1], t0 + dlt[2]), s, Sn, n, fs, k_lo, k_hi)[0]
        pred = dlt @ g @ dlt
        assert 1.0 - F / Fs == pytest.approx(pred, rel=2e-2), direction


# ---------------------------------------------------------------------------
# Eq. (5): chi^2 veto
# ---------------------------------------------------------------------------
def _chisq_case(noise, snr=12.0, j0=7000, m=(1.4, 1.4), seed=41):
    n, fs = 1 << 14, 1024.0
    mc, eta = map(float, synth.mc_eta(*m))
    if noise:
        s, Sn, g = _noise_segment(n, fs, seed, injection=(mc, eta, snr, j0, 0.3) if snr else None)
    else:
        g = O.grid(n, fs)
        Sn = O.psd_bins(n, fs, 40.0)
        h = O.spa_template(n, fs, 40.0, mc, eta)
        sig = math.sqrt(O.sigma_sq(h, Sn, g["df"]))
        s = synth.inject(np.zeros(n // 2 + 1, complex), h, snr / sig, 0.3, j0, n)
    h = O.spa_template(n, fs, 40.0, mc, eta)
    k_lo, k_hi = O.band(n, fs, 40.0, mc, eta)
    return n, fs, s, Sn, g, h, k_lo, k_hi


def test_chisq_band_edges_split_sigma_equally():
    n, fs, s, Sn, g, h, k_lo, k_hi = _chisq_case(noise=False)
    for p in (2, 4, 16):
        e = O.chisq_band_edges(Sn, n, fs, k_lo, k_hi, p)
        assert e[0] == k_lo and e[-1] == k_hi + 1 and np.all(np.diff(e) > 0)
        f = O.freqs(n, fs)
        W = np.zeros(n // 2 + 1)
        W[k_lo: k_hi + 1] = f[k_lo: k_hi + 1] ** (-7.0 / 3.0) / Sn[k_lo: k_hi + 1]
        shares = np.array([W[e[l]: e[l + 1]].sum() for l in range(p)]) / W.sum()
        # each band's share is 1/p up to one bin's weight
        assert np.all(np.abs(shares - 1.0 / p) <= W.max() / W.sum() + 1e-15)


def test_chisq_noiseless_injection_closed_form():
    # s = A e^{i phi} h shifted to j0: z_l(j0) = A e^{i phi} sigma_l^2, so
    # chi^2(j0) = p A^2 / sigma^2 sum_l (sigma_l^2 - sigma^2 / p)^2 (~0: equal bands).
    p = 16
    n, fs, s, Sn, g, h, k_lo, k_hi = _chisq_case(noise=False)
    chi2, zl = O.chisq_series(s, Sn, h, n, fs, k_lo, k_hi, p)
    e = O.chisq_band_edges(Sn, n, fs, k_lo, k_hi, p)
    inv = np.where(np.isfinite(Sn), 1.0 / Sn, 0.0)
    sl2 = np.array([4 * g["df"] * np.sum(np.abs(h[e[l]: e[l + 1]]) ** 2 * inv[e[l]: e[l + 1]]) for l in range(p)])
    s2 = sl2.sum()
    A = 12.0 / math.sqrt(s2)
    closed = p * A * A / s2 * np.sum((sl2 - s2 / p) ** 2)
    assert chi2[7000] == pytest.approx(closed, rel=1e-9, abs=1e-12)
    assert chi2[7000] < 1e-3
    np.testing.assert_allclose(np.abs(zl[:, 7000]), A * sl2, rtol=1e-10)


def test_chisq_bands_sum_to_filter_output():
    n, fs, s, Sn, g, h, k_lo, k_hi = _chisq_case(noise=True)
    chi2, zl = O.chisq_series(s, Sn, h, n, fs, k_lo, k_hi, 8)
    z = O.filter_z(s, Sn, h, n, g["df"])
    np.testing.assert_allclose(zl.sum(axis=0), z, atol=1e-12 * np.abs(z).max())


def test_chisq_noise_mean_is_2p_minus_2():
    # Sec. 1.2: in stationary Gaussian noise chi^2 has nu = 2p - 2 degrees of freedom.
    p = 16
    vals = []
    for seed in range(6):
        n, fs, s, Sn, g, h, k_lo, k_hi = _chisq_case(noise=True, snr=0.0, seed=300 + seed)
        chi2, _ = O.chisq_series(s, Sn, h, n, fs, k_lo, k_hi, p)
        vals.append(chi2.mean())
    assert np.mean(vals) == pytest.approx(2 * p - 2, rel=0.03)


def test_chisq_flags_a_mismatched_glitch():
    # A loud signal that is a poor match (another template) leaves a large chi^2
    # at the peak of the filter output, while a matched signal does not.
    p = 16
    n, fs, s, Sn, g, h, k_lo, k_hi = _chisq_case(noise=True, snr=0.0, seed=77)
    mc2, eta2 = map(float, synth.mc_eta(6.0, 1.1))
    h2 = O.spa_template(n, fs, 40.0, mc2, eta2)
    glitch = synth.inject(s, h2, 80.0 / math.sqrt(O.sigma_sq(h2, Sn, g["df"])), 0.0, 5000, n)
    matched = synth.inject(s, h, 80.0 / math.sqrt(O.sigma_sq(h, Sn, g["df"])), 0.0, 5000, n)
    chi2, zl = O.chisq_series(glitch, Sn, h, n, fs, k_lo, k_hi, p)
    assert chi2[int(np.argmax(np.abs(zl.sum(axis=0))))] > 5 * (2 * p - 2)
    chi2, zl = O.chisq_series(matched, Sn, h, n, fs, k_lo, k_hi, p)
    assert chi2[int(np.argmax(np.abs(zl.sum(axis=0))))] < 2 * (2 * p - 2)


# ---------------------------------------------------------------------------
# Time-domain input (R8) and caller-supplied PSD
# ---------------------------------------------------------------------------
def test_segment_spectrum_matches_explicit_double_loop():
    rng = np.random.default_rng(7)
    n, fs = 48, 16.0
    x = rng.standard_normal(n)
    want = np.zeros(n // 2 + 1, dtype=np.complex128)
    for k in range(n // 2 + 1):
        acc = 0.0 + 0.0j
        for j in range(n):
            acc += x[j] * complex(math.cos(2 * math.pi * j * k / n), -math.sin(2 * math.pi * j * k / n))
        want[k] = acc / fs
    got = O.segment_spectrum(x, fs)
    assert np.max(np.abs(got - want)) < 1e-12


def test_segment_spectrum_of_a_tone_and_parseval():
    n, fs, k0 = 1 << 12, 512.0, 301
    j = np.arange(n)
    x = 2.5 * np.cos(2 * np.pi * k0 * j / n + 0.4)
    s = O.segment_spectrum(x, fs)
    # a real tone at bin k0 puts A N/2 e^{i phi} dt into bin k0 and nothing elsewhere
    assert abs(s[k0] - 2.5 * n / 2 * np.exp(0.4j) / fs) < 1e-9
    others = np.delete(s, k0)
    assert np.max(np.abs(others)) < 1e-9
    rng = np.random.default_rng(8)
    y = rng.standard_normal(n)
    X = O.segment_spectrum(y, fs) * fs
    energy = (abs(X[0]) ** 2 + abs(X[-1]) ** 2 + 2 * np.sum(np.abs(X[1:-1]) ** 2)) / n
    assert energy == pytest.approx(np.sum(y ** 2), rel=1e-12)


def test_prefix_sums_give_sigma_and_ignore_out_of_band_values():
    n, fs, f_low = 1 << 14, 1024.0, 40.0
    Sn = O.psd_bins(n, fs, f_low)
    P = O.prefix_sums(Sn, n, fs)
    mc, eta = map(float, synth.mc_eta(1.4, 1.4))
    k_lo, k_hi = O.band(n, fs, f_low, mc, eta)
    h = O.spa_template(n, fs, f_low, mc, eta)
    assert 4 * (fs / n) * (P[k_hi] - P[k_lo - 1]) == pytest.approx(O.sigma_sq(h, Sn, fs / n), rel=1e-12)
    assert np.all(P[:k_lo] == 0.0) and np.all(np.diff(P) >= 0.0)
    # a full-range user PSD restricted to the band equals the band-limited one
    f = O.freqs(n, fs)
    user = np.empty(n // 2 + 1)
    user[1:] = O.psd_initial_ligo(f[1:])
    user[0] = 1.0
    R = O.psd_from_array(user, n, fs, f_low)
    assert np.array_equal(np.isinf(R), np.isinf(Sn))
    fin = np.isfinite(Sn)
    assert np.max(np.abs(R[fin] / Sn[fin] - 1.0)) < 1e-15


# ---------------------------------------------------------------------------
# Events (R17): hand-built series with their event lists worked out by hand
# ---------------------------------------------------------------------------
def test_unit_events_isolated_peak_and_threshold():
    rho = np.zeros(64)
    rho[10] = 6.0
    rho[40] = 4.0
    assert O.unit_events(rho, 5.0, 16) == [(0, 10, 6.0)]
    assert O.unit_events(rho, 3.5, 16) == [(0, 10, 6.0), (2, 40, 4.0)]
    assert O.unit_events(rho, 7.0, 16) == []


def test_unit_events_merge_across_a_window_edge():
    W = 16
    rho = np.zeros(64)
    rho[15], rho[16] = 8.0, 7.0      # one signal split by the edge at 16: only j = 15 survives
    rho[47], rho[48] = 5.0, 9.0      # the later sample wins here
    assert O.unit_events(rho, 4.0, W) == [(0, 15, 8.0), (3, 48, 9.0)]
    # farther apart than W: both windows keep their winners
    rho2 = np.zeros(64)
    rho2[2], rho2[30] = 8.0, 7.0
    assert O.unit_events(rho2, 4.0, W) == [(0, 2, 8.0), (1, 30, 7.0)]
    # equal values within W: the lower index survives; lowest index inside a window on ties
    rho3 = np.zeros(64)
    rho3[20], rho3[25], rho3[33] = 6.0, 6.0, 6.0
    assert O.unit_events(rho3, 4.0, W) == [(1, 20, 6.0)]


def test_unit_events_properties_on_noise():
    rng = np.random.default_rng(11)
    W = 32
    for _ in range(20):
        rho = np.abs(rng.standard_normal(1024) + 1j * rng.standard_normal(1024))
        ev = O.unit_events(rho, 2.5, W)
        js, vals = O.window_maxima(rho, W)
        for (w, j, v) in ev:
            seg = rho[w * W: (w + 1) * W]
            assert v == seg.max() and j == w * W + int(np.argmax(seg)) and v >= 2.5
        # kept events are more than W apart; a dropped window winner above threshold is
        # beaten by an adjacent winner within W
        ej = [j for (_, j, _) in ev]
        assert all(b - a > W for a, b in zip(ej, ej[1:]))
        kept = {w for (w, _, _) in ev}
        for w in range(len(js)):
            if vals[w] >= 2.5 and w not in kept:
                assert any(0 <= w2 < len(js) and abs(js[w2] - js[w]) <= W and
                           (vals[w2] > vals[w] or (vals[w2] == vals[w] and js[w2] < js[w])) for w2 in (w - 1, w + 1))


def test_segment_events_pick_loudest_template_then_merge():
    n, W = 64, 16
    ev = {0: [(0, 3, 6.0), (2, 40, 5.0)],
          1: [(0, 5, 7.0), (3, 49, 6.0)],
          2: [(2, 41, 5.0)]}
    # window 0: template 1 (7.0); window 2: tie 5.0 -> template 0; window 3: 6.0 at 49 beats 5.0 at 40
    assert O.segment_events(ev, n, 4.0, W) == [(0, 1, 5, 7.0), (3, 1, 49, 6.0)]
