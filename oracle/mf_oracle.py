"""Plain FP64 oracle of the frequency-domain matched filter (test infrastructure).

Sections of arXiv:0906.4175 followed here:

* Sec. 1.1, Eq. (1): complex filter output z(t) = x(t) + i y(t) as a one-sided
  integral of template x data / PSD, inverse-transformed to time.
* Sec. 1.1, Eq. (2): initial-LIGO analytic one-sided PSD S_n(f), f0 = 150 Hz.
* Sec. 1.1, Eq. (3): SNR rho(t) = |z(t)| / sigma, maximised over phase.
* Sec. 1.1, Eq. (4): template norm sigma^2 = 4 int |h_c|^2 / S_n df.
* Sec. 1.1 (template paragraph): spinless circular binaries, 2PN orbital phase,
  Newtonian amplitude; parameters (m1, m2), phase offset, effective distance.
* Sec. 1.1 (cutoff paragraph): f_low = 40 Hz; f_high = min(Nyquist, f_ISCO).
* Sec. 1.1 (segment paragraph): 256 s at 4096 Hz, 2^20 samples.

Readings taken where the paper is silent or ambiguous (each one is also a
documented design decision of the HIP path):

R1  Conjugate placement in Eq. (1).  The printed integrand is h_c * conj(s).
    With h_c = -i h_s and "x = response of h_c, y = response of h_s", only
    conj(h_c) * s gives z = x + i y; the printed form is its time reversal
    (z_lit[j] = conj(z[-j mod N])).  The oracle computes the standard form in
    :func:`filter_z` and keeps the printed one in :func:`filter_z_literal`.
R2  Eq. (2) carries no overall scale; S_0 = 1 (rho is scale invariant).
R3  S_n is evaluated only on the band bins k_lo..N/2-1; 1/S_n = 0 elsewhere.
R4  SPA template (stationary-phase, 2PN phase, Newtonian amplitude, from the
    template references the paper cites): h_c(f) = f^(-7/6) exp(-i Psi(f)),
    Psi(f) = 2 pi f t_c - phi_c - pi/4 + 3/(128 eta v^5) [1 + (3715/756 +
    55 eta/9) v^2 - 16 pi v^3 + (15293365/508032 + 27145 eta/504 +
    3085 eta^2/72) v^4],  v = (pi M f)^(1/3).  Distance/amplitude constants are
    dropped (rho does not depend on them).
R5  f_ISCO = 1 / (6^(3/2) pi M) (Schwarzschild test-mass ISCO, GW frequency).
R6  T_sun = G M_sun / c^3 = 4.925490947641267e-6 s (IAU 2015 nominal GM_sun).
R7  Bins: k_lo = ceil(f_low T); k_hi = min(floor(f_ISCO T), N/2 - 1).  DC and
    Nyquist are always excluded; an empty band is an error.
R8  Discretisation: s~_k = dt sum_j s_j e^{-2 pi i jk/N}; int df -> df sum_k.
R9  Negative frequencies carry zero (one-sided integral), so z is complex.
R10 rho is computed over all N circular lags; an optional window restricts
    the peak search.
R11 Peak: lowest j attaining the maximum; n_above counts rho_j >= threshold.
R12 Bank templates use t_c = phi_c = 0 (the IFFT scans time, |z| maximises
    over phase).
R13 Gradient of rho^2 w.r.t. (M_c, eta, t_c): the band K is frozen at the
    starting template; F(theta) = |Z(theta)|^2 / sigma^2 with
    Z = 4 df sum_K a_k exp(+i Psi_k(theta)) s_k / S_k, which is z(t) at the
    continuous time t = t_c.
R16 chi^2 bands (Eq. (5), Sec. 1.2): p contiguous bands of the template's
    band with equal shares of sigma^2; a bin belongs to the band in which the
    W-sum of the bins before it falls (W_k = f_k^(-7/3) / S_k).
R17 Events (Sec. 3.3 names events with their SNR and chi^2 but gives no
    threshold or clustering rule): the series is cut into windows of W
    samples; a window's winner is its maximum of rho (lowest index on ties);
    it is an event if rho >= rho_th and the winner of neither adjacent window
    lies within W samples of it with a larger rho (or an equal rho at a lower
    index).  Across the templates of one segment the same rule runs on the
    loudest unit event of each window (ties: lowest template index).
"""
from __future__ import annotations

import math

import numpy as np

# R6: G M_sun / c^3 in seconds (IAU 2015 nominal solar mass parameter).
T_SUN = 4.925490947641267e-6
# Eq. (2): knee frequency of the initial-LIGO analytic PSD.
PSD_F0 = 150.0


# ---------------------------------------------------------------------------
# Grid (Sec. 1.1 segment paragraph; reading R8)
# ---------------------------------------------------------------------------
def grid(n: int, fs: float) -> dict:
    """Sample spacing, duration and frequency resolution of an N-point segment."""
    dt = 1.0 / fs
    T = n * dt
    df = 1.0 / T
    return {"n": int(n), "fs": float(fs), "dt": dt, "T": T, "df": df}


def freqs(n: int, fs: float) -> np.ndarray:
    """f_k = k df for the one-sided bins k = 0..N/2."""
    g = grid(n, fs)
    return np.arange(n // 2 + 1, dtype=np.float64) * g["df"]


# ---------------------------------------------------------------------------
# Eq. (2): analytic initial-LIGO PSD (readings R2, R3)
# ---------------------------------------------------------------------------
def psd_initial_ligo(f, f0: float = PSD_F0):
    """S_n(f) of Eq. (2), dimensionless (S_0 = 1).  f must be > 0."""
    x = np.asarray(f, dtype=np.float64) / f0
    return (4.49 * x) ** (-56.0) + 0.16 * x ** (-4.52) + 0.52 + 0.32 * x * x


def psd_bins(n: int, fs: float, f_low: float, f0: float = PSD_F0) -> np.ndarray:
    """S_n on the one-sided bins, +inf outside the band [k_lo, N/2-1] (R3)."""
    k_lo = band_lo(n, fs, f_low)
    S = np.full(n // 2 + 1, np.inf)
    f = freqs(n, fs)
    S[k_lo: n // 2] = psd_initial_ligo(f[k_lo: n // 2], f0)
    return S


def psd_from_array(S_user, n: int, fs: float, f_low: float) -> np.ndarray:
    """A caller-supplied one-sided PSD on the bins, restricted to the band (R3):
    S_k inside [k_lo, N/2-1], +inf elsewhere, so that 1/S_k = 0 outside."""
    S_user = np.asarray(S_user, dtype=np.float64)
    if S_user.shape != (n // 2 + 1,):
        raise ValueError("PSD must have N/2+1 one-sided bins")
    k_lo = band_lo(n, fs, f_low)
    S = np.full(n // 2 + 1, np.inf)
    S[k_lo: n // 2] = S_user[k_lo: n // 2]
    return S


def prefix_sums(Sn: np.ndarray, n: int, fs: float) -> np.ndarray:
    """P_k = sum_{1 <= k' <= k} f_k'^(-7/3) / S_k' over the bins where S is finite:
    the running form of the Eq. (4) sum, so sigma^2 of a template on
    [k_lo, k_hi] is 4 df (P[k_hi] - P[k_lo - 1])."""
    f = freqs(n, fs)
    W = np.zeros(n // 2 + 1)
    ok = np.isfinite(Sn)
    ok[0] = False
    W[ok] = f[ok] ** (-7.0 / 3.0) / Sn[ok]
    return np.cumsum(W)


# ---------------------------------------------------------------------------
# Time-domain input (reading R8): one-sided spectrum of a real segment
# ---------------------------------------------------------------------------
def segment_spectrum(x: np.ndarray, fs: float) -> np.ndarray:
    """s_k = dt sum_j x_j e^{-2 pi i jk/N} for k = 0..N/2 (R8) of a real segment x[N]."""
    x = np.asarray(x, dtype=np.float64)
    return np.fft.rfft(x) / fs


# ---------------------------------------------------------------------------
# Frequency band (Sec. 1.1 cutoff paragraph; readings R5, R7)
# ---------------------------------------------------------------------------
def total_mass_from_mc_eta(mc: float, eta: float) -> float:
    """Total mass [M_sun] from chirp mass and symmetric mass ratio."""
    return mc * eta ** (-0.6)


def f_isco(m_total_sun: float) -> float:
    """GW frequency at the Schwarzschild innermost stable circular orbit (R5)."""
    M = m_total_sun * T_SUN
    return 1.0 / (math.sqrt(216.0) * math.pi * M)


def band_lo(n: int, fs: float, f_low: float) -> int:
    T = n / fs
    return int(math.ceil(f_low * T))


def band(n: int, fs: float, f_low: float, mc: float, eta: float) -> tuple[int, int]:
    """(k_lo, k_hi) of the template's band: f_low up to min(f_ISCO, Nyquist)."""
    T = n / fs
    k_lo = band_lo(n, fs, f_low)
    k_isco = int(math.floor(f_isco(total_mass_from_mc_eta(mc, eta)) * T))
    k_hi = min(k_isco, n // 2 - 1)
    if k_hi < k_lo:
        raise ValueError(f"empty band: k_lo={k_lo} k_hi={k_hi}")
    return k_lo, k_hi


# ---------------------------------------------------------------------------
# SPA template (Sec. 1.1 template paragraph; reading R4)
# ---------------------------------------------------------------------------
def spa_phase(f, mc: float, eta: float, tc: float = 0.0, phic: float = 0.0):
    """Psi(f): 2PN stationary-phase phase of a circular spinless inspiral.

    Written in the post-Newtonian velocity v = (pi M f)^(1/3), term by term as
    in the 2PN template literature the paper cites.  Accepts complex f so that
    tests can take complex-step derivatives.
    """
    M = total_mass_from_mc_eta(mc, eta) * T_SUN
    f = np.asarray(f)
    v = (np.pi * M * f) ** (1.0 / 3.0)
    pn2 = 3715.0 / 756.0 + 55.0 * eta / 9.0
    pn3 = -16.0 * np.pi
    pn4 = 15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta * eta / 72.0
    series = 1.0 + pn2 * v ** 2 + pn3 * v ** 3 + pn4 * v ** 4
    return 2.0 * np.pi * f * tc - phic - np.pi / 4.0 + 3.0 / (128.0 * eta * v ** 5) * series


def spa_amplitude(f):
    """Newtonian SPA amplitude f^(-7/6) (constant factors dropped, R4)."""
    return np.asarray(f, dtype=np.float64) ** (-7.0 / 6.0)


def spa_template(n: int, fs: float, f_low: float, mc: float, eta: float,
                 tc: float = 0.0, phic: float = 0.0, k_hi: int | None = None) -> np.ndarray:
    """h~_c on the one-sided bins k = 0..N/2: f^(-7/6) e^{-i Psi} in band, 0 outside."""
    k_lo, k_hi_default = band(n, fs, f_low, mc, eta)
    if k_hi is None:
        k_hi = k_hi_default
    f = freqs(n, fs)
    h = np.zeros(n // 2 + 1, dtype=np.complex128)
    fb = f[k_lo: k_hi + 1]
    h[k_lo: k_hi + 1] = spa_amplitude(fb) * np.exp(-1j * spa_phase(fb, mc, eta, tc, phic))
    return h


def quadrature_partner(h_c: np.ndarray) -> np.ndarray:
    """h~_s from h~_c = -i h~_s (Sec. 1.1, quadrature pair)."""
    return 1j * h_c


# ---------------------------------------------------------------------------
# Eq. (4): template norm
# ---------------------------------------------------------------------------
def sigma_sq(htilde: np.ndarray, Sn: np.ndarray, df: float) -> float:
    """sigma^2 = 4 df sum_k |h_k|^2 / S_k over the bins where S_k is finite."""
    inv = np.where(np.isfinite(Sn), 1.0 / Sn, 0.0)
    return float(4.0 * df * np.sum(np.abs(htilde) ** 2 * inv))


# ---------------------------------------------------------------------------
# Eq. (1): complex filter output (readings R1, R8, R9)
# ---------------------------------------------------------------------------
def _one_sided_to_full(q_half: np.ndarray, n: int) -> np.ndarray:
    """Place one-sided bins 0..N/2 into an N-point spectrum, zero for k >= N/2 (R9)."""
    q = np.zeros(n, dtype=np.complex128)
    q[: n // 2] = q_half[: n // 2]
    return q


def inverse_dft(q: np.ndarray) -> np.ndarray:
    """sum_k q_k e^{+2 pi i jk/N} (unnormalised), via numpy's ifft."""
    n = q.shape[-1]
    return n * np.fft.ifft(q)


def filter_z(stilde: np.ndarray, Sn: np.ndarray, htilde: np.ndarray, n: int, df: float) -> np.ndarray:
    """z_j = 4 df sum_k conj(h_k) s_k / S_k e^{2 pi i jk/N}  (Eq. (1), reading R1)."""
    inv = np.where(np.isfinite(Sn), 1.0 / Sn, 0.0)
    q_half = np.conj(htilde) * stilde.astype(np.complex128) * inv
    return 4.0 * df * inverse_dft(_one_sided_to_full(q_half, n))


def filter_z_literal(stilde: np.ndarray, Sn: np.ndarray, htilde: np.ndarray, n: int, df: float) -> np.ndarray:
    """Eq. (1) exactly as printed: integrand h_c conj(s) / S_n."""
    inv = np.where(np.isfinite(Sn), 1.0 / Sn, 0.0)
    q_half = htilde * np.conj(stilde.astype(np.complex128)) * inv
    return 4.0 * df * inverse_dft(_one_sided_to_full(q_half, n))


# ---------------------------------------------------------------------------
# Eq. (3) and the peak / threshold reduction (readings R10, R11)
# ---------------------------------------------------------------------------
def snr(z: np.ndarray, sigma: float) -> np.ndarray:
    return np.abs(z) / sigma


def peak(rho: np.ndarray, threshold: float = math.inf, j_begin: int = 0, j_end: int | None = None):
    """(rho_max, j*, n_above) over the window [j_begin, j_end); lowest j on ties."""
    if j_end is None:
        j_end = rho.shape[-1]
    w = rho[j_begin:j_end]
    j = int(np.argmax(w))  # numpy returns the first (lowest) index of the maximum
    n_above = int(np.count_nonzero(w >= threshold))
    return float(w[j]), j + j_begin, n_above


def filter_unit(n: int, fs: float, f_low: float, mc: float, eta: float,
                stilde: np.ndarray, Sn: np.ndarray, threshold: float = math.inf,
                return_series: bool = False):
    """One (template, segment) unit end to end: template, sigma, z, rho, peak."""
    g = grid(n, fs)
    h = spa_template(n, fs, f_low, mc, eta)
    sig = math.sqrt(sigma_sq(h, Sn, g["df"]))
    z = filter_z(stilde, Sn, h, n, g["df"])
    rho = snr(z, sig)
    rmax, j, n_above = peak(rho, threshold)
    out = {"sigma": sig, "rho": rmax, "j": j, "n_above": n_above}
    if return_series:
        out["series"] = rho
        out["z"] = z
    return out


# ---------------------------------------------------------------------------
# Eq. (5): chi^2 time-frequency veto (Sec. 1.2)
# ---------------------------------------------------------------------------
def chisq_band_edges(Sn: np.ndarray, n: int, fs: float, k_lo: int, k_hi: int, p: int) -> np.ndarray:
    """Edges e_0 = k_lo < ... < e_p = k_hi + 1 of p bands that contribute equally to sigma^2.

    Reading R16: with W_k = f_k^(-7/3) / S_k (the integrand of Eq. (4)) and the
    sum of W over the bins before k, bin k belongs to the band in which that
    sum falls: e_l = min{k : sum_{k_lo <= k' < k} W_k' >= l / p * sum_band W}.
    """
    f = freqs(n, fs)[k_lo: k_hi + 1]
    W = f ** (-7.0 / 3.0) / Sn[k_lo: k_hi + 1]
    before = np.concatenate([[0.0], np.cumsum(W)[:-1]])
    total = float(np.sum(W))
    edges = [k_lo]
    for l in range(1, p):
        hit = np.nonzero(before >= l / p * total)[0]
        # no bin starts at or past this share: band l and those above are empty
        edges.append(k_lo + int(hit[0]) if hit.size else k_hi + 1)
    edges.append(k_hi + 1)
    return np.array(edges, dtype=np.int64)


def chisq_series(stilde: np.ndarray, Sn: np.ndarray, htilde: np.ndarray, n: int, fs: float, k_lo: int, k_hi: int,
                 p: int = 16):
    """chi^2(t) = p / sigma^2 sum_l |z_l(t) - z(t)/p|^2 over all N lags (Eq. (5)).

    z_l is Eq. (1) restricted to band l; returns (chi2 [N], z_l [p, N]).
    """
    g = grid(n, fs)
    edges = chisq_band_edges(Sn, n, fs, k_lo, k_hi, p)
    sig2 = sigma_sq(htilde, Sn, g["df"])
    zl = np.empty((p, n), dtype=np.complex128)
    for l in range(p):
        hb = np.zeros_like(htilde)
        hb[edges[l]: edges[l + 1]] = htilde[edges[l]: edges[l + 1]]
        zl[l] = filter_z(stilde, Sn, hb, n, g["df"])
    z = zl.sum(axis=0)
    chi2 = p / sig2 * np.sum(np.abs(zl - z[None, :] / p) ** 2, axis=0)
    return chi2, zl


# ---------------------------------------------------------------------------
# Events: threshold and clustering of rho(t) (Sec. 3.3; reading R17)
# ---------------------------------------------------------------------------
def window_maxima(rho: np.ndarray, W: int):
    """Index and value of the maximum of rho in each window [wW, (w+1)W) (lowest index on ties)."""
    n = rho.shape[0]
    nwin = n // W
    js = np.empty(nwin, dtype=np.int64)
    vals = np.empty(nwin)
    for w in range(nwin):
        seg = rho[w * W: (w + 1) * W]
        i = int(np.argmax(seg))  # first occurrence of the maximum
        js[w] = w * W + i
        vals[w] = seg[i]
    return js, vals


def _keep_window_winners(js, vals, threshold: float, W: int):
    """Windows whose winner reaches the threshold and is not beaten by the winner of an
    adjacent window lying within W samples of it (larger value, or equal value at a lower index)."""
    keep = []
    nwin = len(js)
    for w in range(nwin):
        j, v = int(js[w]), float(vals[w])
        if not v >= threshold:
            continue
        beaten = False
        for w2 in (w - 1, w + 1):
            if 0 <= w2 < nwin and abs(int(js[w2]) - j) <= W:
                v2, j2 = float(vals[w2]), int(js[w2])
                if v2 > v or (v2 == v and j2 < j):
                    beaten = True
        if not beaten:
            keep.append(w)
    return keep


def unit_events(rho: np.ndarray, threshold: float, W: int):
    """Events of one (template, segment) rho series (R17): [(window, j, rho)], time-ordered."""
    js, vals = window_maxima(rho, W)
    return [(w, int(js[w]), float(vals[w])) for w in _keep_window_winners(js, vals, threshold, W)]


def segment_events(events_by_template: dict, n: int, threshold: float, W: int):
    """Events of one segment across templates (R17): in each window the loudest unit event
    (ties: lowest template index), kept under the same adjacent-window rule.
    events_by_template: {t: unit_events(...)}; returns [(window, t, j, rho)]."""
    nwin = n // W
    best_t = np.full(nwin, -1, dtype=np.int64)
    best_j = np.zeros(nwin, dtype=np.int64)
    best_v = np.full(nwin, -np.inf)
    for t in sorted(events_by_template):
        for (w, j, v) in events_by_template[t]:
            if v > best_v[w]:  # strict: an equal value keeps the lower template index
                best_t[w], best_j[w], best_v[w] = t, j, v
    occupied = best_t >= 0
    js = np.where(occupied, best_j, np.arange(nwin) * W)
    keep = _keep_window_winners(js, best_v, threshold, W)
    return [(w, int(best_t[w]), int(best_j[w]), float(best_v[w])) for w in keep if occupied[w]]


# ---------------------------------------------------------------------------
# Gradient of rho^2 with respect to (M_c, eta, t_c)  (reading R13)
# ---------------------------------------------------------------------------
def _spa_phase_and_partials(f: np.ndarray, mc: float, eta: float, tc: float):
    """Psi and its partial derivatives dPsi/dMc [per M_sun], dPsi/deta, dPsi/dtc."""
    M = total_mass_from_mc_eta(mc, eta) * T_SUN
    v = (np.pi * M * f) ** (1.0 / 3.0)
    p2 = 3715.0 / 756.0 + 55.0 * eta / 9.0
    p3 = -16.0 * np.pi
    p4 = 15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta * eta / 72.0
    P = 1.0 + p2 * v ** 2 + p3 * v ** 3 + p4 * v ** 4
    dP_dv = 2.0 * p2 * v + 3.0 * p3 * v ** 2 + 4.0 * p4 * v ** 3
    dP_deta = (55.0 / 9.0) * v ** 2 + (27145.0 / 504.0 + 2.0 * 3085.0 * eta / 72.0) * v ** 4
    C = 3.0 / (128.0 * eta)
    psi = 2.0 * np.pi * f * tc - np.pi / 4.0 + C * v ** (-5) * P
    dpsi_dv = C * (-5.0 * v ** (-6) * P + v ** (-5) * dP_dv)
    # M = mc eta^(-3/5) T_sun and v is proportional to M^(1/3):
    #   dv/dmc = v / (3 mc),  dv/deta = -v / (5 eta).
    dpsi_dmc = dpsi_dv * v / (3.0 * mc)
    dpsi_deta = (-C / eta) * v ** (-5) * P + C * v ** (-5) * dP_deta + dpsi_dv * (-v / (5.0 * eta))
    dpsi_dtc = 2.0 * np.pi * f
    return psi, dpsi_dmc, dpsi_deta, dpsi_dtc


def snr_sq(theta, stilde: np.ndarray, Sn: np.ndarray, n: int, fs: float,
           k_lo: int, k_hi: int, with_grad: bool = False):
    """F = |Z|^2 / sigma^2 at theta = (M_c [M_sun], eta, t_c [s]) with a frozen band.

    Z = 4 df sum_{k in [k_lo,k_hi]} f_k^(-7/6) e^{+i Psi_k(theta)} s_k / S_k.
    Returns (F, Z, grad) with grad = dF/dtheta (None unless requested).
    """
    mc, eta, tc = (float(t) for t in theta)
    g = grid(n, fs)
    f = freqs(n, fs)[k_lo: k_hi + 1]
    a = spa_amplitude(f)
    w = stilde[k_lo: k_hi + 1].astype(np.complex128) / Sn[k_lo: k_hi + 1]
    sig2 = 4.0 * g["df"] * float(np.sum(a * a / Sn[k_lo: k_hi + 1]))
    if not with_grad:
        psi = spa_phase(f, mc, eta, tc)
        Z = 4.0 * g["df"] * np.sum(a * np.exp(1j * psi) * w)
        return float(abs(Z) ** 2 / sig2), complex(Z), None
    psi, d_mc, d_eta, d_tc = _spa_phase_and_partials(f, mc, eta, tc)
    terms = a * np.exp(1j * psi) * w
    Z = 4.0 * g["df"] * np.sum(terms)
    # dZ/dtheta = 4 df sum i a e^{i Psi} w dPsi/dtheta;  dF = 2 Re(conj(Z) dZ) / sigma^2
    grad = []
    for d in (d_mc, d_eta, d_tc):
        dZ = 4.0 * g["df"] * np.sum(1j * terms * d)
        grad.append(2.0 * float(np.real(np.conj(Z) * dZ)) / sig2)
    return float(abs(Z) ** 2 / sig2), complex(Z), np.array(grad)


def template_metric(theta, Sn: np.ndarray, n: int, fs: float, k_lo: int, k_hi: int) -> np.ndarray:
    """Phase-maximised template-space metric g (3x3) at theta over a frozen band.

    With weights W_k = |h_k|^2 / S_k = f_k^(-7/3) / S_k (the integrand of
    Eq. (4)) and d_k = dPsi_k/dtheta, g_ij = <d_i d_j> - <d_i><d_j>, <x> the
    W-weighted mean; near a maximum of rho^2, F(theta + delta) ~
    F(theta) (1 - g_ij delta_i delta_j).
    """
    mc, eta, tc = (float(t) for t in theta)
    f = freqs(n, fs)[k_lo: k_hi + 1]
    W = spa_amplitude(f) ** 2 / Sn[k_lo: k_hi + 1]
    _, d_mc, d_eta, d_tc = _spa_phase_and_partials(f, mc, eta, tc)
    d = np.stack([d_mc, d_eta, d_tc])
    mean = (d * W).sum(axis=1) / W.sum()
    second = (d[:, None, :] * d[None, :, :] * W).sum(axis=2) / W.sum()
    return second - np.outer(mean, mean)


def snr_sq_fd_grad(theta, stilde, Sn, n, fs, k_lo, k_hi, rel: float = 1e-6):
    """Central finite differences of F: relative step for M_c and eta, 1e-6 dt for t_c."""
    theta = np.asarray(theta, dtype=np.float64)
    dt = 1.0 / fs
    steps = np.array([rel * theta[0], rel * theta[1], rel * dt])
    grad = np.zeros(3)
    for i in range(3):
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += steps[i]
        tm[i] -= steps[i]
        Fp = snr_sq(tp, stilde, Sn, n, fs, k_lo, k_hi)[0]
        Fm = snr_sq(tm, stilde, Sn, n, fs, k_lo, k_hi)[0]
        grad[i] = (Fp - Fm) / (2.0 * steps[i])
    return grad


# ---------------------------------------------------------------------------
# Brute-force references for tiny inputs
# ---------------------------------------------------------------------------
def naive_dft(x: np.ndarray, sign: int = +1) -> np.ndarray:
    """O(N^2) sum_k x_k e^{sign 2 pi i jk/N}, for N up to a few hundred."""
    n = x.shape[-1]
    j = np.arange(n)
    W = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
    return W @ x.astype(np.complex128)


__all__ = [
    "window_maxima", "unit_events", "segment_events",
    "psd_from_array", "prefix_sums", "segment_spectrum",
    "T_SUN", "PSD_F0", "grid", "freqs", "psd_initial_ligo", "psd_bins",
    "total_mass_from_mc_eta", "f_isco", "band_lo", "band", "spa_phase",
    "spa_amplitude", "spa_template", "quadrature_partner", "sigma_sq",
    "inverse_dft", "filter_z", "filter_z_literal", "snr", "peak", "filter_unit",
    "snr_sq", "snr_sq_fd_grad", "template_metric", "naive_dft", "chisq_band_edges", "chisq_series",
]
