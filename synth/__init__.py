"""Seeded synthetic inputs shared by the tests and the benchmark.

This module holds no arithmetic of the matched-filter method itself: it draws
Gaussian numbers, scales them by a noise spectrum that the caller supplies,
adds a caller-supplied template spectrum at a chosen time and phase, and lays
out template banks as mass parameters.  Both the oracle side and the GPU side
receive exactly the arrays built here.

Workload shapes follow the paper's search set-up (Sec. 1.1: 256 s segments at
4096 Hz, 2^20 samples, f_low = 40 Hz; masses 1-34 M_sun).  The PSD used to
colour the noise is whatever the caller passes; the tests and the benchmark
pass the analytic initial-LIGO curve of Eq. (2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 20090906


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    fs: float
    f_low: float
    n_seg: int
    description: str
    extra: dict = field(default_factory=dict)


# The five workloads (small FP64 case, single 2^20 segment with a 1024-template
# bank, uneven batched bank, gradient refinement, precision sweep).
WORKLOADS = {
    1: Workload("plain-fp64-n65536-16tmpl", 1 << 16, 2048.0, 40.0, 1,
                "32 s at 2048 Hz, 4x4 grid m1,m2 in [1,3], one SNR-10 injection"),
    2: Workload("single-seg-n1048576-1024tmpl", 1 << 20, 4096.0, 40.0, 1,
                "256 s at 4096 Hz, 32x32 (Mc,eta) grid for m1,m2 in [1,3], 5 injections SNR 8-15"),
    3: Workload("batched-uneven-8192tmpl-x8seg", 1 << 20, 4096.0, 40.0, 8,
                "8192 templates m1,m2 in [1,34], M<=35, 8 segments of 2^20"),
    4: Workload("gradient-4096trig", 1 << 20, 4096.0, 40.0, 1,
                "4096 triggers from the single-segment noise, 20 ascent steps"),
    5: Workload("precision-sweep-32768tmpl-x4seg", 1 << 20, 4096.0, 40.0, 4,
                "32768 templates m1,m2 in [1,34], M<=35, 4 segments of 2^20"),
}


def seed_sequence(cfg: int) -> np.random.SeedSequence:
    return np.random.SeedSequence(BASE_SEED + int(cfg))


def rngs(cfg: int, count: int) -> list[np.random.Generator]:
    """Independent PCG64 generators spawned from the workload's seed."""
    return [np.random.Generator(np.random.PCG64(s)) for s in seed_sequence(cfg).spawn(count)]


# ---------------------------------------------------------------------------
# Mass parameters
# ---------------------------------------------------------------------------
def mc_eta(m1, m2):
    """Chirp mass and symmetric mass ratio from component masses (symmetric in m1,m2)."""
    m1 = np.asarray(m1, dtype=np.float64)
    m2 = np.asarray(m2, dtype=np.float64)
    mt = m1 + m2
    prod = m1 * m2
    return prod ** 0.6 / mt ** 0.2, prod / (mt * mt)


def bank_grid_components(m_values):
    """All ordered (m1, m2) pairs of a component-mass grid, flattened row-major."""
    m = np.asarray(m_values, dtype=np.float64)
    m1, m2 = np.meshgrid(m, m, indexing="ij")
    return m1.ravel(), m2.ravel()


def bank_small_grid():
    """4x4 component-mass grid m in {1, 5/3, 7/3, 3} M_sun (16 templates)."""
    m1, m2 = bank_grid_components([1.0, 5.0 / 3.0, 7.0 / 3.0, 3.0])
    mc, eta = mc_eta(m1, m2)
    return mc, eta


def bank_mc_eta_grid(n_mc: int = 32, n_eta: int = 32, m_lo: float = 1.0, m_hi: float = 3.0):
    """Uniform (Mc, eta) grid spanning the range of m1,m2 in [m_lo, m_hi]."""
    mc_lo = mc_eta(m_lo, m_lo)[0]
    mc_hi = mc_eta(m_hi, m_hi)[0]
    eta_lo = mc_eta(m_lo, m_hi)[1]
    mc_axis = np.linspace(float(mc_lo), float(mc_hi), n_mc)
    eta_axis = np.linspace(float(eta_lo), 0.25, n_eta)
    mc, eta = np.meshgrid(mc_axis, eta_axis, indexing="ij")
    return mc.ravel().copy(), eta.ravel().copy()


def bank_uneven(n_tmpl: int, rng: np.random.Generator, m_min: float = 1.0,
                m_max: float = 34.0, m_total_max: float = 35.0):
    """Uniform draws over {m_min <= m2 <= m1 <= m_max, m1 + m2 <= m_total_max}."""
    out1, out2 = [], []
    need = n_tmpl
    while need > 0:
        a = rng.uniform(m_min, m_max, size=2 * need + 64)
        b = rng.uniform(m_min, m_max, size=2 * need + 64)
        m1 = np.maximum(a, b)
        m2 = np.minimum(a, b)
        ok = (m1 + m2) <= m_total_max
        out1.append(m1[ok][:need])
        out2.append(m2[ok][:need])
        need -= int(min(need, ok.sum()))
    m1 = np.concatenate(out1)[:n_tmpl]
    m2 = np.concatenate(out2)[:n_tmpl]
    mc, eta = mc_eta(m1, m2)
    return mc, eta, m1, m2


# ---------------------------------------------------------------------------
# Coloured Gaussian noise in the frequency domain
# ---------------------------------------------------------------------------
def gaussian_bins(rng: np.random.Generator, count: int) -> np.ndarray:
    """count complex numbers g1 + i g2 with g1, g2 iid N(0,1)."""
    g = rng.standard_normal(size=(count, 2))
    return g[:, 0] + 1j * g[:, 1]


def coloured_noise(Sn_band: np.ndarray, df: float, k_lo: int, n_bins: int,
                   rng: np.random.Generator, dtype=np.complex64) -> np.ndarray:
    """One-sided noise spectrum: s_k = sqrt(S_k / (4 df)) (g1 + i g2) on [k_lo, k_lo+len(Sn_band)).

    E|s_k|^2 = S_k / (2 df), the one-sided convention.  Bins outside the given
    range are zero.  Sn_band holds the caller's PSD values on those bins.
    """
    s = np.zeros(n_bins, dtype=np.complex128)
    m = Sn_band.shape[0]
    s[k_lo: k_lo + m] = np.sqrt(Sn_band / (4.0 * df)) * gaussian_bins(rng, m)
    return s.astype(dtype)


def inject(stilde: np.ndarray, htilde: np.ndarray, amplitude: float, phi0: float,
           j0: int, n: int) -> np.ndarray:
    """s_k += A e^{i phi0} h_k e^{-2 pi i k j0 / N}: the template delayed by j0 samples."""
    k = np.arange(htilde.shape[0], dtype=np.float64)
    shift = np.exp(-2j * np.pi * ((k * j0) % n) / n)
    out = stilde.astype(np.complex128) + amplitude * np.exp(1j * phi0) * htilde * shift
    return out.astype(stilde.dtype)


def injection_params(rng: np.random.Generator, count: int, n: int,
                     m_lo: float = 1.0, m_hi: float = 3.0,
                     snr_lo: float = 8.0, snr_hi: float = 15.0):
    """count injections: masses U[m_lo,m_hi]^2, SNR U[snr_lo,snr_hi], j0 U{0..N-1}, phi0 U[0,2pi)."""
    m1 = rng.uniform(m_lo, m_hi, size=count)
    m2 = rng.uniform(m_lo, m_hi, size=count)
    snr = rng.uniform(snr_lo, snr_hi, size=count)
    j0 = rng.integers(0, n, size=count)
    phi0 = rng.uniform(0.0, 2.0 * np.pi, size=count)
    return [dict(m1=float(a), m2=float(b), snr=float(c), j0=int(d), phi0=float(e))
            for a, b, c, d, e in zip(m1, m2, snr, j0, phi0)]
