"""Seeded test inputs: coloured noise (coloured by the oracle's PSD) and injections.

The same complex arrays are handed to the oracle (up-cast to complex128) and
to the GPU path, so parity measures compute error only.
"""
from __future__ import annotations

import math

import numpy as np

import oracle as O
import synth


def segment(n: int, fs: float, seed, injections=(), f_low: float = 40.0, dtype=np.complex64, noise: bool = True):
    """One-sided data spectrum [N/2+1]: coloured Gaussian noise plus injections.

    injections: iterable of dicts with m1, m2, snr, j0, phi0.
    """
    g = O.grid(n, fs)
    Sn = O.psd_bins(n, fs, f_low)
    k_lo = O.band_lo(n, fs, f_low)
    rng = np.random.Generator(np.random.PCG64(seed))
    if noise:
        s = synth.coloured_noise(Sn[k_lo: n // 2], g["df"], k_lo, n // 2 + 1, rng, dtype=np.complex128)
    else:
        s = np.zeros(n // 2 + 1, dtype=np.complex128)
    for inj in injections:
        mc, eta = map(float, synth.mc_eta(inj["m1"], inj["m2"]))
        h = O.spa_template(n, fs, f_low, mc, eta)
        sig = math.sqrt(O.sigma_sq(h, Sn, g["df"]))
        s = synth.inject(s, h, inj["snr"] / sig, inj["phi0"], inj["j0"], n)
    return s.astype(dtype), Sn


def series_error(rho_gpu: np.ndarray, rho_ora: np.ndarray) -> float:
    """max_j |rho_g - rho_o| / max(rho_o, 1)."""
    return float(np.max(np.abs(rho_gpu - rho_ora) / np.maximum(rho_ora, 1.0)))


def peak_index_ok(j_gpu: int, rho_series_ora: np.ndarray, j_ora: int, rel: float = 2e-4) -> bool:
    """Exact index, or a near-tie: the oracle's rho at the GPU index is within rel of its maximum."""
    if j_gpu == j_ora:
        return True
    return bool(rho_series_ora[j_gpu] >= rho_series_ora[j_ora] * (1.0 - rel))


def n_above_bounds(rho_series_ora: np.ndarray, threshold: float, rel: float = 1e-4) -> tuple[int, int]:
    """Range of threshold counts consistent with a rho series within rel of the oracle's.

    A GPU sample counts when rho_g >= threshold, and rho_g lies in
    [rho_o (1 - rel), rho_o (1 + rel)]; so every sample with rho_o >= th/(1 - rel)
    counts and none with rho_o < th/(1 + rel) does.  Only samples between the two
    (near-ties with the threshold) may go either way.
    """
    lo = int(np.count_nonzero(rho_series_ora >= threshold / (1.0 - rel)))
    hi = int(np.count_nonzero(rho_series_ora >= threshold / (1.0 + rel)))
    return lo, hi
