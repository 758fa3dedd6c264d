"""Oracle side of the full-size parity tests, run in spawned worker processes (CPU only).

Each worker receives the data spectra once (the same complex64 values the GPU
gets) and evaluates the FP64 oracle for one (template, segment) unit per task.
"""
import math

import numpy as np

import oracle as O
from tests import _data as D

_STATE = {}


def init(n, fs, segments):
    _STATE.update(n=n, fs=fs, Sn=O.psd_bins(n, fs, 40.0),
                  segs=[np.asarray(s).astype(np.complex128) for s in segments])


def filter_unit(task):
    """task = (mc, eta, segment, threshold, j_gpu, rho_series_gpu or None).

    Returns the oracle peak (rho, j, sigma), the oracle rho at the GPU's index,
    the tie-aware bounds of the threshold count and, when a GPU series is given,
    the series error max_j |rho_g - rho_o| / max(rho_o, 1)."""
    mc, eta, s, thr, j_gpu, series_gpu = task
    d = _STATE
    o = O.filter_unit(d["n"], d["fs"], 40.0, mc, eta, d["segs"][s], d["Sn"], threshold=thr, return_series=True)
    rho = o["series"]
    out = {"rho": o["rho"], "j": o["j"], "sigma": o["sigma"], "rho_at_gpu": float(rho[j_gpu])}
    if math.isfinite(thr):
        out["n_above_bounds"] = D.n_above_bounds(rho, thr)
    if series_gpu is not None:
        out["series_err"] = D.series_error(np.asarray(series_gpu, dtype=np.float64), rho)
    return out


def chisq_unit(task):
    """task = (mc, eta, segment, p, j_gpu, rho_series_gpu or None, chisq_series_gpu or None).

    Oracle chi^2 series (Eq. (5)) and rho series of one unit; returns the peak,
    chi^2 at the oracle's and at the GPU's peak sample, and the series errors
    (rho: Q20 metric; chi^2: |dchi2| / (chi2 + rho^2 + 1))."""
    mc, eta, s, p, j_gpu, rho_g, chi_g = task
    d = _STATE
    n, fs = d["n"], d["fs"]
    h = O.spa_template(n, fs, 40.0, mc, eta)
    k_lo, k_hi = O.band(n, fs, 40.0, mc, eta)
    sig = math.sqrt(O.sigma_sq(h, d["Sn"], fs / n))
    chi, zl = O.chisq_series(d["segs"][s], d["Sn"], h, n, fs, k_lo, k_hi, p)
    rho = np.abs(zl.sum(axis=0)) / sig
    j = int(np.argmax(rho))
    out = {"rho": float(rho[j]), "j": j, "rho_at_gpu": float(rho[j_gpu]), "chisq_at_gpu": float(chi[j_gpu]),
           "scale_at_gpu": float(chi[j_gpu] + rho[j_gpu] ** 2 + 1.0)}
    if rho_g is not None:
        out["series_err"] = D.series_error(np.asarray(rho_g, dtype=np.float64), rho)
    if chi_g is not None:
        out["chisq_series_err"] = float(np.max(np.abs(np.asarray(chi_g, dtype=np.float64) - chi) /
                                               (chi + rho ** 2 + 1.0)))
    return out
