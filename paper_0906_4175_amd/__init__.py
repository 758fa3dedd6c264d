"""MI355X (gfx950) matched filter for compact-binary inspiral searches.

Python binding of libmf (include/mf.h): argument marshalling only.  Every
step of the path runs in the HIP kernels of libmf.so; PyTorch provides device
memory and the current stream.  There is no CPU fallback: importing the
package without the built library raises.

Calls follow arXiv:0906.4175, Sec. 1.1: :func:`psd` is Eq. (2), :func:`spa_bank`
builds the 2PN stationary-phase templates and their norm (Eq. (4)),
:func:`filter` evaluates Eq. (1) and Eq. (3) with the peak / threshold search,
:func:`snr_sq` and :class:`SnrSq` give rho^2 at continuous template parameters
and its gradient.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

__all__ = ["Grid", "Bank", "psd", "spa_bank", "filter", "filter_plan", "filter_workspace_bytes", "ifft", "snr_sq", "SnrSq",
           "PRECISIONS", "version",
           "template_metric", "chisq", "filter_chisq", "filter_chisq_workspace_bytes",
           "psd_prefix", "rfft", "filter_events", "chisq_events", "filter_chisq_plan",
           "filter_events_workspace_bytes"]

PRECISIONS = {"fp64": L.MF_FP64, "fp32_ph64": L.MF_FP32_PH64, "fp32": L.MF_FP32}
SIGMA_MODES = {"fp64": L.MF_SIGMA_FP64, "comp32": L.MF_SIGMA_COMP32}

_clib = L.load()


def version() -> str:
    return _clib.mf_version().decode()


@dataclass(frozen=True)
class Grid:
    """N-point segment at sample rate fs [Hz], low cutoff f_low [Hz], PSD knee f0 [Hz]."""
    n: int
    fs: float
    f_low: float = 40.0
    f0: float = 150.0

    def c(self) -> L.MfGrid:
        return L.MfGrid(int(self.n), float(self.fs), float(self.f_low), float(self.f0))

    @property
    def T(self) -> float:
        return self.n / self.fs

    @property
    def df(self) -> float:
        return self.fs / self.n

    @property
    def k_lo(self) -> int:
        return int(math.ceil(self.f_low * (self.n / self.fs)))


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _cdtype(prec: int) -> torch.dtype:
    return torch.complex128 if prec == L.MF_FP64 else torch.complex64


def _stream(device: torch.device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(0 if t is None else t.data_ptr())


def _require_cuda(*tensors):
    for t in tensors:
        if t is not None and not t.is_cuda:
            raise ValueError("libmf operates on GPU tensors only")


def psd(grid: Grid, prefix: bool = False, device="cuda"):
    """S_n on the one-sided bins (Eq. (2)), +inf outside [k_lo, N/2-1]; optionally P_k."""
    dev = torch.device(device)
    Sn = torch.empty(grid.n // 2 + 1, dtype=torch.float64, device=dev)
    P = torch.empty_like(Sn) if prefix else None
    g = grid.c()
    L.check(_clib.mf_psd(C.byref(g), _ptr(Sn), _ptr(P), _stream(dev)))
    return (Sn, P) if prefix else Sn


@dataclass
class Bank:
    grid: Grid
    data: torch.Tensor          # device bytes (mf_bank_entry[n_tmpl])
    n_tmpl: int
    k_hi: np.ndarray
    sigma: np.ndarray
    htilde: torch.Tensor | None = None


def spa_bank(grid: Grid, mc, eta, Sn: torch.Tensor, precision="fp32_ph64", sigma_mode="fp64",
             materialise: bool = False) -> Bank:
    """2PN stationary-phase bank for chirp masses mc [M_sun] and symmetric mass ratios eta."""
    _require_cuda(Sn)
    mc = np.ascontiguousarray(mc, dtype=np.float64).ravel()
    eta = np.ascontiguousarray(eta, dtype=np.float64).ravel()
    if mc.shape != eta.shape:
        raise ValueError("mc and eta must have the same length")
    n_tmpl = int(mc.shape[0])
    prec = _prec(precision)
    nbytes = int(_clib.mf_bank_bytes(n_tmpl))
    data = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=Sn.device)
    khi = np.zeros(n_tmpl, dtype=np.int32)
    sig = np.zeros(n_tmpl, dtype=np.float64)
    ht = None
    if materialise:
        ht = torch.empty((n_tmpl, grid.n // 2 + 1), dtype=_cdtype(prec), device=Sn.device)
    g = grid.c()
    DP = C.POINTER(C.c_double)
    st = _clib.mf_spa_bank(C.byref(g), mc.ctypes.data_as(DP), eta.ctypes.data_as(DP), n_tmpl, _ptr(Sn), prec,
                          SIGMA_MODES[sigma_mode] if isinstance(sigma_mode, str) else int(sigma_mode),
                          _ptr(data), khi.ctypes.data_as(C.POINTER(C.c_int32)), sig.ctypes.data_as(DP), _ptr(ht),
                          _stream(Sn.device))
    L.check(st)
    return Bank(grid, data, n_tmpl, khi, sig, ht)


def filter_workspace_bytes(grid: Grid, precision, n_tmpl: int, n_seg: int) -> int:
    g = grid.c()
    nb = int(_clib.mf_filter_workspace_bytes(C.byref(g), _prec(precision), int(n_tmpl), int(n_seg)))
    if nb == 0:
        raise L.MfError(-1, _clib.mf_last_error().decode())
    return nb


def filter_plan(grid: Grid, precision="fp32_ph64") -> dict:
    """The launch plan mf_filter uses for this grid and precision."""
    arr = (C.c_int32 * 8)()
    g = grid.c()
    L.check(_clib.mf_filter_plan(C.byref(g), _prec(precision), arr))
    keys = ("n1", "n2", "cols_per_wg", "rows_per_wg", "threads_pass1", "threads_pass2", "units_per_batch", "flags")
    return dict(zip(keys, [int(x) for x in arr]))


def filter_chisq_plan(grid: Grid, precision="fp32_ph64") -> dict:
    """The launch plan mf_filter_chisq uses for this grid and precision."""
    arr = (C.c_int32 * 8)()
    g = grid.c()
    L.check(_clib.mf_filter_chisq_plan(C.byref(g), _prec(precision), arr))
    keys = ("n1", "n2", "cols_per_wg", "rows_per_wg", "threads_pass1", "threads_pass2", "units_per_batch", "flags")
    return dict(zip(keys, [int(x) for x in arr]))


_tune_cache_loaded = False


def _maybe_load_tune_cache():
    """Install plans from $MF_TUNE_CACHE once per process (first filter call)."""
    global _tune_cache_loaded
    if _tune_cache_loaded:
        return
    _tune_cache_loaded = True
    path = os.environ.get("MF_TUNE_CACHE")
    if path:
        from . import tune
        tune.load_cache(path)


def filter(grid: Grid, bank: Bank, stilde: torch.Tensor, Sn: torch.Tensor, precision="fp32_ph64",
           threshold: float = math.inf, window=None, series_units=None, workspace: torch.Tensor | None = None,
           peaks: torch.Tensor | None = None):
    """Peak rho, its index j and the threshold count for every (template, segment).

    stilde: [n_seg, N/2+1] complex (complex128 for 'fp64', complex64 otherwise) on the GPU.
    Returns dict(rho [n_tmpl, n_seg] float64, j int32, n_above int32, series or None).
    """
    prec = _prec(precision)
    _require_cuda(stilde, Sn)
    _maybe_load_tune_cache()
    if stilde.dim() == 1:
        stilde = stilde.unsqueeze(0)
    if stilde.dtype != _cdtype(prec) or not stilde.is_contiguous() or stilde.shape[-1] != grid.n // 2 + 1:
        raise ValueError(f"stilde must be contiguous {_cdtype(prec)} of shape [n_seg, {grid.n // 2 + 1}]")
    n_seg = int(stilde.shape[0])
    dev = stilde.device
    n_units = bank.n_tmpl * n_seg
    need = filter_workspace_bytes(grid, prec, bank.n_tmpl, n_seg)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    if peaks is None:
        peaks = torch.empty(2 * n_units, dtype=torch.float64, device=dev)
    opts, series, su = _filter_opts(grid, prec, dev, threshold, window, series_units)
    g = grid.c()
    st = _clib.mf_filter(C.byref(g), _ptr(bank.data), bank.n_tmpl, _ptr(stilde), n_seg, _ptr(Sn), prec,
                        C.byref(opts), _ptr(workspace), workspace.numel(), _ptr(peaks), _ptr(series), _stream(dev))
    L.check(st)
    return _peaks_dict(peaks, bank.n_tmpl, n_seg, series)


def _filter_opts(grid: Grid, prec: int, dev, threshold, window, series_units):
    """mf_filter_opts and the series buffer (the unit-id tensor is returned to keep it alive)."""
    opts = L.MfFilterOpts(float(threshold), 0, 0, None, 0)
    if window is not None:
        opts.j_begin, opts.j_end = int(window[0]), int(window[1])
    series = None
    su = None
    if series_units is not None:
        su = torch.as_tensor(np.asarray(series_units, dtype=np.int32), device=dev)
        series = torch.empty((su.numel(), grid.n), dtype=torch.float64 if prec == L.MF_FP64 else torch.float32,
                             device=dev)
        opts.series_units_dev = su.data_ptr()
        opts.n_series = su.numel()
    return opts, series, su


def _peaks_dict(peaks: torch.Tensor, n_tmpl: int, n_seg: int, series):
    pk = peaks.view(n_tmpl, n_seg, 2)
    ints = pk[..., 1].contiguous().view(torch.int32).view(n_tmpl, n_seg, 2)
    return {"rho": pk[..., 0], "j": ints[..., 0], "n_above": ints[..., 1], "series": series, "raw": peaks}


def filter_noalloc(grid: Grid, bank: Bank, stilde: torch.Tensor, Sn: torch.Tensor, peaks: torch.Tensor,
                   precision="fp32_ph64", threshold: float = math.inf, window=None, series_ptr: int = 0,
                   series_units_ptr: int = 0, n_series: int = 0):
    """:func:`filter` through mf_filter_noalloc: the library's static device
    scratch instead of a workspace.  The caller passes every buffer (peaks
    [2 n_tmpl n_seg] float64; optional series and unit ids as device
    pointers), so the call allocates nothing."""
    prec = _prec(precision)
    _require_cuda(stilde, Sn, peaks)
    if stilde.dim() == 1:
        stilde = stilde.unsqueeze(0)
    if stilde.dtype != _cdtype(prec) or not stilde.is_contiguous() or stilde.shape[-1] != grid.n // 2 + 1:
        raise ValueError(f"stilde must be contiguous {_cdtype(prec)} of shape [n_seg, {grid.n // 2 + 1}]")
    n_seg = int(stilde.shape[0])
    if peaks.dtype != torch.float64 or not peaks.is_contiguous() or peaks.numel() < 2 * bank.n_tmpl * n_seg:
        raise ValueError("peaks must be contiguous float64 with 2 n_tmpl n_seg elements")
    opts = L.MfFilterOpts(float(threshold), 0, 0, series_units_ptr or None, int(n_series))
    if window is not None:
        opts.j_begin, opts.j_end = int(window[0]), int(window[1])
    g = grid.c()
    st = _clib.mf_filter_noalloc(C.byref(g), _ptr(bank.data), bank.n_tmpl, _ptr(stilde), n_seg, _ptr(Sn), prec,
                                 C.byref(opts), _ptr(peaks), C.c_void_p(series_ptr or None), _stream(stilde.device))
    L.check(st)
    return _peaks_dict(peaks, bank.n_tmpl, n_seg, None)


def filter_chisq_workspace_bytes(grid: Grid, precision, n_tmpl: int, n_seg: int, p_bands: int = 16) -> int:
    g = grid.c()
    nb = int(_clib.mf_filter_chisq_workspace_bytes(C.byref(g), _prec(precision), int(n_tmpl), int(n_seg),
                                                    int(p_bands)))
    if nb == 0:
        raise L.MfError(-1, "no band-mode workspace for these arguments (N, precision, p_bands in [2, 64])")
    return nb


def filter_chisq(grid: Grid, bank: Bank, stilde: torch.Tensor, Sn: torch.Tensor, prefix: torch.Tensor,
                 precision="fp32_ph64", p_bands: int = 16, threshold: float = math.inf, window=None,
                 series_units=None, workspace: torch.Tensor | None = None):
    """:func:`filter` plus the chi^2 of Eq. (5) at every sample (p_bands equal-sigma^2 bands).

    prefix: the prefix array of :func:`psd` (prefix=True).  Returns the dict of
    :func:`filter` plus "chisq" [n_tmpl, n_seg] float64 (chi^2 at each peak) and
    "chisq_series" ([n_series, N], or None).
    """
    prec = _prec(precision)
    _require_cuda(stilde, Sn, prefix)
    if stilde.dim() == 1:
        stilde = stilde.unsqueeze(0)
    if stilde.dtype != _cdtype(prec) or not stilde.is_contiguous() or stilde.shape[-1] != grid.n // 2 + 1:
        raise ValueError(f"stilde must be contiguous {_cdtype(prec)} of shape [n_seg, {grid.n // 2 + 1}]")
    n_seg = int(stilde.shape[0])
    dev = stilde.device
    n_units = bank.n_tmpl * n_seg
    need = filter_chisq_workspace_bytes(grid, prec, bank.n_tmpl, n_seg, p_bands)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    peaks = torch.empty(2 * n_units, dtype=torch.float64, device=dev)
    chisq = torch.empty((bank.n_tmpl, n_seg), dtype=torch.float64, device=dev)
    opts = L.MfFilterOpts(float(threshold), 0, 0, None, 0)
    if window is not None:
        opts.j_begin, opts.j_end = int(window[0]), int(window[1])
    series = chi_series = su = None
    if series_units is not None:
        su = torch.as_tensor(np.asarray(series_units, dtype=np.int32), device=dev)
        sdt = torch.float64 if prec == L.MF_FP64 else torch.float32
        series = torch.empty((su.numel(), grid.n), dtype=sdt, device=dev)
        chi_series = torch.empty_like(series)
        opts.series_units_dev = su.data_ptr()
        opts.n_series = su.numel()
    g = grid.c()
    L.check(_clib.mf_filter_chisq(C.byref(g), _ptr(bank.data), bank.n_tmpl, _ptr(stilde), n_seg, _ptr(Sn),
                                  _ptr(prefix), prec, int(p_bands), C.byref(opts), _ptr(workspace),
                                  workspace.numel(), _ptr(peaks), _ptr(chisq), _ptr(series), _ptr(chi_series),
                                  _stream(dev)))
    pk = peaks.view(bank.n_tmpl, n_seg, 2)
    ints = pk[..., 1].contiguous().view(torch.int32).view(bank.n_tmpl, n_seg, 2)
    return {"rho": pk[..., 0], "j": ints[..., 0], "n_above": ints[..., 1], "series": series, "raw": peaks,
            "chisq": chisq, "chisq_series": chi_series}


def psd_prefix(grid: Grid, Sn: torch.Tensor) -> torch.Tensor:
    """Prefix array (the chi^2 band edges' sums) of a caller-supplied PSD [N/2+1] on the GPU."""
    _require_cuda(Sn)
    if Sn.dtype != torch.float64 or not Sn.is_contiguous() or Sn.numel() != grid.n // 2 + 1:
        raise ValueError(f"Sn must be contiguous float64 of {grid.n // 2 + 1} bins")
    P = torch.empty_like(Sn)
    g = grid.c()
    L.check(_clib.mf_psd_prefix(C.byref(g), _ptr(Sn), _ptr(P), _stream(Sn.device)))
    return P


def rfft(x: torch.Tensor, fs: float, precision="fp32_ph64", workspace: torch.Tensor | None = None) -> torch.Tensor:
    """One-sided spectra s_k = dt sum_j x_j e^{-2 pi i jk/N}, k = 0..N/2, of real segments x [..., N]."""
    prec = _prec(precision)
    _require_cuda(x)
    want = torch.float64 if prec == L.MF_FP64 else torch.float32
    if x.dtype != want or not x.is_contiguous():
        raise ValueError(f"x must be contiguous {want}")
    n = int(x.shape[-1])
    batch = int(x.numel() // n)
    need = int(_clib.mf_rfft_workspace_bytes(n, prec, batch))
    if need == 0:
        raise L.MfError(-2, _clib.mf_last_error().decode())
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    out = torch.empty(tuple(x.shape[:-1]) + (n // 2 + 1,), dtype=_cdtype(prec), device=x.device)
    L.check(_clib.mf_rfft(n, float(fs), prec, _ptr(x), _ptr(out), batch, _ptr(workspace), workspace.numel(),
                          _stream(x.device)))
    return out


def _events_view(raw: torch.Tensor, shape):
    """(rho float64, j int32, t int32) views of an mf_event buffer (16 bytes per record)."""
    ev = raw.view(*shape, 2)
    ints = ev[..., 1].contiguous().view(torch.int32).view(*shape, 2)
    return {"rho": ev[..., 0], "j": ints[..., 0], "t": ints[..., 1], "raw": raw}


def filter_events_workspace_bytes(grid: Grid, precision, n_tmpl: int, n_seg: int, log2_window: int = 12) -> int:
    g = grid.c()
    nb = int(_clib.mf_filter_events_workspace_bytes(C.byref(g), _prec(precision), int(n_tmpl), int(n_seg),
                                                     int(log2_window)))
    if nb == 0:
        raise L.MfError(-1, "no events workspace for these arguments (log2_window in [4, min(16, log2 N)])")
    return nb


def filter_events(grid: Grid, bank: Bank, stilde: torch.Tensor, Sn: torch.Tensor, precision="fp32_ph64",
                  threshold: float = 5.5, log2_window: int = 12, unit_events: bool = False,
                  workspace: torch.Tensor | None = None):
    """:func:`filter` plus thresholded, clustered events in windows of 2^log2_window samples.

    Returns the dict of :func:`filter` plus "seg_events" ({rho, j, t} of shape
    [n_seg, N >> log2_window]; t = -1 where a window has no event) and, with
    unit_events=True, "unit_events" of shape [n_tmpl, n_seg, N >> log2_window].
    """
    prec = _prec(precision)
    _require_cuda(stilde, Sn)
    if stilde.dim() == 1:
        stilde = stilde.unsqueeze(0)
    if stilde.dtype != _cdtype(prec) or not stilde.is_contiguous() or stilde.shape[-1] != grid.n // 2 + 1:
        raise ValueError(f"stilde must be contiguous {_cdtype(prec)} of shape [n_seg, {grid.n // 2 + 1}]")
    n_seg = int(stilde.shape[0])
    dev = stilde.device
    g = grid.c()
    need = filter_events_workspace_bytes(grid, prec, bank.n_tmpl, n_seg, log2_window)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    n_win = grid.n >> int(log2_window)
    peaks = torch.empty(2 * bank.n_tmpl * n_seg, dtype=torch.float64, device=dev)
    seg = torch.empty(2 * n_seg * n_win, dtype=torch.float64, device=dev)
    unit = torch.empty(2 * bank.n_tmpl * n_seg * n_win, dtype=torch.float64, device=dev) if unit_events else None
    L.check(_clib.mf_filter_events(C.byref(g), _ptr(bank.data), bank.n_tmpl, _ptr(stilde), n_seg, _ptr(Sn), prec,
                                   float(threshold), int(log2_window), _ptr(workspace), workspace.numel(),
                                   _ptr(peaks), _ptr(unit), _ptr(seg), _stream(dev)))
    pk = peaks.view(bank.n_tmpl, n_seg, 2)
    ints = pk[..., 1].contiguous().view(torch.int32).view(bank.n_tmpl, n_seg, 2)
    out = {"rho": pk[..., 0], "j": ints[..., 0], "n_above": ints[..., 1], "raw": peaks,
           "seg_events": _events_view(seg, (n_seg, n_win))}
    if unit is not None:
        out["unit_events"] = _events_view(unit, (bank.n_tmpl, n_seg, n_win))
    return out


def chisq_events(grid: Grid, bank: Bank, stilde: torch.Tensor, Sn: torch.Tensor, prefix: torch.Tensor, events,
                 precision="fp32_ph64", p_bands: int = 16):
    """chi^2 of Eq. (5) and rho at event records ({"raw": ...} of shape [n_seg, n_per_seg]); 0 where t < 0."""
    prec = _prec(precision)
    _require_cuda(stilde, Sn, prefix)
    if stilde.dim() == 1:
        stilde = stilde.unsqueeze(0)
    n_seg = int(stilde.shape[0])
    raw = events["raw"]
    n_per_seg = raw.numel() // 2 // n_seg
    out = torch.empty((n_seg, n_per_seg), dtype=torch.float64, device=stilde.device)
    rho = torch.empty_like(out)
    g = grid.c()
    L.check(_clib.mf_chisq_events(C.byref(g), _ptr(bank.data), bank.n_tmpl, _ptr(stilde), n_seg, _ptr(Sn),
                                  _ptr(prefix), prec, int(p_bands), _ptr(raw), n_per_seg, _ptr(out), _ptr(rho),
                                  _stream(stilde.device)))
    return out, rho


def ifft(q: torch.Tensor, precision="fp32_ph64", workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Unnormalised inverse DFT z_j = sum_k q_k e^{+2 pi i jk/N} over the last axis (diagnostic)."""
    prec = _prec(precision)
    _require_cuda(q)
    if q.dtype != _cdtype(prec) or not q.is_contiguous():
        raise ValueError(f"q must be contiguous {_cdtype(prec)}")
    n = int(q.shape[-1])
    batch = int(q.numel() // n)
    need = int(_clib.mf_ifft_workspace_bytes(n, prec, batch))
    if need == 0:
        raise L.MfError(-2, _clib.mf_last_error().decode())
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=q.device)
    z = torch.empty_like(q)
    L.check(_clib.mf_ifft(n, prec, _ptr(q), _ptr(z), batch, _ptr(workspace), workspace.numel(), _stream(q.device)))
    return z


def snr_sq(grid: Grid, theta: torch.Tensor, seg: torch.Tensor, stilde: torch.Tensor, Sn: torch.Tensor,
           khi: torch.Tensor | None = None, precision="fp32_ph64", gbar: torch.Tensor | None = None):
    """F = rho^2 at theta = [n, 3] (M_c [M_sun], eta, t_c [s]); with gbar also gbar * dF/dtheta."""
    prec = _prec(precision)
    _require_cuda(theta, seg, stilde, Sn, khi, gbar)
    theta = theta.to(torch.float64).contiguous()
    seg = seg.to(torch.int32).contiguous()
    if khi is not None:
        khi = khi.to(torch.int32).contiguous()
    if stilde.dim() == 1:
        stilde = stilde.unsqueeze(0)
    if stilde.dtype != _cdtype(prec) or not stilde.is_contiguous():
        raise ValueError(f"stilde must be contiguous {_cdtype(prec)}")
    n = int(theta.shape[0])
    dev = theta.device
    Z = torch.empty(n, dtype=torch.complex128, device=dev)
    F = torch.empty(n, dtype=torch.float64, device=dev)
    grad = None
    if gbar is not None:
        gbar = gbar.to(torch.float64).contiguous()
        grad = torch.empty((n, 3), dtype=torch.float64, device=dev)
    g = grid.c()
    st = _clib.mf_snr_grad(C.byref(g), _ptr(theta), _ptr(khi), _ptr(seg), n, _ptr(stilde), int(stilde.shape[0]),
                          _ptr(Sn), prec, _ptr(Z), _ptr(F), _ptr(gbar), _ptr(grad), _stream(dev))
    L.check(st)
    return F, Z, grad


def chisq(grid: Grid, bank: Bank, stilde: torch.Tensor, Sn: torch.Tensor, prefix: torch.Tensor, peaks,
          precision="fp32_ph64", p_bands: int = 16):
    """chi^2 of Eq. (5) at each unit's peak sample; returns (chi2, rho) [n_tmpl, n_seg] float64.

    peaks: the dict returned by :func:`filter` (its raw peak records are reused).
    prefix: the prefix array of :func:`psd` (prefix=True).
    """
    prec = _prec(precision)
    _require_cuda(stilde, Sn, prefix)
    if stilde.dim() == 1:
        stilde = stilde.unsqueeze(0)
    if stilde.dtype != _cdtype(prec) or not stilde.is_contiguous():
        raise ValueError(f"stilde must be contiguous {_cdtype(prec)}")
    n_seg = int(stilde.shape[0])
    raw = peaks["raw"]
    out = torch.empty((bank.n_tmpl, n_seg), dtype=torch.float64, device=stilde.device)
    rho = torch.empty_like(out)
    g = grid.c()
    L.check(_clib.mf_chisq(C.byref(g), _ptr(bank.data), bank.n_tmpl, _ptr(stilde), n_seg, _ptr(Sn), _ptr(prefix),
                           prec, int(p_bands), _ptr(raw), _ptr(out), _ptr(rho), _stream(stilde.device)))
    return out, rho


def template_metric(grid: Grid, theta: torch.Tensor, Sn: torch.Tensor, khi: torch.Tensor) -> torch.Tensor:
    """Phase-maximised template metric g [n, 3, 3] at theta over the frozen bands."""
    _require_cuda(theta, Sn, khi)
    theta = theta.to(torch.float64).contiguous()
    khi = khi.to(torch.int32).contiguous()
    n = int(theta.shape[0])
    out = torch.empty((n, 6), dtype=torch.float64, device=theta.device)
    g = grid.c()
    L.check(_clib.mf_template_metric(C.byref(g), _ptr(theta), _ptr(khi), n, _ptr(Sn), _ptr(out),
                                      _stream(theta.device)))
    idx = torch.tensor([[0, 1, 2], [1, 3, 4], [2, 4, 5]], device=theta.device)
    return out[:, idx]


class SnrSq(torch.autograd.Function):
    """rho^2(theta) with the hand-written adjoint kernel as its backward."""

    @staticmethod
    def forward(ctx, theta, grid, seg, stilde, Sn, khi=None, precision="fp32_ph64"):
        F, Z, _ = snr_sq(grid, theta.detach(), seg, stilde, Sn, khi, precision)
        ctx.save_for_backward(theta.detach(), seg, stilde, Sn, khi if khi is not None else torch.empty(0))
        ctx.grid = grid
        ctx.precision = precision
        ctx.has_khi = khi is not None
        return F

    @staticmethod
    def backward(ctx, gF):
        theta, seg, stilde, Sn, khi = ctx.saved_tensors
        _, _, grad = snr_sq(ctx.grid, theta, seg, stilde, Sn, khi if ctx.has_khi else None, ctx.precision,
                            gbar=gF.contiguous())
        return grad, None, None, None, None, None, None
