"""ctypes declarations of libmf's C ABI (include/mf.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmf.so")

MF_OK = 0
STATUS = {0: "MF_OK", -1: "MF_E_ARG", -2: "MF_E_SHAPE", -3: "MF_E_BAND", -4: "MF_E_HIP",
          -5: "MF_E_WORKSPACE", -6: "MF_E_UNSUPPORTED"}
MF_FP64, MF_FP32_PH64, MF_FP32 = 0, 1, 2
MF_SIGMA_FP64, MF_SIGMA_COMP32 = 0, 1


class MfGrid(C.Structure):
    _fields_ = [("n", C.c_int64), ("fs", C.c_double), ("f_low", C.c_double), ("f0", C.c_double)]


class MfPeak(C.Structure):
    _fields_ = [("rho", C.c_double), ("j", C.c_int32), ("n_above", C.c_int32)]


class MfEvent(C.Structure):
    _fields_ = [("rho", C.c_double), ("j", C.c_int32), ("t", C.c_int32)]


class MfFilterOpts(C.Structure):
    _fields_ = [("rho_threshold", C.c_double), ("j_begin", C.c_int64), ("j_end", C.c_int64),
                ("series_units_dev", C.c_void_p), ("n_series", C.c_int32)]


class MfBankEntry(C.Structure):
    _fields_ = [("b1", C.c_double), ("b2", C.c_double), ("b3", C.c_double), ("b5", C.c_double),
                ("c0", C.c_double), ("sigma", C.c_double), ("k_lo", C.c_int32), ("k_hi", C.c_int32),
                ("inv_sigma", C.c_float), ("reserved", C.c_int32)]


# size of the static device array mf_filter_noalloc works in (mf.h)
MF_NOALLOC_SCRATCH_BYTES = 512 << 20


class MfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


EXPORTS = [
    "mf_last_error", "mf_version", "mf_bank_bytes", "mf_filter_workspace_bytes", "mf_psd",
    "mf_spa_bank", "mf_filter", "mf_ifft_workspace_bytes", "mf_ifft", "mf_snr_grad",
    "mf_timing_enable", "mf_timing_read", "mf_probe_copy", "mf_filter_plan", "mf_plan_candidates", "mf_set_plan",
    "mf_template_metric", "mf_chisq", "mf_filter_chisq", "mf_filter_chisq_workspace_bytes",
    "mf_psd_prefix", "mf_rfft", "mf_rfft_workspace_bytes",
    "mf_filter_events", "mf_filter_events_workspace_bytes", "mf_chisq_events", "mf_timing_read_split",
    "mf_filter_chisq_plan", "mf_set_band_plan", "mf_filter_noalloc",
]

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libmf.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libmf.so not found at {path}: build it with "
                          "`python -m paper_0906_4175_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(path)
    P = C.POINTER
    vp, i64, i32, dbl, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_size_t
    lib.mf_last_error.restype = C.c_char_p
    lib.mf_last_error.argtypes = []
    lib.mf_version.restype = C.c_char_p
    lib.mf_version.argtypes = []
    lib.mf_bank_bytes.restype = sz
    lib.mf_bank_bytes.argtypes = [i64]
    lib.mf_filter_workspace_bytes.restype = sz
    lib.mf_filter_workspace_bytes.argtypes = [P(MfGrid), C.c_int, i64, i64]
    lib.mf_psd.restype = C.c_int
    lib.mf_psd.argtypes = [P(MfGrid), vp, vp, vp]
    lib.mf_spa_bank.restype = C.c_int
    lib.mf_spa_bank.argtypes = [P(MfGrid), P(dbl), P(dbl), i64, vp, C.c_int, C.c_int, vp, P(i32), P(dbl), vp, vp]
    lib.mf_filter.restype = C.c_int
    lib.mf_filter.argtypes = [P(MfGrid), vp, i64, vp, i64, vp, C.c_int, P(MfFilterOpts), vp, sz, vp, vp, vp]
    lib.mf_filter_noalloc.restype = C.c_int
    lib.mf_filter_noalloc.argtypes = [P(MfGrid), vp, i64, vp, i64, vp, C.c_int, P(MfFilterOpts), vp, vp, vp]
    lib.mf_ifft_workspace_bytes.restype = sz
    lib.mf_ifft_workspace_bytes.argtypes = [i64, C.c_int, i64]
    lib.mf_ifft.restype = C.c_int
    lib.mf_ifft.argtypes = [i64, C.c_int, vp, vp, i64, vp, sz, vp]
    lib.mf_snr_grad.restype = C.c_int
    lib.mf_snr_grad.argtypes = [P(MfGrid), vp, vp, vp, i64, vp, i64, vp, C.c_int, vp, vp, vp, vp, vp]
    lib.mf_timing_enable.restype = C.c_int
    lib.mf_timing_enable.argtypes = [i32]
    lib.mf_timing_read.restype = C.c_int
    lib.mf_timing_read.argtypes = [P(dbl), P(i64), P(i64), P(i64)]
    lib.mf_filter_chisq_plan.restype = C.c_int
    lib.mf_filter_chisq_plan.argtypes = [P(MfGrid), C.c_int, P(i32)]
    lib.mf_timing_read_split.restype = C.c_int
    lib.mf_timing_read_split.argtypes = [P(dbl), P(i64), P(i64), P(i64)]
    lib.mf_filter_plan.restype = C.c_int
    lib.mf_filter_plan.argtypes = [P(MfGrid), C.c_int, P(i32)]
    lib.mf_plan_candidates.restype = i32
    lib.mf_plan_candidates.argtypes = [P(MfGrid), C.c_int, P(i32), i32]
    lib.mf_set_plan.restype = C.c_int
    lib.mf_set_plan.argtypes = [P(MfGrid), C.c_int, P(i32)]
    lib.mf_set_band_plan.restype = C.c_int
    lib.mf_set_band_plan.argtypes = [P(MfGrid), C.c_int, P(i32)]
    lib.mf_chisq.restype = C.c_int
    lib.mf_chisq.argtypes = [P(MfGrid), vp, i64, vp, i64, vp, vp, C.c_int, i32, vp, vp, vp, vp]
    lib.mf_filter_chisq_workspace_bytes.restype = sz
    lib.mf_filter_chisq_workspace_bytes.argtypes = [P(MfGrid), C.c_int, i64, i64, i32]
    lib.mf_filter_chisq.restype = C.c_int
    lib.mf_filter_chisq.argtypes = [P(MfGrid), vp, i64, vp, i64, vp, vp, C.c_int, i32, P(MfFilterOpts), vp, sz, vp,
                                    vp, vp, vp, vp]
    lib.mf_psd_prefix.restype = C.c_int
    lib.mf_psd_prefix.argtypes = [P(MfGrid), vp, vp, vp]
    lib.mf_rfft_workspace_bytes.restype = sz
    lib.mf_rfft_workspace_bytes.argtypes = [i64, C.c_int, i64]
    lib.mf_rfft.restype = C.c_int
    lib.mf_rfft.argtypes = [i64, dbl, C.c_int, vp, vp, i64, vp, sz, vp]
    lib.mf_filter_events_workspace_bytes.restype = sz
    lib.mf_filter_events_workspace_bytes.argtypes = [P(MfGrid), C.c_int, i64, i64, i32]
    lib.mf_filter_events.restype = C.c_int
    lib.mf_filter_events.argtypes = [P(MfGrid), vp, i64, vp, i64, vp, C.c_int, dbl, i32, vp, sz, vp, vp, vp, vp]
    lib.mf_chisq_events.restype = C.c_int
    lib.mf_chisq_events.argtypes = [P(MfGrid), vp, i64, vp, i64, vp, vp, C.c_int, i32, vp, i64, vp, vp, vp]
    lib.mf_template_metric.restype = C.c_int
    lib.mf_template_metric.argtypes = [P(MfGrid), vp, vp, i64, vp, vp, vp]
    lib.mf_probe_copy.restype = C.c_int
    lib.mf_probe_copy.argtypes = [vp, vp, sz, vp]
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != MF_OK:
        raise MfError(status, _lib.mf_last_error().decode() if _lib else "")
