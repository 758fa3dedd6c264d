"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects bad arguments before enqueueing any device work."""
import ctypes as C
import math
import os
import re
import subprocess

import pytest

from paper_0906_4175_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mf.h")


@pytest.fixture(scope="module")
def lib():
    return L.load()


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mf_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["mf_psd", "mf_spa_bank", "mf_filter", "mf_snr_grad", "mf_last_error",
                     "mf_filter_workspace_bytes", "mf_bank_bytes"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mf_[a-z_0-9]+)", out))
    for name in _declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_struct_sizes_match_header(lib):
    assert C.sizeof(L.MfBankEntry) == 64
    assert C.sizeof(L.MfPeak) == 16
    assert int(lib.mf_bank_bytes(10)) == 640
    assert int(lib.mf_bank_bytes(0)) == 0


def _grid(n=1 << 20, fs=4096.0, f_low=40.0, f0=150.0):
    return L.MfGrid(n, fs, f_low, f0)


@pytest.mark.parametrize("n", [1000, 1 << 9, 1 << 23, 0, -4])
def test_bad_length_rejected(lib, n):
    g = _grid(n=n)
    assert lib.mf_psd(C.byref(g), C.c_void_p(16), None, None) == -2
    assert b"power of two" in lib.mf_last_error()


@pytest.mark.parametrize("f_low", [0.0, -1.0, 2048.0, 5000.0, math.nan])
def test_bad_band_rejected(lib, f_low):
    g = _grid(f_low=f_low)
    assert lib.mf_psd(C.byref(g), C.c_void_p(16), None, None) == -3


def test_null_pointers_rejected(lib):
    g = _grid()
    assert lib.mf_psd(C.byref(g), None, None, None) == -1
    assert lib.mf_psd(None, C.c_void_p(16), None, None) == -1
    peaks = C.c_void_p(16)
    assert lib.mf_filter(C.byref(g), None, 1, C.c_void_p(16), 1, C.c_void_p(16), 1, None,
                         C.c_void_p(256), 1 << 30, peaks, None, None) == -1


def test_bank_parameter_validation(lib):
    g = _grid()
    mc = (C.c_double * 2)(1.2, 1.2)
    for eta_bad in (0.0, 0.26, -0.1, math.nan):
        eta = (C.c_double * 2)(0.25, eta_bad)
        st = lib.mf_spa_bank(C.byref(g), mc, eta, 2, C.c_void_p(16), 1, 0, C.c_void_p(256), None, None, None, None)
        assert st == -1
        assert b"template 1" in lib.mf_last_error()
    eta = (C.c_double * 2)(0.25, 0.25)
    mcb = (C.c_double * 2)(1.2, 0.0)
    assert lib.mf_spa_bank(C.byref(g), mcb, eta, 2, C.c_void_p(16), 1, 0, C.c_void_p(256), None, None, None,
                           None) == -1
    # A 60+60 M_sun template has f_ISCO ~ 37 Hz < f_low: empty band, index named.
    mch = (C.c_double * 2)(1.2, 52.2)
    st = lib.mf_spa_bank(C.byref(g), mch, eta, 2, C.c_void_p(16), 1, 0, C.c_void_p(256), None, None, None, None)
    assert st == -3
    assert b"template 1" in lib.mf_last_error()
    # bad enums
    assert lib.mf_spa_bank(C.byref(g), mc, eta, 2, C.c_void_p(16), 7, 0, C.c_void_p(256), None, None, None,
                           None) == -1
    assert lib.mf_spa_bank(C.byref(g), mc, eta, 2, C.c_void_p(16), 1, 5, C.c_void_p(256), None, None, None,
                           None) == -1


def test_filter_workspace_and_window_validation(lib):
    g = _grid()
    need = int(lib.mf_filter_workspace_bytes(C.byref(g), 1, 1024, 1))
    # w (4 MiB) + intermediates + peak keys
    assert need >= (1 << 20) // 2 * 8 + 8 * (1 << 20) * 8
    args = lambda ws, opts=None, wsp=256: (C.byref(g), C.c_void_p(256), 1024, C.c_void_p(256), 1, C.c_void_p(256),
                                            1, opts, C.c_void_p(wsp), ws, C.c_void_p(256), None, None)
    assert lib.mf_filter(*args(need - 1)) == -5
    assert b"workspace" in lib.mf_last_error()
    assert lib.mf_filter(*args(need, wsp=264)) == -1  # misaligned workspace
    bad = L.MfFilterOpts(math.inf, 10, 5, None, 0)
    assert lib.mf_filter(*args(need, C.byref(bad))) == -2
    bad = L.MfFilterOpts(math.inf, 0, (1 << 20) + 1, None, 0)
    assert lib.mf_filter(*args(need, C.byref(bad))) == -2
    bad = L.MfFilterOpts(math.inf, 0, 0, None, 3)
    assert lib.mf_filter(*args(need, C.byref(bad))) == -1
    bad = L.MfFilterOpts(math.nan, 0, 0, None, 0)
    assert lib.mf_filter(*args(need, C.byref(bad))) == -1
    assert lib.mf_filter(*args(need)[:6], 9, *args(need)[7:]) == -1  # bad precision


def test_noalloc_validation_before_any_device_call(lib):
    # rejected on the host before the scratch is looked up (no GPU needed)
    g = _grid()
    ptr = C.c_void_p(256)
    assert lib.mf_filter_noalloc(C.byref(g), None, 4, ptr, 1, ptr, 1, None, ptr, None, None) == -1
    assert lib.mf_filter_noalloc(C.byref(g), ptr, 4, ptr, 1, ptr, 9, None, ptr, None, None) == -1
    assert lib.mf_filter_noalloc(C.byref(g), ptr, 0, ptr, 1, ptr, 1, None, ptr, None, None) == -1
    # FP64 at N = 2^22: the weights of 17 segments alone exceed the static scratch
    g22 = _grid(n=1 << 22)
    need_w = 17 * ((1 << 21) + 1) * 16
    assert need_w > L.MF_NOALLOC_SCRATCH_BYTES
    assert lib.mf_filter_noalloc(C.byref(g22), ptr, 1, ptr, 17, ptr, 0, None, ptr, None, None) == -5
    assert b"static scratch" in lib.mf_last_error()
    # the FP64 peak partials of a very large bank do not fit either
    assert lib.mf_filter_noalloc(C.byref(g), ptr, 200000, ptr, 1, ptr, 0, None, ptr, None, None) == -5


def test_ifft_and_grad_validation(lib):
    assert lib.mf_ifft_workspace_bytes(1000, 1, 1) == 0
    assert lib.mf_ifft(1 << 12, 1, None, C.c_void_p(256), 1, C.c_void_p(256), 1 << 20, None) == -1
    assert lib.mf_ifft(1 << 12, 1, C.c_void_p(256), C.c_void_p(256), 2, C.c_void_p(256), 10, None) == -5
    g = _grid()
    assert lib.mf_snr_grad(C.byref(g), None, None, C.c_void_p(256), 1, C.c_void_p(256), 1, C.c_void_p(256), 1,
                           C.c_void_p(256), C.c_void_p(256), None, None, None) == -1
    assert lib.mf_snr_grad(C.byref(g), C.c_void_p(256), None, C.c_void_p(256), 1, C.c_void_p(256), 1,
                           C.c_void_p(256), 1, C.c_void_p(256), C.c_void_p(256), C.c_void_p(256), None, None) == -1


def test_plan_candidates_and_set_plan_validation(lib):
    g = _grid()
    n = lib.mf_plan_candidates(C.byref(g), 1, None, 0)
    assert n >= 4
    buf = (C.c_int32 * (8 * n))()
    assert lib.mf_plan_candidates(C.byref(g), 1, buf, n) == n
    shapes = {tuple(buf[8 * i: 8 * i + 4]) for i in range(n)}
    assert (256, 4096, 16, 1) in shapes
    for i in range(n):
        assert buf[8 * i] * buf[8 * i + 1] == 1 << 20
    bad = (C.c_int32 * 8)(512, 512, 16, 8, 256, 256, 8, 0)  # wrong N
    assert lib.mf_set_plan(C.byref(g), 1, bad) == -6
    bad = (C.c_int32 * 8)(256, 4096, 16, 1, 256, 256, 0, 0)  # units 0
    assert lib.mf_set_plan(C.byref(g), 1, bad) == -1
    bad = (C.c_int32 * 8)(1024, 1024, 8, 4, 512, 256, 8, 1)  # fused with unequal work-groups
    assert lib.mf_set_plan(C.byref(g), 1, bad) == -6
    good = (C.c_int32 * 8)(1024, 1024, 8, 4, 512, 256, 16, 0)
    assert lib.mf_set_plan(C.byref(g), 1, good) == 0
    out = (C.c_int32 * 8)()
    assert lib.mf_filter_plan(C.byref(g), 1, out) == 0
    assert list(out)[:4] == [1024, 1024, 8, 4] and out[6] == 16
    assert lib.mf_set_plan(C.byref(g), 1, None) == 0
    assert lib.mf_filter_plan(C.byref(g), 1, out) == 0
    assert list(out)[:4] == [256, 4096, 32, 1]
    # flags: bit 0 pipelined step, bit 1 split pass-2 exchange, bit 2 its conflict-free
    # layouts, bit 3 narrow-band pass 1, bit 4 first row factor in pass 1, bit 5
    # persistent pass 1 (the 2^20 FP32 default: 2 | 4 | 8 | 16 | 32)
    assert out[7] == 62
    flags = {(tuple(buf[8 * i: 8 * i + 6]), buf[8 * i + 7]) for i in range(n)}
    for f in (0, 1, 2, 3):  # separate or pipelined launches, complex or split exchange (narrow-band pass 1 on)
        assert ((256, 4096, 16, 1, 256, 256), f | 8) in flags
    assert ((256, 4096, 16, 1, 256, 256), 32 | 8) in flags  # the tuner also times the persistent pass 1
    for f in (32, 32 | 30):  # persistent pass 1, alone and with the default flags
        good = (C.c_int32 * 8)(256, 4096, 16, 1, 256, 256, 16, f)
        assert lib.mf_set_plan(C.byref(g), 1, good) == 0
        assert lib.mf_filter_plan(C.byref(g), 1, out) == 0 and out[7] == f
    # the persistent pass 1 keeps its work order and queue counter in the workspace
    w_lpt = int(lib.mf_filter_workspace_bytes(C.byref(g), 1, 64, 1))
    good = (C.c_int32 * 8)(256, 4096, 16, 1, 256, 256, 16, 30)
    assert lib.mf_set_plan(C.byref(g), 1, good) == 0
    assert int(lib.mf_filter_workspace_bytes(C.byref(g), 1, 64, 1)) < w_lpt
    bad = (C.c_int32 * 8)(256, 4096, 16, 1, 256, 256, 16, 32 | 1)  # with the pipelined step
    assert lib.mf_set_plan(C.byref(g), 1, bad) == -6
    assert b"bit 5" in lib.mf_last_error()
    bad = (C.c_int32 * 8)(256, 4096, 16, 1, 256, 256, 16, 64)  # unknown flag bit
    assert lib.mf_set_plan(C.byref(g), 1, bad) == -1
    # bit 4 (pass 1 applies the first row factor) needs the pass-1 columns to divide N2/R0
    good = (C.c_int32 * 8)(256, 4096, 16, 1, 256, 256, 16, 16 | 14)
    assert lib.mf_set_plan(C.byref(g), 1, good) == 0
    assert lib.mf_filter_plan(C.byref(g), 1, out) == 0 and out[7] == 30
    bad = (C.c_int32 * 8)(256, 4096, 16, 1, 256, 256, 16, 16 | 1)  # with the pipelined step
    assert lib.mf_set_plan(C.byref(g), 1, bad) == -6
    g10 = _grid(n=1 << 10, fs=256.0, f_low=20.0)
    bad = (C.c_int32 * 8)(32, 32, 16, 32, 64, 64, 4, 16)  # 16 columns per tile, N2/R0 = 2
    assert lib.mf_set_plan(C.byref(g10), 1, bad) == -6
    assert b"bit 4" in lib.mf_last_error()
    bad = (C.c_int32 * 8)(256, 4096, 16, 1, 256, 256, 16, 4)  # conflict-free layouts without the split exchange
    assert lib.mf_set_plan(C.byref(g), 1, bad) == -1
    for f in (6, 7, 14):  # conflict-free split exchange, with the pipelined step, with the narrow-band pass 1
        good = (C.c_int32 * 8)(256, 4096, 16, 1, 256, 256, 16, f)
        assert lib.mf_set_plan(C.byref(g), 1, good) == 0
        assert lib.mf_filter_plan(C.byref(g), 1, out) == 0 and out[7] == f
    both = (C.c_int32 * 8)(256, 4096, 16, 1, 256, 256, 16, 3)  # pipelined step with the split exchange
    assert lib.mf_set_plan(C.byref(g), 1, both) == 0
    assert lib.mf_filter_plan(C.byref(g), 1, out) == 0 and out[7] == 3
    bad = (C.c_int32 * 8)(1024, 1024, 8, 4, 512, 256, 16, 2)  # split exchange not built for this shape
    assert lib.mf_set_plan(C.byref(g), 1, bad) == -6
    good = (C.c_int32 * 8)(256, 4096, 16, 1, 256, 256, 16, 0)
    assert lib.mf_set_plan(C.byref(g), 1, good) == 0
    assert lib.mf_filter_plan(C.byref(g), 1, out) == 0 and out[7] == 0
    assert lib.mf_set_plan(C.byref(g), 1, None) == 0
    g22 = _grid(n=1 << 22)
    assert lib.mf_filter_plan(C.byref(g22), 1, out) == 0
    assert list(out)[:4] == [1024, 4096, 16, 1] and out[7] == 30


@pytest.mark.parametrize("n, prec, shape, threads, units, flags", [
    (1 << 20, 1, [256, 4096, 32, 1], [512, 256], 1024, 62),   # FP32 (FP64 phase): 8 GiB of intermediates
    (1 << 20, 2, [256, 4096, 32, 1], [512, 256], 1024, 62),   # FP32 phase: same plan class
    (1 << 20, 0, [256, 4096, 16, 1], [256, 256], 512, 26),    # FP64: padded split exchange
    (1 << 22, 1, [1024, 4096, 16, 1], [1024, 256], 256, 30),  # 4 x 2^20 samples: conflict-free exchange
])
def test_default_plans(lib, n, prec, shape, threads, units, flags):
    g = _grid(n=n)
    assert lib.mf_set_plan(C.byref(g), prec, None) == 0
    out = (C.c_int32 * 8)()
    assert lib.mf_filter_plan(C.byref(g), prec, out) == 0
    assert list(out)[:4] == shape and list(out)[4:6] == threads and out[6] == units
    assert out[7] == flags  # separate launches, split pass-2 exchange, narrow-band pass 1, first row factor in pass 1


def test_tune_cache_corrupt_and_foreign(tmp_path):
    import warnings
    from paper_0906_4175_amd import tune
    p = tmp_path / "cache.json"
    p.write_text("{not json")
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        assert tune.load_cache(str(p), arch="gfx950") == 0
        assert any("ignored" in str(x.message) for x in w)
    # a well-formed cache for another architecture installs nothing
    tune.save_cache(str(p), "gfx942", 1 << 20, 1, {k: 1 for k in tune.PLAN_KEYS})
    assert tune.load_cache(str(p), arch="gfx950") == 0
    # a valid entry for this architecture is installed, a bad one is skipped
    plan = dict(n1=1024, n2=1024, cols_per_wg=8, rows_per_wg=4, threads_pass1=512, threads_pass2=256,
                units_per_batch=32, flags=0)
    tune.save_cache(str(p), "gfx950", 1 << 20, 1, plan, 1.0)
    tune.save_cache(str(p), "gfx950", 1 << 16, 1, dict(plan, n1=7), 1.0)
    with warnings.catch_warnings(record=True):
        warnings.simplefilter("always")
        assert tune.load_cache(str(p), arch="gfx950") == 1
    assert tune.current_plan(1 << 20, 1)["units_per_batch"] == 32
    tune.set_plan(1 << 20, 1, None)
    assert tune.current_plan(1 << 20, 1)["n1"] == 256


def test_chisq_entry_points_validation(lib):
    g = _grid()
    vp = C.c_void_p
    # point chi^2: bad band count, null pointers, bad precision
    args = lambda p=16, prec=1, peaks=vp(256): (C.byref(g), vp(256), 4, vp(256), 1, vp(256), vp(256), prec, p, peaks,
                                                vp(256), None, None)
    assert lib.mf_chisq(*args(p=1)) == -1
    assert b"p_bands" in lib.mf_last_error()
    assert lib.mf_chisq(*args(p=65)) == -1
    assert lib.mf_chisq(*args(peaks=None)) == -1
    assert lib.mf_chisq(*args(prec=9)) == -1
    # band-mode filter: workspace size depends on p and the batch, rejects bad p
    w16 = int(lib.mf_filter_chisq_workspace_bytes(C.byref(g), 1, 8, 2, 16))
    w64 = int(lib.mf_filter_chisq_workspace_bytes(C.byref(g), 1, 8, 2, 64))
    assert w64 > w16 > 0
    # weights + product + one intermediate per unit of the batch
    assert w16 >= 2 * ((1 << 19) + 1) * 8 + 16 * (3 << 19) * 8
    assert lib.mf_filter_chisq_workspace_bytes(C.byref(g), 1, 8, 2, 1) == 0
    assert lib.mf_filter_chisq_workspace_bytes(C.byref(g), 1, 8, 2, 65) == 0
    fargs = lambda ws, p=16, chi=vp(256), opts=None, wsp=256: (
        C.byref(g), vp(256), 8, vp(256), 2, vp(256), vp(256), 1, p, opts, vp(wsp), ws, vp(256), chi, None, None, None)
    assert lib.mf_filter_chisq(*fargs(w16 - 1)) == -5
    assert lib.mf_filter_chisq(*fargs(w16, chi=None)) == -1
    assert lib.mf_filter_chisq(*fargs(w16, p=0)) == -1
    assert lib.mf_filter_chisq(*fargs(w16, wsp=264)) == -1
    su = L.MfFilterOpts(math.inf, 0, 0, vp(256), 2)  # series without output arrays
    assert lib.mf_filter_chisq(*fargs(w16, opts=C.byref(su))) == -1
    assert b"chisq_series" in lib.mf_last_error()


def test_set_band_plan_validation(lib):
    """The band mode's launch plan is set only through mf_set_band_plan (no hidden switches)."""
    g = _grid()
    out = (C.c_int32 * 8)()
    assert lib.mf_set_band_plan(C.byref(g), 1, None) == 0
    assert lib.mf_filter_chisq_plan(C.byref(g), 1, out) == 0
    default = list(out)
    assert default[:6] == [256, 4096, 16, 1, 256, 256] and default[6] == 24 and default[7] == 0
    w_default = int(lib.mf_filter_chisq_workspace_bytes(C.byref(g), 1, 64, 1, 16))
    r8 = (C.c_int32 * 8)(*(default[:5] + [512, 5, 0]))  # radix-8 rows, 5 units per batch
    assert lib.mf_set_band_plan(C.byref(g), 1, r8) == 0
    assert lib.mf_filter_chisq_plan(C.byref(g), 1, out) == 0
    assert list(out)[5:7] == [512, 5]
    # the workspace follows the installed batch
    assert int(lib.mf_filter_chisq_workspace_bytes(C.byref(g), 1, 64, 1, 16)) < w_default
    bad = (C.c_int32 * 8)(*(default[:5] + [384, 5, 0]))  # no such row radix
    assert lib.mf_set_band_plan(C.byref(g), 1, bad) == -6
    bad = (C.c_int32 * 8)(*(default[:6] + [0, 0]))  # units 0
    assert lib.mf_set_band_plan(C.byref(g), 1, bad) == -1
    bad = (C.c_int32 * 8)(*(default[:6] + [4, 1]))  # flags must be 0
    assert lib.mf_set_band_plan(C.byref(g), 1, bad) == -1
    bad = (C.c_int32 * 8)(512, 512, 16, 8, 512, 256, 4, 0)  # wrong N
    assert lib.mf_set_band_plan(C.byref(g), 1, bad) == -6
    # the FP64 class is separate and keeps its default
    assert lib.mf_filter_chisq_plan(C.byref(g), 0, out) == 0 and out[6] == 12
    assert lib.mf_set_band_plan(C.byref(g), 1, None) == 0
    assert lib.mf_filter_chisq_plan(C.byref(g), 1, out) == 0 and list(out) == default


def test_no_environment_switches_in_the_library():
    """Launch structure and workspace layout depend only on declared calls."""
    csrc = os.path.join(ROOT, "paper_0906_4175_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        txt = open(os.path.join(csrc, f)).read()
        assert "getenv" not in txt, f


def test_kernel_hash_ignores_comments_and_whitespace(tmp_path, monkeypatch):
    """Profiles stay valid across comment edits and go stale on code edits."""
    from paper_0906_4175_amd import profile_summary as ps
    code = "__global__ void k(float* x) { x[threadIdx.x] *= 2.0f; }\n"
    f = tmp_path / "k.hip"
    monkeypatch.setattr(ps, "KERNEL_SOURCES", [str(f)])
    f.write_text(code)
    h0 = ps.kernel_hash()
    f.write_text("// a note\n/* a block\n   comment */\n" + code.replace("{ ", "{\n    ") + "// end\n")
    assert ps.kernel_hash() == h0
    f.write_text(code.replace("2.0f", "3.0f"))
    assert ps.kernel_hash() != h0
