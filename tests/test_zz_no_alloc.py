"""mf_filter_noalloc (the library's static device scratch instead of a
caller workspace) against mf_filter, through the C ABI.

Every launch plan gives bitwise the same peaks, so the bar is bitwise
equality of the peak records (rho, index, threshold count) and of the rho
series.  Two calls in a row, the second smaller, so the second runs on the
first one's leftover scratch contents.
"""
import numpy as np
import pytest
import torch

import synth
from paper_0906_4175_amd import _lib as L
from tests import _data as D

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0906_4175_amd as m
    return m


def _inputs(mf, n, fs, n_tmpl, n_seg, prec, seed):
    dev = torch.device("cuda:0")
    cdt = np.complex128 if prec == "fp64" else np.complex64
    segs = []
    for s in range(n_seg):
        inj = [dict(m1=1.6, m2=1.3, snr=11.0, j0=(12345 + 777 * s) % n, phi0=0.4 + s)]
        x, _ = D.segment(n, fs, seed + s, injections=inj, dtype=cdt)
        segs.append(x)
    stilde = torch.from_numpy(np.stack(segs)).to(dev)
    g = mf.Grid(n, fs)
    Sn = mf.psd(g, device=dev)
    mc, eta, _, _ = synth.bank_uneven(n_tmpl, np.random.Generator(np.random.PCG64(seed)))
    mc = np.concatenate([synth.mc_eta(1.6, 1.3)[0][None], mc[: n_tmpl - 1]])
    eta = np.concatenate([synth.mc_eta(1.6, 1.3)[1][None], eta[: n_tmpl - 1]])
    bank = mf.spa_bank(g, mc, eta, Sn, prec)
    return g, bank, stilde, Sn


def _compare(mf, g, bank, stilde, Sn, prec, threshold, window, series_units):
    dev = stilde.device
    n_seg = stilde.shape[0]
    ref = mf.filter(g, bank, stilde, Sn, prec, threshold=threshold, window=window, series_units=series_units)
    peaks = torch.full((2 * bank.n_tmpl * n_seg,), float("nan"), dtype=torch.float64, device=dev)
    su = torch.as_tensor(np.asarray(series_units, dtype=np.int32), device=dev)
    sdt = torch.float64 if prec == "fp64" else torch.float32
    series = torch.full((su.numel(), g.n), float("nan"), dtype=sdt, device=dev)
    got = mf.filter_noalloc(g, bank, stilde, Sn, peaks, prec, threshold=threshold, window=window,
                            series_ptr=series.data_ptr(), series_units_ptr=su.data_ptr(), n_series=su.numel())
    torch.cuda.synchronize()
    assert torch.equal(got["raw"].view(torch.int64), ref["raw"].view(torch.int64))
    assert torch.equal(series.view(torch.int32 if prec != "fp64" else torch.int64),
                       ref["series"].view(torch.int32 if prec != "fp64" else torch.int64))
    assert int(got["n_above"].sum()) > 0
    return got


@pytest.mark.parametrize("prec", ["fp32_ph64", "fp64"])
def test_noalloc_matches_filter_two_calls(mf, prec):
    n, fs = 1 << 20, 4096.0
    # first call: more units than one batch of the static scratch holds
    # (63 per batch in FP32, 31 in FP64 at N = 2^20), with a ragged last batch
    print(f"[noalloc] {prec} call 1: 80 templates x 2 segments", flush=True)
    g, bank, stilde, Sn = _inputs(mf, n, fs, 80, 2, prec, 20090906)
    got = _compare(mf, g, bank, stilde, Sn, prec, 4.5, None, [0, 1, 77, 159])
    # the injected template finds its injection on both segments
    assert abs(int(got["j"][0, 0]) - 12345) <= 2 and abs(int(got["j"][0, 1]) - (12345 + 777)) <= 2
    # second call: smaller, windowed, on the scratch the first call left behind
    print(f"[noalloc] {prec} call 2: 9 templates x 1 segment, window", flush=True)
    g, bank, stilde, Sn = _inputs(mf, n, fs, 9, 1, prec, 4242)
    _compare(mf, g, bank, stilde, Sn, prec, 4.0, (1000, n - 5000), [3])


def test_noalloc_rejects_oversized_request(mf):
    # FP64 at N = 2^22: 16 segments of weights alone exceed the static scratch
    n, fs = 1 << 22, 4096.0
    g = mf.Grid(n, fs)
    dev = torch.device("cuda:0")
    Sn = mf.psd(g, device=dev)
    bank = mf.spa_bank(g, *synth.mc_eta(np.array([1.4]), np.array([1.4])), Sn, "fp64")
    stilde = torch.zeros((17, n // 2 + 1), dtype=torch.complex128, device=dev)
    peaks = torch.empty(2 * 17, dtype=torch.float64, device=dev)
    with pytest.raises(L.MfError) as e:
        mf.filter_noalloc(g, bank, stilde, Sn, peaks, "fp64")
    assert e.value.status == -5
    assert "static scratch" in str(e.value)
