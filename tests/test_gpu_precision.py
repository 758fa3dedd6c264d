"""Precision study on the uneven bank (m1, m2 in [1, 34], M <= 35): 256 sampled
templates x 4 segments of 2^20 at 4096 Hz, every mode against the FP64 oracle.

Modes: FP64 phase or FP32 phase, FFT/products FP32 (or everything FP64), sigma
accumulated in FP64 or compensated FP32.  The target mode (FP32 with FP64 phase
and FP64 sigma) must meet: peak rho relative error <= 1e-4, peak index exact
or a near-tie (rho_oracle at the GPU index within 2e-4 of the maximum), units
with rho >= 8 exact; the FP64 path meets the same at 1e-10; the FP32-phase mode
is reported (it is expected to miss the 1e-4 bar).  The error table is written
to $MF_PRECISION_REPORT (JSON) when that variable is set.
"""
import json
import multiprocessing as mp
import os

import numpy as np
import pytest
import torch

import synth
from tests import _precision_worker as W

pytestmark = pytest.mark.gpu

N, FS, N_SEG, N_SAMPLE = 1 << 20, 4096.0, 4, 256


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0906_4175_amd as m
    return m


def test_precision_study(mf):
    print("[precision] setup", flush=True)
    rng = synth.rngs(5, 3)
    mc_all, eta_all, m1, m2 = synth.bank_uneven(32768, rng[0])
    idx = np.sort(rng[1].choice(32768, size=N_SAMPLE, replace=False))
    mc, eta = mc_all[idx], eta_all[idx]
    # one injection per segment, using sampled templates so that rho >= 8 units exist
    injections = {s: [dict(m1=float(m1[idx[7 * s]]), m2=float(m2[idx[7 * s]]), snr=10.0 + s,
                           j0=int(rng[2].integers(0, N)), phi0=float(rng[2].uniform(0, 6.28)))] for s in range(N_SEG)}
    W.init(N, FS, N_SEG, 5, injections)
    S32 = np.stack(W.segments())
    g = mf.Grid(N, FS)
    Sn = mf.psd(g)
    dev = torch.device("cuda:0")
    st32 = torch.from_numpy(S32).to(dev)
    st64 = st32.to(torch.complex128)
    modes = {"fp32_ph64+sigma_fp64": ("fp32_ph64", "fp64"), "fp32_ph64+sigma_comp32": ("fp32_ph64", "comp32"),
             "fp32_ph32+sigma_fp64": ("fp32", "fp64"), "fp32_ph32+sigma_comp32": ("fp32", "comp32"),
             "fp64": ("fp64", "fp64")}
    gpu = {}
    for name, (prec, smode) in modes.items():
        bank = mf.spa_bank(g, mc, eta, Sn, prec, smode)
        res = mf.filter(g, bank, st64 if prec == "fp64" else st32, Sn, prec)
        gpu[name] = {"rho": res["rho"].cpu().numpy(), "j": res["j"].cpu().numpy(), "sigma": bank.sigma.copy()}
        print(f"[precision] gpu {name} done", flush=True)
    tasks = [(float(mc[t]), float(eta[t]), s, {k: int(gpu[k]["j"][t, s]) for k in modes})
             for t in range(N_SAMPLE) for s in range(N_SEG)]
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs, initializer=W.init, initargs=(N, FS, N_SEG, 5, injections)) as pool:
        ora = pool.map(W.unit, tasks, chunksize=4)
    print(f"[precision] oracle done on {procs} processes", flush=True)
    report = {}
    for name in modes:
        r = gpu[name]
        rel, mism, ties, strong_bad, sig = [], 0, 0, 0, []
        for i, (t, s) in enumerate([(t, s) for t in range(N_SAMPLE) for s in range(N_SEG)]):
            o = ora[i]
            rel.append(abs(r["rho"][t, s] - o["rho"]) / o["rho"])
            jg = int(r["j"][t, s])
            if jg != o["j"]:
                mism += 1
                if o["rho_at"][name] >= o["rho"] * (1 - 2e-4):
                    ties += 1
                if o["rho"] >= 8.0:
                    strong_bad += 1
            if s == 0:
                sig.append(abs(r["sigma"][t] - o["sigma"]) / o["sigma"])
        rel = np.array(rel)
        report[name] = {"units": len(rel), "rho_rel_max": float(rel.max()), "rho_rel_p99": float(np.quantile(rel, 0.99)),
                        "rho_rel_median": float(np.median(rel)), "index_mismatch": mism, "near_tie_accepts": ties,
                        "index_mismatch_rho_ge_8": strong_bad, "sigma_rel_max": float(np.max(sig))}
        print(f"[precision] {name}: {json.dumps(report[name])}", flush=True)
    path = os.environ.get("MF_PRECISION_REPORT")
    if path:
        with open(path, "w") as fh:
            json.dump({"workload": "256 of 32768 uneven-bank templates x 4 segments, N=2^20, 4096 Hz",
                       "modes": report}, fh, indent=1)
    tgt = report["fp32_ph64+sigma_fp64"]
    assert tgt["rho_rel_max"] <= 1e-4
    assert tgt["index_mismatch"] == tgt["near_tie_accepts"] and tgt["index_mismatch_rho_ge_8"] == 0
    assert tgt["sigma_rel_max"] <= 1e-12
    assert report["fp32_ph64+sigma_comp32"]["sigma_rel_max"] <= 1e-6
    assert report["fp32_ph64+sigma_comp32"]["rho_rel_max"] <= 1e-4
    f64 = report["fp64"]
    assert f64["rho_rel_max"] <= 1e-10 and f64["index_mismatch"] == f64["near_tie_accepts"]
    assert report["fp32_ph32+sigma_fp64"]["rho_rel_max"] > tgt["rho_rel_max"]
