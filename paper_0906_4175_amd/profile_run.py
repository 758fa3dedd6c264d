"""Workload driver for hardware-counter runs (rocprofv3 --pmc).

Runs, in one process: the calibration copy kernel over a buffer of known size
(it reads and writes exactly that many bytes), then mf_filter on a benchmark
workload for a few steps.  Usage (from the repository root):

  rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o run -- \\
      python3 paper_0906_4175_amd/profile_run.py --workload 2 --steps 2 [--chisq-bands 16]
"""
from __future__ import annotations

import argparse
import ctypes as C
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--precision", default="fp32_ph64",
                    help="precision, or several separated by commas (run one after the other)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--chisq-bands", type=int, default=0, help="also run the chi^2 band mode with p bands")
    args = ap.parse_args()

    import torch

    import paper_0906_4175_amd as mf
    import synth
    from paper_0906_4175_amd import _lib as L

    dev = torch.device("cuda:0")
    lib = L.load()
    nb = args.copy_mib << 20
    a = torch.empty(nb, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    L.check(lib.mf_probe_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), nb, None))
    torch.cuda.synchronize()
    del a, b

    if args.workload == 4:
        run_gradient(args, mf, synth, dev)
        return
    wl = synth.WORKLOADS[args.workload]
    grid = mf.Grid(wl.n, wl.fs, wl.f_low)
    Sn = mf.psd(grid, device=dev)
    Sh = Sn.cpu().numpy()
    k_lo = grid.k_lo
    rngs = synth.rngs(args.workload, wl.n_seg)
    segs = [synth.coloured_noise(Sh[k_lo: wl.n // 2], grid.df, k_lo, wl.n // 2 + 1, rngs[i], dtype=np.complex64)
            for i in range(wl.n_seg)]
    st32 = torch.from_numpy(np.stack(segs)).to(dev)
    if args.workload == 2:
        mc, eta = synth.bank_mc_eta_grid()
    else:
        mc, eta, _, _ = synth.bank_uneven({3: 8192, 5: 32768}[args.workload], synth.rngs(args.workload, 1)[0])
    for prec in args.precision.split(","):
        st = st32.to(torch.complex128) if prec == "fp64" else st32
        bank = mf.spa_bank(grid, mc, eta, Sn, prec)
        ws = torch.empty(mf.filter_workspace_bytes(grid, prec, bank.n_tmpl, wl.n_seg), dtype=torch.uint8,
                         device=dev)
        for _ in range(args.steps):
            res = mf.filter(grid, bank, st, Sn, prec, workspace=ws)
        torch.cuda.synchronize()
        del ws
        if args.chisq_bands > 0:
            _, P = mf.psd(grid, prefix=True, device=dev)
            wsb = torch.empty(mf.filter_chisq_workspace_bytes(grid, prec, bank.n_tmpl, wl.n_seg,
                                                              args.chisq_bands), dtype=torch.uint8, device=dev)
            for _ in range(args.steps):
                mf.filter_chisq(grid, bank, st, Sn, P, prec, p_bands=args.chisq_bands, workspace=wsb)
            torch.cuda.synchronize()
            del wsb
        print(f"profile_run: {args.steps} steps of {wl.name} in {prec}, max rho {float(res['rho'].max()):.4f}",
              flush=True)
    print(f"profile_run done: copy {args.copy_mib} MiB, {wl.name}")


def run_gradient(args, mf, synth, dev):
    """ρ² forward, then forward + adjoint, over 4096 triggers (4 times per template
    of the 1024-template bank, at spread times) of one 2^20 segment; prints the
    bins each dispatch evaluates (the denominator of per-bin counter figures)."""
    import torch

    wl = synth.WORKLOADS[2]
    grid = mf.Grid(wl.n, wl.fs, wl.f_low)
    Sn = mf.psd(grid, device=dev)
    Sh = Sn.cpu().numpy()
    k_lo = grid.k_lo
    seg = synth.coloured_noise(Sh[k_lo: wl.n // 2], grid.df, k_lo, wl.n // 2 + 1, synth.rngs(4, 1)[0],
                               dtype=np.complex64)
    st = torch.from_numpy(seg[None]).to(dev)
    mc, eta = synth.bank_mc_eta_grid()
    bank = mf.spa_bank(grid, mc, eta, Sn, "fp32_ph64")
    reps = 4
    T = wl.n / wl.fs
    theta = torch.tensor([[m, e, T * (0.1 + 0.2 * r)] for r in range(reps) for m, e in zip(mc, eta)],
                         dtype=torch.float64, device=dev)
    khi = torch.tensor(np.tile(bank.k_hi, reps), dtype=torch.int32, device=dev)
    segi = torch.zeros(theta.shape[0], dtype=torch.int32, device=dev)
    bins = int(np.sum(np.tile(bank.k_hi, reps).astype(np.int64) - k_lo + 1))
    for _ in range(args.steps):
        F, _, _ = mf.snr_sq(grid, theta, segi, st, Sn, khi)
    gbar = torch.ones_like(F)
    for _ in range(args.steps):
        mf.snr_sq(grid, theta, segi, st, Sn, khi, gbar=gbar)
    torch.cuda.synchronize()
    print(f"profile_run done: gradient workload, {theta.shape[0]} triggers, {bins} bins per dispatch; "
          f"{args.steps} forward then {args.steps} forward+adjoint dispatches")


if __name__ == "__main__":
    main()
