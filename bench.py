#!/usr/bin/env python3
"""Throughput of the matched-filter hot path on one MI355X.

One step = one mf_filter call over the whole workload: per-segment data
weights, then for every (template, segment) unit the stationary-phase template,
the weighted product, the 2^20-point inverse DFT, rho = |z|/sigma and its
peak / threshold count.  Inputs (data spectra, PSD, bank) are resident in HBM
before the timed region.

Prints ONE JSON line: units/s (templates x segments per second), the roofline
of the dominant kernel (HIP events on the launch stream during the timed
steps), the plain FP64 path on the same GPU, and the FP64 oracle timed on the
host cores over a bounded sample of the same workload.

The default workload is the largest single-GPU one: 32768 uneven templates x 4
segments of 2^20 samples.  Extra legs: the plain FP64 path and HIP-graph replay
on the same workload; the single-segment workload (1024 templates x one 2^20
segment with 5 injections) with the chi^2 band mode, events and the 4 x 2^20
segment length.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2|3|5]
"""
from __future__ import annotations

import argparse
import contextlib
import gc
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "templates×segments/s at 2^20-pt IFFT; HBM GB/s fraction; vs FP64 path"
UNIT = "templates×segments/s"
HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")

@contextlib.contextmanager
def quiet_gc():
    """Timed regions run with a fresh heap and the garbage collector off (as timeit
    does): a full collection of an interpreter that holds torch takes tens of ms."""
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()


def kernel_hash() -> str:
    from paper_0906_4175_amd.profile_summary import kernel_hash as khash
    return khash()


def workload_bank(cfg: int):
    """(mc, eta) of the workload's template bank."""
    if cfg == 2:
        return synth.bank_mc_eta_grid()
    if cfg == 3:
        mc, eta, _, _ = synth.bank_uneven(8192, synth.rngs(3, 1)[0])
        return mc, eta
    if cfg == 5:
        mc, eta, _, _ = synth.bank_uneven(32768, synth.rngs(5, 1)[0])
        return mc, eta
    raise SystemExit(f"workload {cfg} is not a filter-throughput workload (use 2, 3 or 5)")


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on the host cores (runs before any GPU use)
# ---------------------------------------------------------------------------
_CPU = {}


def _cpu_unit(t: int):
    import oracle as O
    d = _CPU
    out = O.filter_unit(d["n"], d["fs"], 40.0, float(d["mc"][t]), float(d["eta"][t]), d["s"], d["Sn"])
    return out["rho"]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg: int, seconds: float, max_procs: int):
    """The FP64 oracle on the host cores, one process per core, over a bounded
    sample of the workload's templates on its first segment.  The process count
    is the number of cores this process may run on, capped at max_procs (the
    host's CPU share for one GPU on the boxes this runs on is 16 cores)."""
    import multiprocessing as mp

    import oracle as O
    wl = synth.WORKLOADS[cfg]
    n, fs = wl.n, wl.fs
    g = O.grid(n, fs)
    Sn = O.psd_bins(n, fs, wl.f_low)
    k_lo = O.band_lo(n, fs, wl.f_low)
    rng = synth.rngs(cfg, 1)[0]
    s = synth.coloured_noise(Sn[k_lo: n // 2], g["df"], k_lo, n // 2 + 1, rng, dtype=np.complex64)
    mc, eta = workload_bank(cfg)
    _CPU.update(n=n, fs=fs, s=s.astype(np.complex128), Sn=Sn, mc=mc, eta=eta)
    affinity = len(os.sched_getaffinity(0))
    procs = max(1, min(max_procs, affinity))
    t0 = time.perf_counter()
    _cpu_unit(0)
    t_one = time.perf_counter() - t0
    n_units = int(min(len(mc), max(procs, round(procs * seconds / max(t_one, 1e-3)))))
    idx = np.linspace(0, len(mc) - 1, n_units).astype(int).tolist()
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        pool.map(_cpu_unit, idx, chunksize=1)
    dt = time.perf_counter() - t0
    return {"value": n_units / dt, "unit": UNIT, "cores": procs, "kind": "oracle",
            "sample": f"{n_units} of the {len(mc)} templates x 1 segment (N={n}), FP64 NumPy oracle, "
                      f"{procs} single-threaded processes, {dt:.1f} s wall",
            "affinity_cpus": affinity, "cpu_model": cpu_model()}


# ---------------------------------------------------------------------------
# GPU
# ---------------------------------------------------------------------------
def read_traffic(kernel: str, workload: str, khash: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it is
    for the current kernel source; else None."""
    path = os.path.join(PROFILE_DIR, f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != khash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_gpu(args):
    import torch

    import paper_0906_4175_amd as mf
    from paper_0906_4175_amd import _lib as L

    dev = torch.device("cuda:0")

    class Inputs:
        """A workload's grid, PSD, bank parameters and data spectra, resident on the GPU."""

        def __init__(self, cfg: int):
            wl = synth.WORKLOADS[cfg]
            self.cfg, self.wl = cfg, wl
            self.grid = mf.Grid(wl.n, wl.fs, wl.f_low)
            self.Sn = mf.psd(self.grid, device=dev)
            Sn_h = self.Sn.cpu().numpy()
            self.mc, self.eta = workload_bank(cfg)
            self.n_seg = wl.n_seg
            k_lo = self.grid.k_lo
            rngs = synth.rngs(cfg, wl.n_seg + 1)
            segs = [synth.coloured_noise(Sn_h[k_lo: wl.n // 2], self.grid.df, k_lo, wl.n // 2 + 1, rngs[i],
                                         dtype=np.complex64) for i in range(wl.n_seg)]
            if cfg == 2:
                # five injections with SNR 8-15, templates synthesised by the library itself
                injs = synth.injection_params(rngs[-1], 5, wl.n)
                imc, ieta = synth.mc_eta([i["m1"] for i in injs], [i["m2"] for i in injs])
                ib = mf.spa_bank(self.grid, imc, ieta, self.Sn, "fp32_ph64", materialise=True)
                ht = ib.htilde.cpu().numpy()
                for q, inj in enumerate(injs):
                    segs[0] = synth.inject(segs[0], ht[q], inj["snr"] / ib.sigma[q], inj["phi0"], inj["j0"], wl.n)
            self.S32 = torch.from_numpy(np.stack(segs)).to(dev)
            self._S64 = None

        def stilde(self, prec: str):
            if prec != "fp64":
                return self.S32
            if self._S64 is None:
                self._S64 = self.S32.to(torch.complex128)
            return self._S64

    def measure(inp, prec: str, steps: int, warmup: int, stride: int):
        grid, Sn, n_seg = inp.grid, inp.Sn, inp.n_seg
        bank = mf.spa_bank(grid, inp.mc, inp.eta, Sn, prec)
        st = inp.stilde(prec)
        ws = torch.empty(mf.filter_workspace_bytes(grid, prec, bank.n_tmpl, n_seg), dtype=torch.uint8, device=dev)
        peaks = torch.empty(2 * bank.n_tmpl * n_seg, dtype=torch.float64, device=dev)
        for _ in range(warmup):
            res = mf.filter(grid, bank, st, Sn, prec, workspace=ws, peaks=peaks)
        torch.cuda.synchronize()
        lib = L.load()
        lib.mf_timing_enable(stride)
        with quiet_gc():
            t0 = time.perf_counter()
            for _ in range(steps):
                res = mf.filter(grid, bank, st, Sn, prec, workspace=ws, peaks=peaks)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        import ctypes as C
        ms, nl, u1, u2 = C.c_double(), C.c_int64(), C.c_int64(), C.c_int64()
        L.check(lib.mf_timing_read(C.byref(ms), C.byref(nl), C.byref(u1), C.byref(u2)))
        lib.mf_timing_enable(0)
        b = 16 if prec == "fp64" else 8
        n = inp.wl.n
        n_act = (bank.k_hi.astype(np.int64) - grid.k_lo + 1)
        # per-unit algorithmic bytes (averaged over the workload's units):
        #   pass 1 reads the weights over the band and writes the intermediate,
        #   pass 2 reads the intermediate and writes a 16-byte peak record
        pass1_unit = float(np.mean(b * n_act + b * n))
        pass2_unit = float(b * n + 16)
        out = {"prec": prec, "ms_per_step": 1e3 * wall / steps, "steps": steps, "plan": mf.filter_plan(grid, prec),
               "units": bank.n_tmpl * n_seg, "peaks": res,
               "kern": {"ms": ms.value, "launches": nl.value, "u1": u1.value, "u2": u2.value,
                        "bytes": u1.value * pass1_unit + u2.value * pass2_unit},
               "b_alg_unit": float(np.mean(b * n_act + 2 * b * n + 16)),
               "mean_active_bins": float(np.mean(n_act))}
        del ws
        return out

    def measure_chisq(inp, prec: str, steps: int, warmup: int, stride: int, p_bands: int):
        """Band mode: the filter plus chi^2 (Eq. (5)) at every sample of every unit."""
        import ctypes as C
        grid, Sn, n_seg = inp.grid, inp.Sn, inp.n_seg
        bank = mf.spa_bank(grid, inp.mc, inp.eta, Sn, prec)
        _, P = mf.psd(grid, prefix=True, device=dev)
        st = inp.stilde(prec)
        ws = torch.empty(mf.filter_chisq_workspace_bytes(grid, prec, bank.n_tmpl, n_seg, p_bands),
                         dtype=torch.uint8, device=dev)
        for _ in range(warmup):
            res = mf.filter_chisq(grid, bank, st, Sn, P, prec, p_bands=p_bands, workspace=ws)
        torch.cuda.synchronize()
        lib = L.load()
        lib.mf_timing_enable(stride)
        with quiet_gc():
            t0 = time.perf_counter()
            for _ in range(steps):
                res = mf.filter_chisq(grid, bank, st, Sn, P, prec, p_bands=p_bands, workspace=ws)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        ms, nl, u1, u2 = (C.c_double * 3)(), (C.c_int64 * 3)(), (C.c_int64 * 3)(), (C.c_int64 * 3)()
        L.check(lib.mf_timing_read_split(ms, nl, u1, u2))
        lib.mf_timing_enable(0)
        units = bank.n_tmpl * n_seg
        chi = res["chisq"].cpu().numpy()
        return {"prec": prec, "p_bands": p_bands, "ms_per_step": 1e3 * wall / steps, "steps": steps, "units": units,
                "plan": mf.filter_chisq_plan(grid, prec),
                "pass2": {"ms": ms[1], "launches": nl[1], "units": u2[1]},
                "pass1": {"ms": ms[0], "launches": nl[0], "units": u1[0]},
                "chisq_at_peaks_median": float(np.median(chi))}

    def measure_events(inp, prec: str, steps: int, threshold: float, log2w: int, p_bands: int):
        """Events path: filter + clustering, then chi^2 at the segment events."""
        grid, Sn, n_seg = inp.grid, inp.Sn, inp.n_seg
        bank = mf.spa_bank(grid, inp.mc, inp.eta, Sn, prec)
        _, P = mf.psd(grid, prefix=True, device=dev)
        st = inp.stilde(prec)
        ws = torch.empty(mf.filter_events_workspace_bytes(grid, prec, bank.n_tmpl, n_seg, log2w), dtype=torch.uint8,
                         device=dev)

        def step():
            r = mf.filter_events(grid, bank, st, Sn, prec, threshold=threshold, log2_window=log2w, workspace=ws)
            c, _ = mf.chisq_events(grid, bank, st, Sn, P, r["seg_events"], prec, p_bands=p_bands)
            return r, c
        for _ in range(3):  # warm-up steps, as in the other legs
            step()
        torch.cuda.synchronize()
        with quiet_gc():
            t0 = time.perf_counter()
            for _ in range(steps):
                res, chi = step()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        ev = res["seg_events"]
        t, j, rho = ev["t"].cpu().numpy(), ev["j"].cpu().numpy(), ev["rho"].cpu().numpy()
        chi = chi.cpu().numpy()
        recs = {(s_, w): (int(t[s_, w]), int(j[s_, w]), float(rho[s_, w]), float(chi[s_, w]))
                for s_ in range(t.shape[0]) for w in range(t.shape[1]) if t[s_, w] >= 0}
        return {"ms_per_step": 1e3 * wall / steps, "steps": steps, "units": bank.n_tmpl * n_seg, "events": recs}

    def measure_n4m(inp, prec: str, steps: int):
        """The filter on 4 x 2^20-sample segments (1024 s at 4096 Hz), same bank."""
        wl = inp.wl
        g4 = mf.Grid(wl.n * 4, wl.fs, wl.f_low)
        Sn4 = mf.psd(g4, device=dev)
        S4h = Sn4.cpu().numpy()
        s4 = synth.coloured_noise(S4h[g4.k_lo: g4.n // 2], g4.df, g4.k_lo, g4.n // 2 + 1,
                                  synth.rngs(inp.cfg, 1)[0], dtype=np.complex64 if prec != "fp64" else np.complex128)
        st4 = torch.from_numpy(s4[None]).to(dev)
        bank = mf.spa_bank(g4, inp.mc, inp.eta, Sn4, prec)
        ws = torch.empty(mf.filter_workspace_bytes(g4, prec, bank.n_tmpl, 1), dtype=torch.uint8, device=dev)
        peaks = torch.empty(2 * bank.n_tmpl, dtype=torch.float64, device=dev)
        for _ in range(3):  # warm-up steps
            mf.filter(g4, bank, st4, Sn4, prec, workspace=ws, peaks=peaks)
        torch.cuda.synchronize()
        with quiet_gc():
            t0 = time.perf_counter()
            for _ in range(steps):
                mf.filter(g4, bank, st4, Sn4, prec, workspace=ws, peaks=peaks)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        del ws
        return {"ms_per_step": 1e3 * wall / steps, "steps": steps, "units": bank.n_tmpl, "n": g4.n,
                "plan": mf.filter_plan(g4, prec)}

    def measure_graph(inp, prec: str, replays: int):
        """The step captured once in a HIP graph and replayed.  Replays and eager steps
        alternate (so both see the same clock), each timed with an event pair on the
        stream it runs on; medians are reported, and every replay's peaks are checked
        against the eager result."""
        grid, Sn, n_seg = inp.grid, inp.Sn, inp.n_seg
        bank = mf.spa_bank(grid, inp.mc, inp.eta, Sn, prec)
        st = inp.stilde(prec)
        ws = torch.empty(mf.filter_workspace_bytes(grid, prec, bank.n_tmpl, n_seg), dtype=torch.uint8, device=dev)
        peaks = torch.empty(2 * bank.n_tmpl * n_seg, dtype=torch.float64, device=dev)
        eager_peaks = torch.empty_like(peaks)
        mf.filter(grid, bank, st, Sn, prec, workspace=ws, peaks=eager_peaks)
        ref = eager_peaks.clone()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # warm-up off the capture stream
            mf.filter(grid, bank, st, Sn, prec, workspace=ws, peaks=peaks)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            mf.filter(grid, bank, st, Sn, prec, workspace=ws, peaks=peaks)
        torch.cuda.synchronize()
        same = True
        for _ in range(3):  # warm-up replays and steps
            graph.replay()
            mf.filter(grid, bank, st, Sn, prec, workspace=ws, peaks=eager_peaks)
        torch.cuda.synchronize()
        t_graph, t_eager = [], []
        with quiet_gc():
            for _ in range(replays):
                peaks.fill_(-1.0)
                e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
                e0.record()
                graph.replay()
                e1.record()
                mf.filter(grid, bank, st, Sn, prec, workspace=ws, peaks=eager_peaks)
                e2.record()
                e2.synchronize()
                t_graph.append(e0.elapsed_time(e1))
                t_eager.append(e1.elapsed_time(e2))
                same = same and bool(torch.equal(peaks, ref)) and bool(torch.equal(eager_peaks, ref))
        del graph, ws
        return {"units": bank.n_tmpl * n_seg, "replays": replays, "peaks_equal_eager": same,
                "graph_ms_median": float(np.median(t_graph)), "eager_ms_median": float(np.median(t_eager)),
                "graph_ms": [round(x, 4) for x in t_graph], "eager_ms": [round(x, 4) for x in t_eager]}

    main_inp = Inputs(args.workload)
    tuned = None
    if args.tune:
        # time every built plan on this workload and install the fastest (untimed)
        from paper_0906_4175_amd import tune
        tb = mf.spa_bank(main_inp.grid, main_inp.mc, main_inp.eta, main_inp.Sn, args.precision)
        r = tune.tune(main_inp.grid, tb, main_inp.stilde(args.precision), main_inp.Sn, args.precision,
                      units=(256, 512, 1024), steps=2, warmup=1, install=True)
        tuned = {"plan": r["best"], "ms": round(r["best_ms"], 4), "candidates": len(r["table"])}
        del tb
    print(f"[bench] main leg: {args.steps} steps", file=sys.stderr, flush=True)
    main = measure(main_inp, args.precision, args.steps, args.warmup, args.timing_stride)
    main["tuned"] = tuned
    graph = None
    if args.graph_replays > 0:
        print("[bench] graph leg", file=sys.stderr, flush=True)
        graph = measure_graph(main_inp, args.precision, args.graph_replays)
    fp64 = None
    if args.fp64_steps > 0:
        print("[bench] fp64 leg", file=sys.stderr, flush=True)
        fp64 = measure(main_inp, "fp64", args.fp64_steps, 2, args.timing_stride)
    main_inp.__dict__.pop("_S64", None)
    # legs on the single-segment workload (1024 templates x one 2^20 segment)
    seg_inp = main_inp if args.workload == 2 else Inputs(2)
    single = None
    if args.workload != 2 and args.single_steps > 0:
        print("[bench] single-segment leg", file=sys.stderr, flush=True)
        single = measure(seg_inp, args.precision, args.single_steps, 3, args.timing_stride)
    chisq = None
    if args.chisq_steps > 0:
        print("[bench] chi^2 leg", file=sys.stderr, flush=True)
        chisq = measure_chisq(seg_inp, args.precision, args.chisq_steps, 2, args.timing_stride, args.chisq_bands)
    events = None
    if args.events_steps > 0:
        print("[bench] events leg", file=sys.stderr, flush=True)
        e32 = measure_events(seg_inp, args.precision, args.events_steps, args.events_threshold, args.events_log2w,
                             args.chisq_bands)
        e64 = measure_events(seg_inp, "fp64", 1, args.events_threshold, args.events_log2w, args.chisq_bands)
        events = (e32, e64)
    n4m = None
    if args.n4m_steps > 0:
        print("[bench] 4M-point leg", file=sys.stderr, flush=True)
        n4m = measure_n4m(seg_inp, args.precision, args.n4m_steps)
    return main, fp64, chisq, events, n4m, graph, single, seg_inp.wl


def run_refine(args):
    """Gradient refinement of 4096 triggers (4 windows x 1024 templates of the
    single-segment workload): 20 preconditioned ascent steps through the
    forward / adjoint kernels.  ALU-bound; reported as evaluations per second."""
    import torch

    import paper_0906_4175_amd as mf
    from paper_0906_4175_amd import refine as R

    wl = synth.WORKLOADS[2]
    dev = torch.device("cuda:0")
    grid = mf.Grid(wl.n, wl.fs, wl.f_low)
    Sn = mf.psd(grid, device=dev)
    Sh = Sn.cpu().numpy()
    k_lo = grid.k_lo
    rngs = synth.rngs(2, 2)
    seg = synth.coloured_noise(Sh[k_lo: wl.n // 2], grid.df, k_lo, wl.n // 2 + 1, rngs[0], dtype=np.complex64)
    injs = synth.injection_params(rngs[1], 5, wl.n)
    imc, ieta = synth.mc_eta([i["m1"] for i in injs], [i["m2"] for i in injs])
    ib = mf.spa_bank(grid, imc, ieta, Sn, "fp32_ph64", materialise=True)
    ht = ib.htilde.cpu().numpy()
    for q, inj in enumerate(injs):
        seg = synth.inject(seg, ht[q], inj["snr"] / ib.sigma[q], inj["phi0"], inj["j0"], wl.n)
    st = torch.from_numpy(seg[None]).to(dev)
    mc, eta = workload_bank(2)
    bank = mf.spa_bank(grid, mc, eta, Sn, "fp32_ph64")
    theta0, khi, segi, rho0 = R.triggers_from_peaks(grid, bank, st, Sn, mc, eta, n_windows=4)
    n_trig = theta0.shape[0]
    # warm-up, then the timed refinement
    R.refine(grid, theta0[:64], segi[:64], st, Sn, khi[:64], steps=1)
    torch.cuda.synchronize()
    with quiet_gc():
        t0 = time.perf_counter()
        theta, F, evals = R.refine(grid, theta0, segi, st, Sn, khi, steps=args.refine_steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    # finite-difference check of the adjoint on 64 triggers, at their starting
    # points (after refinement the gradient vanishes and a relative check is void)
    sel = torch.arange(0, n_trig, max(1, n_trig // 64), device=dev)[:64]
    th_chk = theta0[sel]
    F_chk, g = R.rho2_and_grad(grid, th_chk, segi[sel], st, Sn, khi[sel])
    fd = R.finite_difference_grad(grid, th_chk, segi[sel], st, Sn, khi[sel])
    Dm = torch.stack([th_chk[:, 0] * 1e-3, torch.full_like(th_chk[:, 0], 1e-3), torch.full_like(th_chk[:, 0], 1e-4)],
                     dim=1)
    num = ((Dm * (g - fd)) ** 2).sum(1).sqrt()
    den = ((Dm * fd) ** 2).sum(1).sqrt() + 1e-6 * F_chk
    fd_rel = float((num / den).max())
    n_act = float(np.mean(bank.k_hi.astype(np.int64) - k_lo + 1))
    evals_total = evals * n_trig
    line = {
        "metric": "trigger rho^2 evaluations/s (forward or adjoint, N=2^20 band)", "value": round(evals_total / wall, 1),
        "unit": "evaluations/s", "n_gpus": 1, "steps": args.refine_steps, "warmup": 1,
        "ms_per_step": round(1e3 * wall / args.refine_steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": synth.WORKLOADS[4].name, "triggers": n_trig, "mean_band_bins": round(n_act),
                   "refine_steps": args.refine_steps},
        "rho2_gain_median": round(float((F / rho0 ** 2).median()), 5),
        "fd_check_max_rel": fd_rel, "fd_check_triggers": int(sel.numel()),
        "bin_evaluations_per_s": round(evals_total * n_act / wall, 1),
    }
    line["roofline"] = refine_roofline(line["bin_evaluations_per_s"], wl_name="gradient-4096trig")
    print(json.dumps(line), flush=True)


def refine_roofline(bin_evals_per_s: float, wl_name: str):
    """ALU roofline of the refinement: bin evaluations/s x the FP32 + FP64 VALU flops of one
    forward bin evaluation, counted with SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F{32,64} in the committed
    profile (an adjoint evaluation costs more, so this is a lower bound)."""
    path = os.path.join(PROFILE_DIR, f"flops_k_snr_grad_fp32_{wl_name}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for ln in fh:
            if ":" in ln and not ln.startswith("#"):
                k, v = ln.split(":", 1)
                vals[k.strip()] = v.strip()
    try:
        per_bin = float(vals["total_flops_per_element_min"])
    except (KeyError, ValueError):
        return None
    ach = bin_evals_per_s * per_bin / 1e12
    return {"bound": "alu", "achieved": round(ach, 2), "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / FP64_VALU_PEAK_TFLOPS, 4), "traffic": None, "kernel": "k_snr_grad",
            "flops_per_bin_evaluation": per_bin, "note": "forward-evaluation flops (lower bound)"}


def launches_per_step(m) -> int:
    """Transform launches in one mf_filter call under the plan."""
    u = m["plan"]["units_per_batch"]
    nb = -(-m["units"] // u)
    return nb + 1 if m["plan"]["flags"] & 1 else 2 * nb


def roofline(m, workload_name: str, khash: str):
    """Roofline record of the transform kernels (the filter's dominant launches)."""
    k = m["kern"]
    if k["launches"] == 0 or k["ms"] <= 0:
        return None
    avg_ms = k["ms"] / k["launches"]
    bytes_per_launch = k["bytes"] / k["launches"]
    ach = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    prec = "fp64" if m["prec"] == "fp64" else "fp32"
    fused = bool(m["plan"]["flags"] & 1)
    shape = f"{m['plan']['n1']}x{m['plan']['n2']}"
    names = [f"k_step_{prec}_{shape}"] if fused else [f"k_pass1_{prec}_{shape}", f"k_pass2_{prec}_{shape}"]
    rec = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "+".join(names),
           "avg_launch_ms": round(avg_ms, 5), "alg_bytes_per_launch": round(bytes_per_launch),
           "launches_timed": k["launches"],
           "share_of_step": round(avg_ms * launches_per_step(m) / m["ms_per_step"], 3)}
    tb = [read_traffic(nm, workload_name, khash) for nm in names]
    if all(t is not None for t in tb):
        # separate launches alternate pass 1 / pass 2: per-launch average
        rec["traffic"] = round(sum(tb) / len(tb))
    return rec


FP32_VALU_PEAK_TFLOPS = 78.6  # 256 CUs x 2.4 GHz x 64 lanes x 2 (FMA); packed FP32 is not used
FP64_VALU_PEAK_TFLOPS = 78.6


def chisq_roofline(c, wl, khash: str):
    """Roofline record of the band-mode pass 2 (the chi^2 path's dominant kernel): p row
    transforms of N2 points for each of the N1 rows, counted as 5 N2 log2 N2 flops each."""
    k = c["pass2"]
    if k["launches"] == 0 or k["ms"] <= 0:
        return None
    n1, n2 = c["plan"]["n1"], c["plan"]["n2"]
    flops_unit = c["p_bands"] * n1 * 5.0 * n2 * math.log2(n2)
    avg_ms = k["ms"] / k["launches"]
    units_per_launch = k["units"] / k["launches"]
    ach = flops_unit * units_per_launch / (avg_ms * 1e-3) / 1e12
    peak = FP64_VALU_PEAK_TFLOPS if c["prec"] == "fp64" else FP32_VALU_PEAK_TFLOPS
    prec = "fp64" if c["prec"] == "fp64" else "fp32"
    name = f"k_pass2_band_{prec}_{n1}x{n2}"
    tb = read_traffic(name, wl.name, khash)
    return {"bound": "alu", "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
            "traffic": round(tb) if tb is not None else None, "kernel": name, "avg_launch_ms": round(avg_ms, 4),
            "units_per_launch": round(units_per_launch, 2), "flops_per_unit": flops_unit,
            "launches_timed": k["launches"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=5)
    ap.add_argument("--precision", default="fp32_ph64", choices=["fp32_ph64", "fp32", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--single-steps", type=int, default=30,
                    help="steps of the single-segment (1024-template) leg when the main workload is another")
    ap.add_argument("--timing-stride", type=int, default=1)  # 1: every transform launch is timed
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-procs", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--refine-steps", type=int, default=20)
    ap.add_argument("--chisq-steps", type=int, default=5)
    ap.add_argument("--chisq-bands", type=int, default=16)
    ap.add_argument("--events-steps", type=int, default=3)
    ap.add_argument("--events-threshold", type=float, default=4.0)
    ap.add_argument("--events-log2w", type=int, default=11)
    ap.add_argument("--n4m-steps", type=int, default=3)
    ap.add_argument("--graph-replays", type=int, default=10)
    ap.add_argument("--tune", action="store_true", help="autotune the launch plan on the workload first")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}); "
              "the per-GPU share of a sharded bank is the single-GPU workload.", file=sys.stderr)
        sys.exit(2)
    wl = synth.WORKLOADS[args.workload]
    if args.workload == 4:
        run_refine(args)
        return

    cpu = None
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        print(f"[bench] cpu baseline: oracle on host cores (~{args.cpu_seconds:.0f} s)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload, args.cpu_seconds, args.cpu_procs)
        print(f"[bench] cpu baseline {cpu['value']:.2f} {UNIT} on {cpu['cores']} cores", file=sys.stderr, flush=True)

    print(f"[bench] gpu workload {wl.name} precision {args.precision}", file=sys.stderr, flush=True)
    m, fp64, chisq, events, n4m, graph, single, seg_wl = run_gpu(args)
    khash = kernel_hash()
    value = m["units"] / (m["ms_per_step"] * 1e-3)
    eff_gbs = m["b_alg_unit"] * m["units"] / (m["ms_per_step"] * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(m["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision != "fp64" else "f64", "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "fs": wl.fs, "f_low": wl.f_low,
                   "n_tmpl": m["units"] // wl.n_seg, "n_seg": wl.n_seg, "precision": args.precision,
                   "phase_dtype": "f64" if args.precision != "fp32" else "f32", "sigma_dtype": "f64",
                   "mean_active_bins": round(m["mean_active_bins"]), "plan": m["plan"]},
        "effective_hbm": {"achieved": round(eff_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(eff_gbs / HBM_PEAK_GBS, 4),
                          "b_alg_per_unit": round(m["b_alg_unit"])},
        "roofline": roofline(m, wl.name, khash),
        "cpu_baseline": cpu,
        "kernel_source_hash": khash,
        "autotuned": m.get("tuned"),
    }
    if fp64 is not None:
        v64 = fp64["units"] / (fp64["ms_per_step"] * 1e-3)
        e64 = fp64["b_alg_unit"] * fp64["units"] / (fp64["ms_per_step"] * 1e-3) / 1e9
        line["fp64_path"] = {"value": round(v64, 1), "ms_per_step": round(fp64["ms_per_step"], 4),
                             "steps": fp64["steps"], "effective_hbm_frac": round(e64 / HBM_PEAK_GBS, 4),
                             "roofline": roofline(fp64, wl.name, khash),
                             "speedup_fp32_over_fp64": round(value / v64, 3)}
    if single is not None:
        vs = single["units"] / (single["ms_per_step"] * 1e-3)
        es = single["b_alg_unit"] * single["units"] / (single["ms_per_step"] * 1e-3) / 1e9
        line["single_segment_path"] = {
            "workload": seg_wl.name, "value": round(vs, 1), "unit": UNIT,
            "ms_per_step": round(single["ms_per_step"], 4), "steps": single["steps"],
            "effective_hbm_frac": round(es / HBM_PEAK_GBS, 4), "roofline": roofline(single, seg_wl.name, khash)}
    if chisq is not None:
        vc = chisq["units"] / (chisq["ms_per_step"] * 1e-3)
        vs_ref = vs if single is not None else value
        line["chisq_path"] = {
            "workload": seg_wl.name, "value": round(vc, 1), "unit": UNIT, "p_bands": chisq["p_bands"],
            "ms_per_step": round(chisq["ms_per_step"], 4), "steps": chisq["steps"],
            "us_per_unit": round(chisq["ms_per_step"] * 1e3 / chisq["units"], 3),
            "slowdown_vs_filter": round(vs_ref / vc, 3),
            "chisq_at_peaks_median": round(chisq["chisq_at_peaks_median"], 3),
            "plan": chisq["plan"],
            "roofline": chisq_roofline(chisq, seg_wl, khash)}
    if events is not None:
        e32, e64 = events
        a, b = e32["events"], e64["events"]
        both = [k for k in a if k in b and a[k][:2] == b[k][:2]]
        drho = np.array([abs(a[k][2] / b[k][2] - 1.0) for k in both]) if both else np.zeros(0)
        dchi = np.array([abs(a[k][3] / b[k][3] - 1.0) for k in both if b[k][3] != 0.0]) if both else np.zeros(0)
        line["events_path"] = {
            "workload": seg_wl.name, "value": round(e32["units"] / (e32["ms_per_step"] * 1e-3), 1), "unit": UNIT,
            "ms_per_step": round(e32["ms_per_step"], 4), "steps": e32["steps"],
            "threshold": args.events_threshold, "window_samples": 1 << args.events_log2w,
            "events": len(a), "chisq_p_bands": args.chisq_bands,
            "accuracy_vs_fp64": {"matched": len(both), "fp32_only": len(a) - len(both), "fp64_only": len(b) - len(both),
                                 "rho_within_0.03pct": round(float(np.mean(drho < 3e-4)), 5) if both else None,
                                 "chisq_within_0.5pct": round(float(np.mean(dchi < 5e-3)), 5) if both else None,
                                 "rho_max_rel_err": float(drho.max()) if both else None,
                                 "chisq_max_rel_err": float(dchi.max()) if dchi.size else None}}
    if graph is not None:
        line["graph_path"] = {"value": round(graph["units"] / (graph["graph_ms_median"] * 1e-3), 1), "unit": UNIT,
                              "ms_per_replay_median": round(graph["graph_ms_median"], 4),
                              "eager_ms_per_step_median": round(graph["eager_ms_median"], 4),
                              "graph_over_eager": round(graph["eager_ms_median"] / graph["graph_ms_median"], 4),
                              "replays": graph["replays"], "peaks_equal_eager": graph["peaks_equal_eager"],
                              "replay_ms": graph["graph_ms"], "eager_ms": graph["eager_ms"]}
    if n4m is not None:
        v4 = n4m["units"] / (n4m["ms_per_step"] * 1e-3)
        v_ref = vs if single is not None else value
        line["n4m_path"] = {"workload": "single-seg bank on one 4x2^20 segment", "value": round(v4, 1), "unit": UNIT,
                            "n": n4m["n"], "ms_per_step": round(n4m["ms_per_step"], 4),
                            "steps": n4m["steps"], "samples_per_s": round(v4 * n4m["n"], 1),
                            "samples_per_s_vs_2e20": round(v4 * n4m["n"] / (v_ref * seg_wl.n), 4),
                            "plan": n4m["plan"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
