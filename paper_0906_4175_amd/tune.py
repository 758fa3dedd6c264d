"""Launch-plan autotuner for mf_filter.

The library builds a fixed list of transform shapes (N1 x N2 split, columns
per pass-1 work-group, rows per pass-2 work-group) and, per shape, launch
structures (the flags of mf_filter_plan): pass 1 of one batch together with
pass 2 of the previous one in a single launch, a persistent pass 1 with a
longest-first queue, the first row factor applied in pass 1.  `tune`
times every built shape, each launch structure and a set of batch sizes on
the caller's real workload with HIP events on the current stream, installs the
fastest with mf_set_plan and can record it in a JSON cache keyed by
(GPU architecture, N, precision class).  `load_cache` re-installs cached plans
(environment variable MF_TUNE_CACHE: loaded on the first filter call); a
corrupt or foreign cache is ignored with a warning and the built-in defaults
stay in force.
"""
from __future__ import annotations

import ctypes as C
import json
import os
import tempfile
import warnings

from . import _lib as L

PLAN_KEYS = ("n1", "n2", "cols_per_wg", "rows_per_wg", "threads_pass1", "threads_pass2", "units_per_batch", "flags")


def _prec_class(prec: int) -> str:
    return "fp64" if prec == L.MF_FP64 else "fp32"


def _canonical_grid(n: int) -> L.MfGrid:
    # only N matters for a plan; any valid grid of that length selects it
    return L.MfGrid(int(n), 4096.0, 40.0, 150.0)


def candidates(n: int, prec: int) -> list[dict]:
    lib = L.load()
    g = _canonical_grid(n)
    count = lib.mf_plan_candidates(C.byref(g), prec, None, 0)
    if count < 0:
        raise L.MfError(-1, lib.mf_last_error().decode())
    buf = (C.c_int32 * (8 * max(count, 1)))()
    lib.mf_plan_candidates(C.byref(g), prec, buf, count)
    return [dict(zip(PLAN_KEYS, [int(x) for x in buf[8 * i: 8 * i + 8]])) for i in range(count)]


def set_plan(n: int, prec: int, plan: dict | None) -> None:
    lib = L.load()
    g = _canonical_grid(n)
    if plan is None:
        L.check(lib.mf_set_plan(C.byref(g), prec, None))
        return
    arr = (C.c_int32 * 8)(*[int(plan[k]) for k in PLAN_KEYS])
    L.check(lib.mf_set_plan(C.byref(g), prec, arr))


def set_band_plan(n: int, prec: int, plan: dict | None) -> None:
    """Install a plan for the chi^2 band mode (mf_set_band_plan); None restores the default."""
    lib = L.load()
    g = _canonical_grid(n)
    if plan is None:
        L.check(lib.mf_set_band_plan(C.byref(g), prec, None))
        return
    arr = (C.c_int32 * 8)(*[int(plan[k]) for k in PLAN_KEYS])
    L.check(lib.mf_set_band_plan(C.byref(g), prec, arr))


def current_band_plan(n: int, prec: int) -> dict:
    lib = L.load()
    g = _canonical_grid(n)
    arr = (C.c_int32 * 8)()
    L.check(lib.mf_filter_chisq_plan(C.byref(g), prec, arr))
    return dict(zip(PLAN_KEYS, [int(x) for x in arr]))


def current_plan(n: int, prec: int) -> dict:
    lib = L.load()
    g = _canonical_grid(n)
    arr = (C.c_int32 * 8)()
    L.check(lib.mf_filter_plan(C.byref(g), prec, arr))
    return dict(zip(PLAN_KEYS, [int(x) for x in arr]))


def gpu_arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def tune(grid, bank, stilde, Sn, precision="fp32_ph64", units=(128, 256, 512, 1024), steps: int = 3,
         warmup: int = 1, install: bool = True, cache: str | None = None, verbose: bool = False) -> dict:
    """Time every candidate plan on this workload; return {"best": plan, "table": rows}."""
    import torch

    from . import PRECISIONS, filter as mf_filter, filter_workspace_bytes

    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    n = grid.n
    n_seg = int(stilde.shape[0]) if stilde.dim() == 2 else 1
    n_units = bank.n_tmpl * n_seg
    before = current_plan(n, prec)
    rows = []
    try:
        for cand in candidates(n, prec):
            for u in units:
                if u > max(n_units, 1) and u != min(units):
                    continue
                plan = dict(cand, units_per_batch=int(u))
                set_plan(n, prec, plan)
                ws = torch.empty(filter_workspace_bytes(grid, prec, bank.n_tmpl, n_seg), dtype=torch.uint8,
                                 device=stilde.device)
                for _ in range(warmup):
                    mf_filter(grid, bank, stilde, Sn, prec, workspace=ws)
                start = torch.cuda.Event(enable_timing=True)
                stop = torch.cuda.Event(enable_timing=True)
                start.record()
                for _ in range(steps):
                    mf_filter(grid, bank, stilde, Sn, prec, workspace=ws)
                stop.record()
                stop.synchronize()
                ms = start.elapsed_time(stop) / steps
                rows.append(dict(plan, ms=ms))
                if verbose:
                    print(f"  tune {plan} -> {ms:.3f} ms", flush=True)
                del ws
    finally:
        set_plan(n, prec, None)
        if before != current_plan(n, prec):
            set_plan(n, prec, before)
    best = min(rows, key=lambda r: r["ms"])
    best_plan = {k: best[k] for k in PLAN_KEYS}
    if install:
        set_plan(n, prec, best_plan)
    if cache:
        save_cache(cache, gpu_arch(), n, prec, best_plan, best["ms"])
    return {"best": best_plan, "best_ms": best["ms"], "table": rows}


def _key(n: int, prec: int) -> str:
    return f"n={int(n)},prec={_prec_class(prec)}"


def save_cache(path: str, arch: str, n: int, prec: int, plan: dict, ms: float | None = None) -> None:
    data = {}
    if os.path.exists(path):
        try:
            with open(path) as fh:
                data = json.load(fh)
            if not isinstance(data, dict):
                data = {}
        except (OSError, ValueError):
            data = {}
    data.setdefault(arch, {})[_key(n, prec)] = dict(plan, ms=ms)
    d = os.path.dirname(os.path.abspath(path))
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".mf_tune_")
    with os.fdopen(fd, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load_cache(path: str, arch: str | None = None) -> int:
    """Install every cached plan for this GPU architecture; returns how many."""
    try:
        with open(path) as fh:
            data = json.load(fh)
        if not isinstance(data, dict):
            raise ValueError("top level is not an object")
    except (OSError, ValueError) as e:
        warnings.warn(f"mf tune cache {path!r} ignored ({e}); using built-in plans")
        return 0
    if arch is None:
        arch = gpu_arch()
    entries = data.get(arch, {})
    applied = 0
    for key, plan in entries.items():
        try:
            parts = dict(p.split("=") for p in key.split(","))
            n = int(parts["n"])
            prec = L.MF_FP64 if parts["prec"] == "fp64" else L.MF_FP32_PH64
            set_plan(n, prec, {k: int(plan[k]) for k in PLAN_KEYS})
            applied += 1
        except (KeyError, ValueError, TypeError, L.MfError) as e:
            warnings.warn(f"mf tune cache entry {key!r} ignored ({e})")
    return applied
