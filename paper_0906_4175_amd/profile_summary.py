"""Summarise rocprofv3 output into the short text files kept under profiles/.

  python3 paper_0906_4175_amd/profile_summary.py --stats DIR_KTRACE \\
      --fetch DIR_FETCH --write DIR_WRITE --workload NAME --copy-mib 1024 --out OUTDIR

--stats: a `rocprofv3 --kernel-trace --stats --output-format csv` directory;
--fetch / --write: `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of
profile_run.py.  The byte counters are scaled by the factor that makes the
calibration copy kernel read and write exactly --copy-mib MiB.
--sq: a `rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU ...` run; with --elements
(kernel=output elements per dispatch, comma-separated) and the kernel trace of
--stats it writes VALU instructions per element and the VALU issue fraction
(wave64 instructions x 4 cycles / (duration x 2.4 GHz x 1024 SIMDs)).
--flops: a `rocprofv3 --pmc SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_{F32,F64}` run; per
dispatch, flops = 64 x (add + mul + trans + 2 fma) for each precision, listed in
dispatch order, per element with --elements.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# every device source: a profile goes stale when any kernel's code changes
KERNEL_SOURCES = sorted(os.path.join(ROOT, "paper_0906_4175_amd", "csrc", f)
                        for f in os.listdir(os.path.join(ROOT, "paper_0906_4175_amd", "csrc"))
                        if f.endswith((".hip", ".hpp")))


def kernel_hash() -> str:
    """Hash of the device code (every .hip and .hpp source): comments and whitespace
    are left out, so a profile stays valid across edits that change neither."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


# position of (N1, N2) among the template arguments of the transform kernels
_SHAPE_ARGS = {"k_pass1_band": 2, "k_pass2_band": 1, "k_pass1_lpt": 3, "k_pass1": 3, "k_pass2": 2, "k_step": 2}
# the persistent pass 1 is reported under the pass-1 name of its shape (one of
# the two forms runs in a given plan)
_ROLE = {"k_pass1_lpt": "k_pass1"}


def short(name: str) -> str:
    for key, at in _SHAPE_ARGS.items():
        if f"::{key}<" in name:
            args = [x.strip() for x in name.split("<", 1)[1].split(">", 1)[0].split(",")]
            prec = "fp64" if args[0] == "double" else "fp32"
            return f"{_ROLE.get(key, key)}_{prec}_{args[at]}x{args[at + 1]}"
    for key in ("k_pass1_band", "k_pass2_band", "k_lpt_order", "k_pass1", "k_pass2", "k_step", "k_copy_probe", "k_finalize32",
                "k_finalize64", "k_finalize_band", "k_band_table", "k_weights", "k_sigma", "k_psd", "k_spa_synth",
                "k_snr_grad", "k_prefix", "k_chisq", "k_events_unit", "k_events_best", "k_events_merge",
                "k_fill_u64", "k_rfft_pack", "k_rfft_post"):
        if key in name:
            prec = "fp64" if "<double" in name else ("fp32" if "<float" in name else "")
            return f"{key}_{prec}" if prec else key
    return name.split("(")[0][:40]


def find(d, pattern):
    hits = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not hits:
        raise SystemExit(f"no {pattern} under {d}")
    return hits[0]


def counters(d, counter):
    rows = list(csv.DictReader(open(find(d, "*counter_collection.csv"))))
    per = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        per.setdefault(short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return per


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command-stats", default="")
    ap.add_argument("--command-fetch", default="")
    ap.add_argument("--command-write", default="")
    ap.add_argument("--sq")
    ap.add_argument("--command-sq", default="")
    ap.add_argument("--elements", default="")
    ap.add_argument("--flops")
    ap.add_argument("--command-flops", default="")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    khash = kernel_hash()
    if args.stats:
        rows = list(csv.DictReader(open(find(args.stats, "*kernel_stats.csv"))))
        lines = [f"# rocprofv3 kernel trace statistics, workload {args.workload}",
                 f"# command: {args.command_stats}", f"kernel_source_hash: {khash}",
                 f"{'kernel':<22} {'calls':>7} {'avg_us':>10} {'total_ms':>10} {'pct':>6}"]
        for r in rows:
            avg_ns = float(r.get("AverageNs", 0.0))
            tot_ns = float(r.get("TotalDurationNs", 0.0))
            lines.append(f"{short(r['Name']):<22} {int(float(r['Calls'])):>7} {avg_ns / 1e3:>10.2f} "
                         f"{tot_ns / 1e6:>10.3f} {float(r.get('Percentage', 0.0)):>6.2f}")
        with open(os.path.join(args.out, f"ktrace_{args.workload}.txt"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
    if args.fetch and args.write:
        f = counters(args.fetch, "FETCH_SIZE")
        w = counters(args.write, "WRITE_SIZE")
        copy_bytes = args.copy_mib << 20
        f_copy = statistics.mean(f["k_copy_probe"]) * 1024.0
        w_copy = statistics.mean(w["k_copy_probe"]) * 1024.0
        sf, sw = copy_bytes / f_copy, copy_bytes / w_copy
        for k in sorted(set(f) & set(w)):
            if not k.startswith(("k_pass1", "k_pass2", "k_step")):
                continue
            fb = statistics.mean(f[k]) * 1024.0 * sf
            wb = statistics.mean(w[k]) * 1024.0 * sw
            path = os.path.join(args.out, f"traffic_{k}_{args.workload}.txt")
            with open(path, "w") as fh:
                fh.write(f"# HBM traffic per dispatch of {k}, workload {args.workload}\n")
                fh.write(f"# fetch command: {args.command_fetch}\n# write command: {args.command_write}\n")
                fh.write(f"kernel_source_hash: {khash}\n")
                fh.write(f"dispatches: {len(f[k])}\n")
                fh.write(f"fetch_kib_raw: {statistics.mean(f[k]):.1f}\nwrite_kib_raw: {statistics.mean(w[k]):.1f}\n")
                fh.write(f"copy_calibration: {args.copy_mib} MiB copy read FETCH_SIZE {f_copy / 1024:.1f} KiB, "
                         f"WRITE_SIZE {w_copy / 1024:.1f} KiB -> scale fetch x{sf:.4f}, write x{sw:.4f}\n")
                fh.write(f"fetch_bytes_per_launch: {fb:.0f}\nwrite_bytes_per_launch: {wb:.0f}\n")
                fh.write(f"hbm_bytes_per_launch: {fb + wb:.0f}\n")
    if args.sq:
        rows = list(csv.DictReader(open(find(args.sq, "*counter_collection.csv"))))
        per = {}
        for r in rows:
            per.setdefault(short(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
        dur = {}
        if args.stats:
            for r in csv.DictReader(open(find(args.stats, "*kernel_stats.csv"))):
                dur[short(r["Name"])] = float(r.get("AverageNs", 0.0))
        elements = dict(kv.split("=") for kv in args.elements.split(",") if kv)
        for k, cnt in sorted(per.items()):
            if k not in elements:
                continue
            path = os.path.join(args.out, f"valu_{k}_{args.workload}.txt")
            with open(path, "w") as fh:
                fh.write(f"# SQ counters per dispatch of {k}, workload {args.workload}\n")
                fh.write(f"# command: {args.command_sq}\nkernel_source_hash: {khash}\n")
                fh.write(f"dispatches: {len(next(iter(cnt.values())))}\n")
                for name, vals in sorted(cnt.items()):
                    fh.write(f"{name}: {statistics.mean(vals):.1f}\n")
                el = float(elements[k])
                valu = statistics.mean(cnt.get("SQ_INSTS_VALU", [0.0]))
                fh.write(f"output_elements_per_dispatch: {el:.0f}\n")
                fh.write(f"valu_instructions_per_element: {valu * 64.0 / el:.2f}\n")
                if k in dur and dur[k] > 0:
                    frac = valu * 4.0 / (dur[k] * 1e-9 * 2.4e9 * 1024.0)
                    fh.write(f"avg_duration_us: {dur[k] / 1e3:.2f}\nvalu_issue_fraction: {frac:.3f}\n")
    if args.flops:
        rows = list(csv.DictReader(open(find(args.flops, "*counter_collection.csv"))))
        per = {}
        for r in rows:
            key = (short(r["Kernel_Name"]), int(r.get("Dispatch_Id", 0)))
            per.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
        elements = dict(kv.split("=") for kv in args.elements.split(",") if kv)
        by_kernel = {}
        for (k, d), c in sorted(per.items(), key=lambda x: x[0][1]):
            def fl(p):
                return 64.0 * (c.get(f"SQ_INSTS_VALU_ADD_{p}", 0.0) + c.get(f"SQ_INSTS_VALU_MUL_{p}", 0.0) +
                               c.get(f"SQ_INSTS_VALU_TRANS_{p}", 0.0) + 2.0 * c.get(f"SQ_INSTS_VALU_FMA_{p}", 0.0))
            by_kernel.setdefault(k, []).append((fl("F32"), fl("F64")))
        for k, lst in sorted(by_kernel.items()):
            if k not in elements:
                continue
            el = float(elements[k])
            path = os.path.join(args.out, f"flops_{k}_{args.workload}.txt")
            with open(path, "w") as fh:
                fh.write(f"# VALU flops per dispatch of {k}, workload {args.workload}\n")
                fh.write(f"# command: {args.command_flops}\nkernel_source_hash: {khash}\n")
                fh.write(f"dispatches: {len(lst)}\nelements_per_dispatch: {el:.0f}\n")
                for name, vals in (("fp32", [a / el for a, _ in lst]), ("fp64", [b / el for _, b in lst]),
                                   ("total", [(a + b) / el for a, b in lst])):
                    fh.write(f"{name}_flops_per_element_mean: {statistics.mean(vals):.2f}\n"
                             f"{name}_flops_per_element_min: {min(vals):.2f}\n"
                             f"{name}_flops_per_element_max: {max(vals):.2f}\n")
                if k in dur_all(args.stats):
                    d_ns = dur_all(args.stats)[k]
                    tot = statistics.mean(a + b for a, b in lst)
                    fh.write(f"avg_duration_us: {d_ns / 1e3:.2f}\nachieved_tflops: {tot / (d_ns * 1e-9) / 1e12:.2f}\n")
    print("written to", args.out)


def dur_all(stats_dir):
    if not stats_dir:
        return {}
    return {short(r["Name"]): float(r.get("AverageNs", 0.0))
            for r in csv.DictReader(open(find(stats_dir, "*kernel_stats.csv")))}


if __name__ == "__main__":
    main()
