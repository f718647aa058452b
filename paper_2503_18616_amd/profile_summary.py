"""Summarise rocprofv3 outputs of the step kernel into profiles/.

    python -m paper_2503_18616_amd.profile_summary \\
        --trace DIR --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \\
        --copy-mib 256 --workload NAME --colouring C --command "..." --out profiles/NAME.md \\
        [--record xpbd_step_traffic.json]

DIR are rocprofv3 ``--output-format csv`` directories: a ``--kernel-trace
--stats`` run of the bench, ``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``
runs of the bench, and the same two counters over ``bench.py
--copy-calibration MIB`` (a plain device copy of known size, which gives the
scale of each counter).  Writes the markdown summary and
a traffic record under profiles/ (HBM bytes per step launch, scaled, with the
SHA-256 of the kernel and runtime sources they were measured on and the
colouring).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
KERNEL_SOURCE = os.path.join(PKG, "csrc", "xpbd_kernels.hip")
RUNTIME_SOURCE = os.path.join(PKG, "csrc", "xpbd_runtime.hip")
STEP_KERNEL = "xpbd_step_"


def source_sha256(path) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _csv(directory, suffix):
    files = glob.glob(os.path.join(directory, f"*{suffix}"))
    if not files:
        raise FileNotFoundError(f"no *{suffix} in {directory}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def counter_mean(directory, counter, match):
    vals = [float(r["Counter_Value"]) for r in _csv(directory, "counter_collection.csv")
            if r["Counter_Name"] == counter and match(r["Kernel_Name"])]
    if not vals:
        raise ValueError(f"{counter} not found for the kernel in {directory}")
    return sum(vals) / len(vals), len(vals)


def main():
    ap = argparse.ArgumentParser()
    for k in ("trace", "fetch", "write", "copy_fetch", "copy_write"):
        ap.add_argument("--" + k.replace("_", "-"), required=True)
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--colouring", type=int, required=True,
                    help="the colouring the profiled runs used (bench.py --colouring)")
    ap.add_argument("--command", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--record", default="xpbd_step_traffic.json",
                    help="file under profiles/ that receives the traffic record")
    ap.add_argument("--extra", nargs="*", default=[],
                    help="further --pmc csv directories; their counters are listed per dispatch")
    args = ap.parse_args()

    stats = _csv(args.trace, "kernel_stats.csv")
    is_step = lambda name: STEP_KERNEL in name
    is_copy = lambda name: "copyBuffer" in name or "elementwise" in name or "copy" in name.lower()
    copy_kib = args.copy_mib * 1024.0
    cf, _ = max((counter_mean(args.copy_fetch, "FETCH_SIZE", lambda n, s=s: n == s)
                 for s in {r["Kernel_Name"] for r in _csv(args.copy_fetch, "counter_collection.csv")}
                 if is_copy(s)), key=lambda t: t[0])
    cw, _ = max((counter_mean(args.copy_write, "WRITE_SIZE", lambda n, s=s: n == s)
                 for s in {r["Kernel_Name"] for r in _csv(args.copy_write, "counter_collection.csv")}
                 if is_copy(s)), key=lambda t: t[0])
    fetch_scale, write_scale = copy_kib / cf, copy_kib / cw
    fk, nf = counter_mean(args.fetch, "FETCH_SIZE", is_step)
    wk, nw = counter_mean(args.write, "WRITE_SIZE", is_step)
    traffic = (fk * fetch_scale + wk * write_scale) * 1024.0

    lines = [f"# Step kernel — {args.workload}", "", "Command (from the repository root):", "",
             "    " + args.command, "",
             "| kernel | calls | total (ns) | average (ns) | share |", "|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {r['Name'][:90]} | {r['Calls']} | {r['TotalDurationNs']} | "
                     f"{float(r['AverageNs']):.1f} | {float(r['Percentage']):.2f} % |")
    lines += ["", "HBM bytes of the step kernel (rocprofv3 --pmc, mean per dispatch):", "",
              f"- FETCH_SIZE {fk:.1f} KiB x scale {fetch_scale:.3f} (a {args.copy_mib} MiB copy reads "
              f"{cf:.1f} KiB) = {fk * fetch_scale / 1024:.2f} MiB ({nf} dispatches)",
              f"- WRITE_SIZE {wk:.1f} KiB x scale {write_scale:.3f} (the copy writes {cw:.1f} KiB) = "
              f"{wk * write_scale / 1024:.2f} MiB ({nw} dispatches)",
              f"- traffic per launch: {traffic / 1e6:.2f} MB", ""]
    if args.extra:
        lines += ["Other counters of the step kernel (mean per dispatch; SQ_ cycle counters "
                  "are in units of 4 cycles, summed over waves):", "",
                  "| counter | value |", "|---|---|"]
        for d in args.extra:
            names = sorted({r["Counter_Name"] for r in _csv(d, "counter_collection.csv")})
            for c in names:
                v, _ = counter_mean(d, c, is_step)
                lines.append(f"| {c} | {v:.4g} |")
        lines.append("")
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    rec = {"kernel_source_sha256": source_sha256(KERNEL_SOURCE),
           "runtime_source_sha256": source_sha256(RUNTIME_SOURCE),
           "workload": args.workload, "colouring": args.colouring,
           "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
           "fetch_scale": fetch_scale, "write_scale": write_scale,
           "traffic_bytes_per_launch": traffic, "command": args.command}
    with open(os.path.join(ROOT, "profiles", args.record), "w") as f:
        json.dump(rec, f, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
