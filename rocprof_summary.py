#!/usr/bin/env python3
"""Short text summaries of rocprofv3 CSV output, for the files under profiles/.

    python rocprof_summary.py stats KERNEL_STATS_CSV --command CMD [--trace TRACE_CSV --detail K1,K2]
    python rocprof_summary.py traffic --fetch FETCH_CSV --write WRITE_CSV \\
        --kernel NAME --source FILE --copy-bytes B --command CMD
    python rocprof_summary.py util COUNTER_CSV --command CMD --kernels K1,K2

`stats` lists every kernel of a `--kernel-trace --stats` run (calls, total and
average duration).  `traffic` turns the FETCH_SIZE and WRITE_SIZE counters
(KiB per dispatch, one `--pmc` run each) of one kernel into HBM bytes per
launch, scaled by what the same counters read for the largest device copy of
the run (`__amd_rocclr_copyBuffer` of --copy-bytes bytes read and written),
and records the SHA-256 of the kernel's source file so that a reader can tell
whether the kernel has changed since the counters were taken.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
import sys


def short_name(name: str) -> str:
    m = re.search(r"(k_[A-Za-z0-9_]+(<\d+>)?|__amd_rocclr_\w+|\w*elementwise_kernel\w*)", name)
    return m.group(1) if m else name[:48]


def stats(path: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["# rocprofv3 kernel statistics", "", "Command (from /tmp, TMPDIR=/tmp):", "",
           "    " + command, "",
           f"Total kernel time {total / 1e6:.3f} ms over the whole run.", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append("| {} | {} | {:.3f} | {:.1f} | {:.1f} | {:.1f} | {:.2f} |".format(
            short_name(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    return "\n".join(out) + "\n"


def detail(trace: str, kernels) -> str:
    """Per-dispatch durations (us, in launch order) of the named kernels from a
    --kernel-trace CSV, with their mean and median."""
    rows = list(csv.DictReader(open(trace)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    out = ["", "Per-dispatch durations (us, launch order) from the kernel trace:", ""]
    for k in kernels:
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows
             if short_name(r["Kernel_Name"]) == k]
        if not d:
            continue
        srt = sorted(d)
        med = srt[len(srt) // 2]
        out.append(f"* {k} ({len(d)}): " + ", ".join(f"{x:.1f}" for x in d)
                   + f"; mean {sum(d) / len(d):.1f}, median {med:.1f}")
    return "\n".join(out) + "\n"


def _counter(path: str, counter: str):
    """Counter values per kernel, keyed by the short name without template arguments."""
    per = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        name = re.sub(r"<.*>$", "", short_name(r["Kernel_Name"]))
        per.setdefault(name, []).append(float(r["Counter_Value"]))
    return per


def traffic(fetch: str, write: str, kernel: str, source: str, copy_bytes: float, command: str,
            first: int = 0) -> str:
    f = _counter(fetch, "FETCH_SIZE")
    w = _counter(write, "WRITE_SIZE")
    if kernel not in f or kernel not in w:
        raise SystemExit(f"kernel {kernel} not found in the counter files")
    copy_f = max(f.get("__amd_rocclr_copyBuffer", [0.0]))
    copy_w = max(w.get("__amd_rocclr_copyBuffer", [0.0]))
    if first > 0:   # the kernel's first dispatches only (those of the timed step)
        f[kernel] = f[kernel][:first]
        w[kernel] = w[kernel][:first]
    if copy_f <= 0 or copy_w <= 0:
        raise SystemExit("no copy kernel in the counter files")
    sf = copy_bytes / (copy_f * 1024.0)
    sw = copy_bytes / (copy_w * 1024.0)
    kf = sum(f[kernel]) / len(f[kernel])
    kw = sum(w[kernel]) / len(w[kernel])
    bytes_per_launch = kf * 1024.0 * sf + kw * 1024.0 * sw
    sha = hashlib.sha256(open(source, "rb").read()).hexdigest()
    out = ["# HBM traffic of " + kernel, "",
           "Commands (from /tmp, TMPDIR=/tmp), one counter per run:", "",
           "    " + command.replace("COUNTER", "FETCH_SIZE"),
           "    " + command.replace("COUNTER", "WRITE_SIZE"), "",
           "| counter | dispatches | mean KiB/dispatch | min | max |", "|---|---:|---:|---:|---:|",
           f"| FETCH_SIZE | {len(f[kernel])} | {kf:.1f} | {min(f[kernel]):.1f} | {max(f[kernel]):.1f} |",
           f"| WRITE_SIZE | {len(w[kernel])} | {kw:.1f} | {min(w[kernel]):.1f} | {max(w[kernel]):.1f} |",
           "",
           f"Calibration: a device copy of {copy_bytes:.0f} bytes (read and written once) reads "
           f"FETCH_SIZE {copy_f:.1f} KiB and WRITE_SIZE {copy_w:.1f} KiB, so the counters are scaled by "
           f"{sf:.4f} (fetch) and {sw:.4f} (write)."
           + (f" Only the kernel's first {first} dispatches of each run are used (the warm-up, timed"
              " and event-timed steps; later dispatches belong to other timings of the run)." if first else ""),
           "",
           f"traffic_bytes_per_launch: {bytes_per_launch:.6e}",
           f"source_sha256: {os.path.relpath(source)} {sha}", ""]
    return "\n".join(out)


def util(path: str, command: str, kernels) -> str:
    """Mean of each derived counter per kernel (percent or flops per dispatch)."""
    per = {}
    for r in csv.DictReader(open(path)):
        name = re.sub(r"<.*>$", "", short_name(r["Kernel_Name"]))
        per.setdefault(name, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({c for d in per.values() for c in d})
    out = ["# Matrix-core and vector-ALU utilisation per kernel", "", "Command (from /tmp, TMPDIR=/tmp):", "",
           "    " + command, "",
           "MfmaUtil: percent of the time the matrix units are busy (sum of busy cycles over all",
           "SIMDs / (GPU active cycles x SIMDs)); VALUBusy: percent of the time vector instructions",
           "are processed; MfmaFlopsF32: FP32 matrix flops per dispatch.  Kernels run one at a time",
           "under counter collection.", "",
           "| kernel | dispatches | " + " | ".join(names) + " |",
           "|---|---:|" + "---:|" * len(names)]
    for k in kernels:
        if k not in per:
            continue
        d = per[k]
        n = max(len(v) for v in d.values())
        cells = []
        for c in names:
            v = d.get(c)
            cells.append("-" if not v else (f"{sum(v) / len(v):.3e}" if "Flops" in c else f"{sum(v) / len(v):.1f}"))
        out.append(f"| {k} | {n} | " + " | ".join(cells) + " |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--command", required=True)
    a.add_argument("--trace", help="kernel trace CSV of the same run, for --detail")
    a.add_argument("--detail", default="", help="comma-separated short kernel names")
    a.add_argument("--note", default="", help="a line of text appended after the table")
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--source", required=True)
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--command", required=True)
    b.add_argument("--first", type=int, default=0, help="use only the kernel's first N dispatches")
    c = sub.add_parser("util")
    c.add_argument("csv")
    c.add_argument("--command", required=True)
    c.add_argument("--kernels", required=True, help="comma-separated short kernel names")
    args = ap.parse_args()
    if args.what == "util":
        sys.stdout.write(util(args.csv, args.command, args.kernels.split(",")))
        return
    if args.what == "stats":
        sys.stdout.write(stats(args.csv, args.command))
        if args.trace and args.detail:
            sys.stdout.write(detail(args.trace, args.detail.split(",")))
        if args.note:
            sys.stdout.write("\n" + args.note + "\n")
    else:
        sys.stdout.write(traffic(args.fetch, args.write, args.kernel, args.source, args.copy_bytes,
                                 args.command, args.first))


if __name__ == "__main__":
    main()
