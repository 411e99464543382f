"""Summaries of rocprofv3 output (kernel-trace statistics and the FETCH_SIZE /
WRITE_SIZE counters) for the committed profile notes.

    python -m paper_2410_20429_amd.profiling stats <kernel_stats.csv> <command...>
    python -m paper_2410_20429_amd.profiling traffic <fetch.csv> <write.csv> <kernel> <calls/step>

HBM counters are calibrated with a plain device copy of known size run in the
same process (1 GiB read + 1 GiB written): each counter is scaled by
known bytes / counted bytes of that copy.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30


def short_name(name):
    n = name.split("(")[0]
    for pre in ("void ", "mars::"):
        n = n.replace(pre, "")
    return n


def kernel_stats_md(path, command):
    rows = list(csv.DictReader(open(path)))
    lines = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| {short_name(r['Name'])} | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |")
    return f"Command: `{command}`\n\n" + "\n".join(lines) + "\n"


def _per_kernel(path):
    out = {}
    for r in csv.DictReader(open(path)):
        out.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "device_math.hpp", "mars_internal.h"):
        with open(os.path.join(ROOT, "paper_2410_20429_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic(fetch_csv, write_csv, kernel):
    f, w = _per_kernel(fetch_csv), _per_kernel(write_csv)
    # the calibration copy is the largest copy dispatch
    cf = max(f.get("__amd_rocclr_copyBuffer", [0]))
    cw = max(w.get("__amd_rocclr_copyBuffer", [0]))
    fs = COPY_BYTES / (cf * 1024.0) if cf > 0 else None
    ws = COPY_BYTES / (cw * 1024.0) if cw > 0 else None
    kf, kw = f.get(kernel, []), w.get(kernel, [])
    if not kf or not kw or fs is None or ws is None:
        return None
    fetch = sum(kf) / len(kf) * 1024.0 * fs
    write = sum(kw) / len(kw) * 1024.0 * ws
    return {"kernel": kernel, "launches": len(kf), "fetch_scale": fs, "write_scale": ws,
            "hbm_fetch_bytes_per_launch": fetch, "hbm_write_bytes_per_launch": write,
            "hbm_bytes_per_launch": fetch + write, "kernel_source_hash": kernel_source_hash()}


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(kernel_stats_md(sys.argv[2], " ".join(sys.argv[3:])))
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], sys.argv[4]), indent=1))
