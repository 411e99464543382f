"""Summaries of rocprofv3 output (kernel-trace statistics and the FETCH_SIZE /
WRITE_SIZE counters) for the committed profile notes.

    python -m paper_2410_20429_amd.profiling stats <kernel_stats.csv> <command...>
    python -m paper_2410_20429_amd.profiling window <kernel_trace.csv> <kernel> <last_n>
    python -m paper_2410_20429_amd.profiling traffic <fetch.csv> <write.csv> <kernel> <last_n> \
        <workload> <warmup> <steps> [<occupancy.csv>]

`last_n` selects the last n dispatches of the kernel: a profiling run of
bench.py (--profile-steps) stops after its timed steps, which it reports as
trace_launches_timed, so these are exactly the timed region's launches.

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


def _order(r):
    for k in ("Dispatch_Id", "Correlation_Id", "Index"):
        if k in r and r[k] not in (None, ""):
            return int(r[k])
    return 0


def _per_kernel(path, counter=None):
    """{kernel: [value per dispatch in dispatch order]} of one counter"""
    rows = [r for r in csv.DictReader(open(path))
            if counter is None or r.get("Counter_Name", counter) == counter]
    rows.sort(key=_order)
    out = {}
    for r in rows:
        out.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def window_stats(trace_csv, kernel, last_n):
    """average and total duration of the last `last_n` dispatches of a kernel"""
    rows = [r for r in csv.DictReader(open(trace_csv)) if short_name(r["Kernel_Name"]) == kernel]
    rows.sort(key=_order)
    d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in rows[-last_n:]]
    return {"kernel": kernel, "launches": len(d), "avg_us": sum(d) / len(d) / 1e3,
            "total_ms": sum(d) / 1e6, "all_launches": len(rows)}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "device_math.hpp", "mars_internal.h"):
        with open(os.path.join(ROOT, "paper_2410_20429_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic(fetch_csv, write_csv, kernel, last_n=None, window=None, occupancy_csv=None):
    """Measured HBM bytes per launch of `kernel` over its last `last_n`
    dispatches, each counter scaled by known / counted bytes of the plain
    1 GiB copy in the same process.  With an occupancy counter file
    (SQ_WAVE_CYCLES and SQ_BUSY_CYCLES, or the derived MeanOccupancyPerCU),
    the mean waves resident per SIMD over the same dispatches."""
    f, w = _per_kernel(fetch_csv), _per_kernel(write_csv)
    # the calibration copy is the largest copy dispatch
    cf = max(f.get("__amd_rocclr_copyBuffer", [0]))
    cw = max(w.get("__amd_rocclr_copyBuffer", [0]))
    fs = COPY_BYTES / (cf * 1024.0) if cf > 0 else None
    ws = COPY_BYTES / (cw * 1024.0) if cw > 0 else None
    kf, kw = f.get(kernel, []), w.get(kernel, [])
    if last_n:
        kf, kw = kf[-last_n:], kw[-last_n:]
    if not kf or not kw or fs is None or ws is None:
        return None
    fetch = sum(kf) / len(kf) * 1024.0 * fs
    write = sum(kw) / len(kw) * 1024.0 * ws
    out = {"kernel": kernel, "launches": len(kf), "fetch_scale": fs, "write_scale": ws,
           "hbm_fetch_bytes_per_launch": fetch, "hbm_write_bytes_per_launch": write,
           "hbm_bytes_per_launch": fetch + write, "kernel_source_hash": kernel_source_hash()}
    if window:
        out["window"] = window
    if occupancy_csv:
        occ = _occupancy(occupancy_csv, kernel, last_n)
        if occ is not None:
            out["occupancy_waves_per_simd"] = occ
        occ_t = _occupancy_time_weighted(occupancy_csv, kernel, last_n)
        if occ_t is not None:
            out["occupancy_waves_per_simd_time_weighted"] = occ_t
    return out


def _occupancy_time_weighted(path, kernel, last_n):
    """MeanOccupancyPerCU / 4 over the last `last_n` dispatches, each weighted
    by its duration in the counter run (the plain mean weighs the short
    launches of the deep bounces as much as the long ones)"""
    rows = [r for r in csv.DictReader(open(path))
            if r.get("Counter_Name") == "MeanOccupancyPerCU" and short_name(r["Kernel_Name"]) == kernel]
    rows.sort(key=_order)
    rows = rows[-last_n:] if last_n else rows
    w = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows]
    if not rows or sum(w) <= 0:
        return None
    return sum(float(r["Counter_Value"]) * d for r, d in zip(rows, w)) / sum(w) / 4.0


def _occupancy(path, kernel, last_n, simds=4 * 256):
    """mean resident waves per SIMD: SQ_WAVE_CYCLES (wave-cycles summed over
    the chip) / SQ_BUSY_CYCLES / SIMDs, or MeanOccupancyPerCU / 4"""
    wc = _per_kernel(path, "SQ_WAVE_CYCLES").get(kernel, [])
    bc = _per_kernel(path, "SQ_BUSY_CYCLES").get(kernel, [])
    if wc and bc:
        wc, bc = wc[-last_n:], bc[-last_n:]
        return sum(wc) / max(sum(bc), 1.0) / simds
    mo = _per_kernel(path, "MeanOccupancyPerCU").get(kernel, [])
    if mo:
        mo = mo[-last_n:]
        return sum(mo) / len(mo) / 4.0
    return None


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(kernel_stats_md(sys.argv[2], " ".join(sys.argv[3:])))
    elif sys.argv[1] == "window":
        print(json.dumps(window_stats(sys.argv[2], sys.argv[3], int(sys.argv[4])), indent=1))
    elif sys.argv[1] == "traffic":
        win = {"workload": sys.argv[6], "warmup": int(sys.argv[7]), "steps": int(sys.argv[8])}
        occ = sys.argv[9] if len(sys.argv) > 9 else None
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), win, occ),
                         indent=1))
