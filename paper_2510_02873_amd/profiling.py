"""Summaries of rocprofv3 runs of the benchmark (text, for profiles/).

    python -m paper_2510_02873_amd.profiling summarize --kernel k_classic_f64 \
        --trace DIR --fetch DIR --write DIR --calib-mib 1024 --out profiles/X.txt \
        --command "..."

DIRs are rocprofv3 output directories written with --output-format csv
(kernel trace with --stats; one --pmc FETCH_SIZE run; one --pmc WRITE_SIZE
run).  HBM bytes per dispatch are the counters (KiB) scaled by what the same
counter reads for the benchmark's calibration copy of known size.  The
summary records a digest of the kernel sources; the benchmark reports the
traffic only while the sources still match it.
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def source_digest() -> str:
    """sha256 over the HIP sources and headers of the library."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _csv(directory, suffix):
    hits = glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    return list(csv.DictReader(open(hits[0])))


def _counter(rows, counter, kernel):
    vals = [(float(r["Counter_Value"]), r) for r in rows if r["Counter_Name"] == counter and re.search(kernel, r["Kernel_Name"])]
    return vals


def summarize(kernel, trace, fetch, write, calib_mib, out, command):
    stats = _csv(trace, "kernel_stats.csv")
    ks = [r for r in stats if re.search(kernel, r["Name"])]
    lines = [f"# rocprofv3 summary: {kernel}", f"command: {command}", f"source_digest: {source_digest()}", ""]
    lines.append("kernel stats (--kernel-trace --stats):")
    for r in ks:
        lines.append(f"  {r['Name']}: calls={r['Calls']} total_ns={r['TotalDurationNs']} "
                     f"average_ns={float(r['AverageNs']):.1f} min_ns={r['MinNs']} max_ns={r['MaxNs']}")
    calib_kib = calib_mib * 1024.0
    res = {}
    for label, d, counter in (("fetch", fetch, "FETCH_SIZE"), ("write", write, "WRITE_SIZE")):
        rows = _csv(d, "counter_collection.csv")
        kvals = _counter(rows, counter, kernel)
        # the calibration copy is the dispatch whose counter is nearest the copy size
        allv = [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == counter]
        copies = [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == counter
                  and re.search("copy", r["Kernel_Name"], re.I)]
        ref = max(copies) if copies else max(allv)
        factor = calib_kib / ref
        per = np.array([v for v, _ in kvals]) * factor * 1024.0
        res[label] = (factor, per)
        lines.append(f"{counter}: {len(per)} dispatches of {kernel}; calibration copy of {calib_mib} MiB "
                     f"read {ref:.0f} KiB -> scale {factor:.4f}; bytes per dispatch mean {per.mean():.4e} "
                     f"min {per.min():.4e} max {per.max():.4e}")
    fetch_mean = float(res["fetch"][1].mean())
    write_mean = float(res["write"][1].mean())
    lines.append("")
    lines.append(f"traffic_bytes_per_launch: {fetch_mean + write_mean:.6e}")
    lines.append(f"fetch_bytes_per_launch: {fetch_mean:.6e}")
    lines.append(f"write_bytes_per_launch: {write_mean:.6e}")
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_traffic(path):
    """(traffic bytes per launch, digest) from a summary, or (None, None)."""
    if not os.path.exists(path):
        return None, None
    traffic = digest = None
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch:"):
            traffic = float(line.split(":", 1)[1])
        elif line.startswith("source_digest:"):
            digest = line.split(":", 1)[1].strip()
    return traffic, digest


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("summarize")
    s.add_argument("--kernel", required=True)
    s.add_argument("--trace", required=True)
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--calib-mib", type=int, default=1024)
    s.add_argument("--out", required=True)
    s.add_argument("--command", default="")
    a = ap.parse_args()
    summarize(a.kernel, a.trace, a.fetch, a.write, a.calib_mib, a.out, a.command)


if __name__ == "__main__":
    main()
