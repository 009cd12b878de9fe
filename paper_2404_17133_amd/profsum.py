"""Summarise rocprofv3 CSV output into short text tables for profiles/.

  python paper_2404_17133_amd/profsum.py stats  <kernel_stats.csv> <out.md> --cmd "<command>"
  python paper_2404_17133_amd/profsum.py pmc    <fetch_counter_collection.csv> <write_counter_collection.csv>
                                                <out.md> --cmd "<command>" --copy-mib 1024

The pmc summary calibrates FETCH_SIZE and WRITE_SIZE (KiB per dispatch) with
the plain copy kernel of known size that bench.py --copy-probe runs (a float32
x * 1.0 over copy-mib MiB), and records the hash of the GEMM source, so that a
later reader can tell whether the kernel changed since the counters were taken.
"""

from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
GEMM_SRC = os.path.join(HERE, "csrc", "gemm.hip")

FAMILIES = {"1": "coul_fwd", "2": "exch_s", "3": "exch_w", "4": "exch_q", "5": "exch_wp", "0": "generic"}


def gemm_source_hash() -> str:
    with open(GEMM_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def short_name(name: str) -> str:
    m = re.search(r"gemm_nt_kernel<([^,]+), (\d+), (\d+), \d+, \d+, (\w+), (\d+)>", name)
    if m:
        t = m.group(1).replace("rid::", "")
        return "gemm_nt<%s,%sx%s,%s> [%s]" % (t, m.group(2), m.group(3), "vec" if m.group(4) == "true" else "scalar",
                                             FAMILIES.get(m.group(5), m.group(5)))
    m = re.search(r"rid::\(anonymous namespace\)::(\w+)", name)
    if m:
        return m.group(1)
    return name[:60]


def stats(path, out, cmd):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["# rocprofv3 kernel statistics", "", "Command: `%s`" % cmd, "",
             "GEMM source hash: %s" % gemm_source_hash(), "",
             "| kernel | calls | avg ms | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:20]:
        lines.append("| %s | %s | %.4f | %.1f | %.1f |" % (short_name(r["Name"]), r["Calls"],
                                                         float(r["AverageNs"]) / 1e6,
                                                         float(r["TotalDurationNs"]) / 1e6,
                                                         100.0 * float(r["TotalDurationNs"]) / total))
    lines.append("")
    lines.append("All kernels: %.1f ms in %d kernel symbols." % (total / 1e6, len(rows)))
    open(out, "w").write("\n".join(lines) + "\n")


def _load(path, cname):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == cname:
            d[r["Kernel_Name"]].append((float(r["Counter_Value"]), int(r["Grid_Size"])))
    return d


def pmc(fetch_path, write_path, out, cmd, copy_mib):
    f = _load(fetch_path, "FETCH_SIZE")
    w = _load(write_path, "WRITE_SIZE")
    probe = None
    want_grid = copy_mib * (1 << 20) // 16  # 4 floats per thread
    for name, vals in f.items():
        if "MulFunctor<float>" in name:
            for v, g in vals:
                if g == want_grid:
                    probe = (name, v)
    if probe is None:
        raise SystemExit("copy probe dispatch not found")
    wprobe = [v for v, g in w[probe[0]] if g == want_grid][0]
    kib = copy_mib * 1024.0
    ff, wf = kib / probe[1], kib / wprobe
    lines = ["# rocprofv3 HBM traffic counters", "", "Commands: `%s` (one run per counter)" % cmd, "",
             "GEMM source hash: %s" % gemm_source_hash(), "",
             "Calibration: a plain copy of %d MiB read %.0f KiB by FETCH_SIZE and wrote %.0f KiB by WRITE_SIZE; "
             "scale factors %.4f (fetch) and %.4f (write) turn counter KiB into bytes moved."
             % (copy_mib, probe[1], wprobe, ff, wf), "",
             "| kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | calibrated GB/dispatch |",
             "|---|---:|---:|---:|---:|"]
    for name, vals in sorted(f.items(), key=lambda kv: -sum(v for v, _ in kv[1])):
        if "gemm_nt_kernel" not in name:
            continue
        fv = sum(v for v, _ in vals) / len(vals)
        wl = w.get(name, [])
        wv = sum(v for v, _ in wl) / max(1, len(wl))
        gb = (fv * ff + wv * wf) * 1024.0 / 1e9
        lines.append("| %s | %d | %.0f | %.0f | %.3f |" % (short_name(name), len(vals), fv, wv, gb))
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "pmc"])
    ap.add_argument("paths", nargs="+")
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--copy-mib", type=int, default=1024)
    a = ap.parse_args()
    if a.mode == "stats":
        stats(a.paths[0], a.paths[1], a.cmd)
    else:
        pmc(a.paths[0], a.paths[1], a.paths[2], a.cmd, a.copy_mib)
