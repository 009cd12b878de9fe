"""Summarise rocprofv3 CSV output into short text tables for profiles/.

  python paper_2404_17133_amd/profsum.py stats  <kernel_stats.csv> <out.md> --cmd "<command>"
  python paper_2404_17133_amd/profsum.py pmc    <fetch_counter_collection.csv> <write_counter_collection.csv>
                                                <out.md> --cmd "<command>" --copy-mib 1024
                                                [--stats <kernel_stats.csv>]
  python paper_2404_17133_amd/profsum.py mfma   <counter_collection.csv> <out.md> --cmd "<command>"
  python paper_2404_17133_amd/profsum.py busy   <kernel_trace.csv> <out.md> --cmd "<command>" [--tail-s S]

The pmc summary calibrates FETCH_SIZE and WRITE_SIZE (KiB per dispatch) with
the plain copy kernel of known size that bench.py --copy-probe runs (a float32
x * 1.0 over copy-mib MiB), and records the hash of the GEMM source, so that a
later reader can tell whether the kernel changed since the counters were
taken.  Given the kernel statistics of the same command, it also reports the
achieved rate (calibrated bytes per dispatch over the average duration) of
every kernel, the memory-bound ones included.

The mfma summary reads a run with --pmc MfmaUtil SQ_INSTS_VALU_MFMA_MOPS_F32
SQ_INSTS_VALU_MFMA_MOPS_BF16 SQ_INSTS_VALU_MFMA_MOPS_F64: the share of SIMD
cycles the matrix cores were busy, and the MFMA operations issued, per kernel.
The busy summary reads a kernel trace and reports the fraction of the traced
span during which at least one kernel was running on the device.
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
    # gemm_nt_kernel<type, BM, BN, WM, WN, vector loads, [interleaved chunks,] family>
    m = re.search(r"gemm_nt_kernel<([^,]+), (\d+), (\d+), \d+, \d+, (\w+), (?:(\w+), )?(\d+)>", name)
    if m:
        t = m.group(1).replace("rid::", "")
        form = "vec" if m.group(4) == "true" else "scalar"
        if m.group(5) == "true":
            form += ",il"
        return "gemm_nt<%s,%sx%s,%s> [%s]" % (t, m.group(2), m.group(3), form, FAMILIES.get(m.group(6), m.group(6)))
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


def _avg_ms(stats_path):
    if not stats_path:
        return {}
    return {r["Name"]: float(r["AverageNs"]) / 1e6 for r in csv.DictReader(open(stats_path))}


def pmc(fetch_path, write_path, out, cmd, copy_mib, stats_path=None):
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

    def avg(vals):
        return sum(v for v, _ in vals) / max(1, len(vals))

    for name, vals in sorted(f.items(), key=lambda kv: -sum(v for v, _ in kv[1])):
        if "gemm_nt_kernel" not in name:
            continue
        fv, wv = avg(vals), avg(w.get(name, []))
        gb = (fv * ff + wv * wf) * 1024.0 / 1e9
        lines.append("| %s | %d | %.0f | %.0f | %.3f |" % (short_name(name), len(vals), fv, wv, gb))
    ms = _avg_ms(stats_path)
    if ms:
        lines += ["", "Achieved rate per kernel (calibrated bytes per dispatch over the kernel's average duration in "
                  "the kernel statistics of the same workload, %s; HBM peak 8000 GB/s; the kernels of the "
                  "synthetic input generator are left out):" % os.path.basename(stats_path), "",
                  "| kernel | dispatches | GB/dispatch | avg ms | GB/s | of 8 TB/s |", "|---|---:|---:|---:|---:|---:|"]
        rows = []
        for name, vals in f.items():
            # torch and rocBLAS kernels belong to the synthetic input generator
            if name not in ms or "MulFunctor" in name or name.startswith(("void at::", "Cijk_")):
                continue
            gb = (avg(vals) * ff + avg(w.get(name, [])) * wf) * 1024.0 / 1e9
            rows.append((gb * len(vals), name, len(vals), gb, ms[name]))
        for _, name, n, gb, t in sorted(rows, reverse=True)[:30]:
            lines.append("| %s | %d | %.4f | %.4f | %.0f | %.1f%% |" % (short_name(name), n, gb, t, gb / t * 1e3,
                                                                    gb / t * 1e5 / 8000.0))
    open(out, "w").write("\n".join(lines) + "\n")


def mfma(path, out, cmd):
    d = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        d[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = ["# rocprofv3 matrix-core counters", "", "Command: `%s`" % cmd, "",
             "GEMM source hash: %s" % gemm_source_hash(), "",
             "MfmaUtil = busy cycles of the matrix cores summed over SIMDs / (GPU active cycles x SIMDs), "
             "per dispatch, averaged over dispatches; MFMA GFLOP/dispatch = MOPS x 512 (operations issued, "
             "tile padding included).", "",
             "| kernel | dispatches | MfmaUtil % | MFMA GFLOP/dispatch (F32, BF16, F64) |", "|---|---:|---:|---:|"]
    rows = []
    for name, c in d.items():
        u = c.get("MfmaUtil", [])
        if not u:
            continue
        g = []
        for t in ("F32", "BF16", "F64"):
            v = c.get("SQ_INSTS_VALU_MFMA_MOPS_" + t, [])
            g.append(sum(v) / max(1, len(v)) * 512 / 1e9)
        if sum(g) <= 0:
            continue
        rows.append((sum(g) * len(u), name, len(u), sum(u) / len(u), g))
    for _, name, n, util, g in sorted(rows, reverse=True)[:30]:
        lines.append("| %s | %d | %.1f | %.2f, %.2f, %.2f |" % (short_name(name), n, util, g[0], g[1], g[2]))
    open(out, "w").write("\n".join(lines) + "\n")


def busy(path, out, cmd, tail_s=None):
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in csv.DictReader(open(path)))
    if not iv:
        raise SystemExit("empty kernel trace")
    if tail_s:
        t_end = max(e for _, e in iv)
        iv = [(a, b) for a, b in iv if a >= t_end - tail_s * 1e9]
    tot, cur_s, cur_e = 0, iv[0][0], iv[0][1]
    for s0, e0 in iv[1:]:
        if s0 > cur_e:
            tot += cur_e - cur_s
            cur_s, cur_e = s0, e0
        else:
            cur_e = max(cur_e, e0)
    tot += cur_e - cur_s
    span = max(e for _, e in iv) - iv[0][0]
    scope = ("the last %.3f s of the trace" % tail_s) if tail_s else "the whole trace"
    lines = ["# Device busy fraction from a rocprofv3 kernel trace", "", "Command: `%s`" % cmd, "",
             "Window: %s." % scope, "",
             "%d kernels; traced span %.3f s (first kernel start to last kernel end); at least one kernel "
             "running for %.3f s = %.1f%% of the span." % (len(iv), span / 1e9, tot / 1e9, 100.0 * tot / span)]
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "pmc", "mfma", "busy"])
    ap.add_argument("paths", nargs="+")
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--stats", default=None, help="pmc: kernel_stats.csv of the same command")
    ap.add_argument("--tail-s", type=float, default=None, help="busy: only the last seconds of the trace")
    a = ap.parse_args()
    if a.mode == "stats":
        stats(a.paths[0], a.paths[1], a.cmd)
    elif a.mode == "pmc":
        pmc(a.paths[0], a.paths[1], a.paths[2], a.cmd, a.copy_mib, a.stats)
    elif a.mode == "mfma":
        mfma(a.paths[0], a.paths[1], a.cmd)
    else:
        busy(a.paths[0], a.paths[1], a.cmd, a.tail_s)
