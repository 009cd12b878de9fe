"""Benchmark: converged roots per second of the rid-preconditioned Davidson
solver on one MI355X, mixed precision against the FP64 GPU path.

One step = one full-TDDFT eigen-solve for the 10 lowest roots plus one static
polarizability solve for 3 dipole right-hand sides on the no=200, nv=800
(N = 160000), Naux = 4000, Naux_ris = 900 synthetic molecule, with the rid
(minimal-auxiliary ris) preconditioner.  A step yields 13 converged
solutions (10 roots + 3 response vectors); value = solutions per second over
the timed steps, inputs resident in HBM before timing starts.

The JSON line also carries the per-step latency percentiles, the FP64 GPU
path's throughput on the same workload, the roofline figure of the dominant
kernel (the FP32 exchange contraction, timed with HIP events on the library's
stream), and the CPU oracle timed on a bounded sample of the same work.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0}  # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0  # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(p, n_mv_per_step, roots_per_step, naux_sample=200):
    """The FP64 oracle's outer product timed on a slice of the auxiliary index.

    The oracle's (A+B, A-B) product is linear in Naux; it is timed on the
    first `naux_sample` rows of the same tensors for one vector and scaled to
    the full Naux, then multiplied by the number of outer products one step
    needs (from the GPU run of the same algorithm).  Preconditioner and
    subspace work are left out, which favours the CPU.
    """
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import operators as ops
    from oracle.operators import OracleProblem

    d = {
        "no": p.no, "nv": p.nv, "a_x": p.a_x,
        "eps_occ": p.eps_occ.cpu().numpy(), "eps_vir": p.eps_vir.cpu().numpy(),
        "b_ia": p.b_ia[:naux_sample].cpu().numpy(), "b_ij": p.b_ij[:naux_sample].cpu().numpy(),
        "b_ab": p.b_ab[:naux_sample].cpu().numpy(),
    }
    op = OracleProblem.from_arrays(d)
    x = np.random.default_rng(0).standard_normal((op.n, 1))
    ops.apply_apb_amb(op, x)  # warm
    t0 = time.perf_counter()
    reps = 0
    while True:
        ops.apply_apb_amb(op, x)
        reps += 1
        if time.perf_counter() - t0 > 10.0 or reps >= 20:
            break
    t_slice = (time.perf_counter() - t0) / reps
    t_vec = t_slice * p.naux / naux_sample
    t_step = t_vec * n_mv_per_step
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {
        "value": roots_per_step / t_step,
        "unit": "roots/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": ("oracle (A+B, A-B) product of one vector on Naux rows 0..%d of the same tensors, "
                   "%d repetitions, %.3f s each, scaled by Naux/%d and by the %d outer products per step "
                   "of the GPU run (preconditioner and subspace work excluded)"
                   % (naux_sample - 1, reps, t_slice, naux_sample, n_mv_per_step)),
    }


def measured_traffic(family: str, dtype: str):
    """Calibrated HBM bytes per launch of `family` from the committed counter
    summary, or None when the GEMM source changed since the counters were
    taken (or no summary exists)."""
    import re

    path = os.path.join(ROOT, "profiles", "exch_contractions_c2_mixed_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    sys.path.insert(0, os.path.join(ROOT, "paper_2404_17133_amd"))
    from profsum import gemm_source_hash

    text = open(path).read()
    m = re.search(r"GEMM source hash: (\w+)", text)
    if not m or m.group(1) != gemm_source_hash():
        return None
    t = {"f32": "float", "bf16": "bf16_t", "f64": "double"}[dtype]
    fam = family[4:] if family.startswith("ris_") else family
    for line in text.splitlines():
        if line.startswith("| gemm_nt<%s,128x128," % t) and line.split("|")[1].strip().endswith("[%s]" % fam):
            return float(line.split("|")[5]) * 1e9
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precond", default="ris", choices=["ris", "diag"])
    ap.add_argument("--fp64-steps", type=int, default=1, help="steps of the FP64 GPU comparison (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="MiB of a plain device copy (x * 1.0 on float32) run before timing, so that "
                         "hardware-counter runs can calibrate byte counters against a known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2404_17133_amd as rid
    from synth import config_sizes, make_dipoles, make_problem

    no, nv, naux, nris, seed = config_sizes("c2")
    t0 = time.time()
    p = make_problem(no, nv, naux, nris, seed=seed, device="cuda:0")
    pm = make_dipoles(p, 3)
    torch.cuda.synchronize()
    log("inputs generated on the device in %.1f s" % (time.time() - t0))
    if args.copy_probe > 0:
        xs = torch.ones(args.copy_probe * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        ys = xs * 1.0  # reads and writes copy_probe MiB
        torch.cuda.synchronize()
        del xs, ys
        log("copy probe: %d MiB read + %d MiB written" % (args.copy_probe, args.copy_probe))
    ctx = rid.Context(0)
    prob = rid.Problem.from_synth(ctx, p)
    k = args.k
    roots_per_step = k + pm.shape[0]

    def step(precision):
        e = prob.eigen(k, "rpa", args.precond, precision, vectors=False)
        a = prob.polarizability(pm, [0.0], args.precond, precision)
        if e["status"] != 0 or a["status"] != 0:
            raise RuntimeError("solve did not converge: %d %d" % (e["status"], a["status"]))
        return e, a

    for w in range(args.warmup):
        step("mixed")
        log("warmup step %d done" % w)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    lat = []
    last = None
    n_mv = 0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        ts = time.perf_counter()
        e, a = step("mixed")
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        n_mv = e["stats"]["n_mv"] + a["stats"]["n_mv"]
        last = (e, a)
        log("step %d: %.2f s (eigen %d iterations, %d outer products; alpha %d iterations)"
            % (s, lat[-1], e["stats"]["n_iter"], e["stats"]["n_mv"], a["stats"]["n_iter"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = ctx.profile_read()
    ctx.profile(False)
    value = roots_per_step * args.steps / elapsed

    # dominant kernel: the family with the largest summed event time
    fam, st = max(prof.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = st["ms"] / st["launches"]
    dtype = "f32" if not fam.startswith("ris_") else "bf16"
    achieved = st["flops"] / st["launches"] / (avg_ms * 1e-3) / 1e12
    traffic = measured_traffic(fam, dtype)
    roofline = {"bound": "mfma", "kernel": fam, "achieved": round(achieved, 2), "peak": PEAK[dtype],
                "unit": "TFLOP/s", "frac": round(achieved / PEAK[dtype], 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": st["bytes"] / st["launches"],
                "avg_launch_ms": round(avg_ms, 4), "launches": st["launches"],
                "flops_per_launch": st["flops"] / st["launches"]}

    out = {
        "metric": "converged roots/sec + p50/p99 solve latency, mixed-precision vs FP64 Davidson",
        "value": round(value, 4),
        "unit": "roots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "full-TDDFT 10 lowest roots + static polarizability (3 RHS), no=200 nv=800 "
                        "(N=160000) Naux=4000 Naux_ris=900, rid preconditioner, mixed precision "
                        "(FP32 outer products, BF16 ris products, FP64 subspace)",
            "precond": args.precond,
            "roots_per_step": roots_per_step,
        },
        "latency_s": {"p50": round(float(np.percentile(lat, 50)), 3),
                      "p99": round(float(np.percentile(lat, 99)), 3)},
        "roofline": roofline,
        "kernels": {kf: {"launches": v["launches"], "ms": round(v["ms"], 1),
                         "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 1)}
                    for kf, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:12]},
        "solve": {"eigen_iters": last[0]["stats"]["n_iter"], "eigen_n_mv": last[0]["stats"]["n_mv"],
                  "eigen_inner_mv": last[0]["stats"]["n_inner_mv"],
                  "alpha_iters": last[1]["stats"]["n_iter"],
                  "omega": [round(float(x), 10) for x in last[0]["omega"]]},
    }

    if args.fp64_steps > 0:
        lat64 = []
        for s in range(args.fp64_steps):
            ts = time.perf_counter()
            e64, a64 = step("fp64")
            torch.cuda.synchronize()
            lat64.append(time.perf_counter() - ts)
            log("fp64 step %d: %.2f s" % (s, lat64[-1]))
        v64 = roots_per_step * len(lat64) / sum(lat64)
        dom = float(np.max(np.abs(last[0]["omega"] - e64["omega"])))
        dal = float(np.max(np.abs(last[1]["alpha"] - a64["alpha"])) / np.max(np.abs(a64["alpha"])))
        out["fp64_gpu"] = {"value": round(v64, 4), "unit": "roots/s",
                           "latency_s_p50": round(float(np.percentile(lat64, 50)), 3),
                           "speedup_mixed_vs_fp64": round(value / v64, 3),
                           "max_abs_omega_diff_Ha": dom, "max_rel_alpha_diff": dal}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, n_mv, roots_per_step)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
