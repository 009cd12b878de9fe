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
    # about 10 s of CPU work (at least 5 repetitions)
    while True:
        ops.apply_apb_amb(op, x)
        reps += 1
        if (time.perf_counter() - t0 > 10.0 and reps >= 5) or reps >= 400:
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


def oracle_solves(precond, reps=3, no100=False):
    """The FP64 oracle's whole step -- full-TDDFT 10 lowest roots plus the
    static polarizability of 3 dipole right-hand sides, the same algorithm
    and preconditioner as the GPU step -- timed end to end on the no=20
    molecule (median of `reps` solves with all BLAS threads, and with one),
    and with no100 once on the no=100 molecule (minutes of CPU time).
    Returns a dict for the JSON line."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import OracleProblem, eigen_rpa, polarizability
    from synth import config_sizes, make_dipoles, make_problem

    def one(name):
        no, nv, naux, nris, seed = config_sizes(name)
        p = make_problem(no, nv, naux, nris, seed=seed)
        op = OracleProblem.from_arrays(p.numpy())
        pm = make_dipoles(p, 3).numpy().T

        def run():
            t0 = time.perf_counter()
            e = eigen_rpa(op, 10, precond)
            a = polarizability(op, pm, [0.0], precond)
            if not (e.converged and a.converged):
                raise RuntimeError("oracle solve did not converge")
            return time.perf_counter() - t0, e.n_iter, a.n_iter
        return run

    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    out = {"what": "oracle full-TDDFT 10 roots + static alpha (3 RHS), %s preconditioner, tolerance 1e-5, "
                   "time.perf_counter per whole step" % ("rid" if precond == "ris" else "diagonal"),
           "blas": sorted({"%s (%s)" % (i.get("internal_api"), i.get("version")) for i in threadpool_info()})}
    run0 = one("c0")
    run0()  # warm (imports, first BLAS calls)
    ts = [run0() for _ in range(reps)]
    out["no20_all_threads"] = {"threads": int(threads), "median_s": round(float(np.median([t[0] for t in ts])), 3),
                               "roots_per_s": round(13.0 / float(np.median([t[0] for t in ts])), 3),
                               "eigen_iters": ts[0][1], "alpha_iters": ts[0][2], "repeats": reps}
    with threadpool_limits(1):
        ts1 = [run0() for _ in range(reps)]
    out["no20_one_thread"] = {"threads": 1, "median_s": round(float(np.median([t[0] for t in ts1])), 3),
                              "roots_per_s": round(13.0 / float(np.median([t[0] for t in ts1])), 3)}
    if not no100:
        return out
    t1 = one("c1")()
    out["no100_all_threads"] = {"threads": int(threads), "seconds": round(t1[0], 2),
                                "roots_per_s": round(13.0 / t1[0], 4), "eigen_iters": t1[1], "alpha_iters": t1[2],
                                "repeats": 1}
    return out


def per_root_error(size, omega, alpha):
    """Errors of a GPU step against the stored FP64 oracle results of the
    same molecule (tolerance 1e-8; tests/golden/make_golden.py): per root
    |Omega - Omega_oracle| in Ha, and the largest |alpha - alpha_oracle|
    relative to max |alpha_oracle| of the static polarizability."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", "oracle_%s.json" % size)
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    ref = np.array(g["rpa_omega"])
    a0 = np.array(g["alpha"][g["alpha_omegas"].index(0.0)])
    return {"omega_abs_err_Ha": [float(v) for v in np.abs(np.asarray(omega)[:len(ref)] - ref)],
            "alpha_max_rel_err": float(np.abs(np.asarray(alpha) - a0).max() / np.abs(a0).max()),
            "oracle": "tests/golden/oracle_%s.json (FP64 CPU oracle, tolerance %g)" % (size, g["tol"])}


def residual_slope(history):
    """Least-squares slope of log10 of the largest residual norm per outer
    iteration (the convergence rate the paper plots for one molecule)."""
    import numpy as np

    h = np.asarray([v for v in history if v > 0])
    if len(h) < 2:
        return None
    return round(float(np.polyfit(np.arange(len(h)), np.log10(h), 1)[0]), 4)


def measured_traffic(family: str, dtype: str, size: str = "c2"):
    """Calibrated HBM bytes per launch of `family` from the committed counter
    summary of the no=200 workload, or None for another workload, when the
    GEMM source changed since the counters were taken, or when no summary
    exists."""
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
    if size != "c2":
        return None
    t = {"f32": "float", "bf16": "bf16_t", "f64": "double"}[dtype]
    fam = family[4:] if family.startswith("ris_") else family
    # dispatch-weighted mean over the tile shapes the autotuner picked (the
    # counter table only: the summary's second table lists rates)
    n_tot, b_tot = 0, 0.0
    for line in text.split("Achieved rate")[0].splitlines():
        cells = [c.strip() for c in line.split("|")]
        if len(cells) > 5 and cells[1].startswith("gemm_nt<%s," % t) and cells[1].endswith("[%s]" % fam):
            n = int(cells[2])
            n_tot += n
            b_tot += n * float(cells[5]) * 1e9
    return b_tot / n_tot if n_tot else None


def f32_problem(rid, ctx, d, dipoles=False):
    """A synthetic molecule generated in FP64 on the device and lent to the
    library as FP32 tensors (the FP64 copy is freed; only mixed-precision
    solves run on it).  Returns (problem, dipole block or None)."""
    import torch

    from synth import make_dipoles, make_problem

    p = make_problem(d["no"], d["nv"], d["naux"], d["naux_ris"], naux_ris_k=d["naux_ris_k"], seed=d["seed"],
                     device="cuda:0")
    dip = make_dipoles(p, 3) if dipoles else None
    t = [x.float() for x in (p.b_ia, p.b_ij, p.b_ab, p.bris_ia, p.bris_ij, p.bris_ab)]
    eo, ev = p.eps_occ.cpu().numpy(), p.eps_vir.cpu().numpy()
    a_x, nk, tc = p.a_x, p.naux_ris_k, p.t_cut
    del p
    torch.cuda.empty_cache()
    return rid.Problem(ctx, eo, ev, t[0], t[1], t[2], a_x, t[3], t[4], t[5], nk, tc), dip


def bench_batch(args):
    """Batched workload: molecules m = 0..M-1 of synth.batch_member (no
    log-uniform in [20, 200], RPA eigen-solves with k in {5, 10, 20}), mixed
    precision, rid preconditioner, solved together by rid_batch_solve."""
    import numpy as np
    import torch

    import paper_2404_17133_amd as rid
    from synth import batch_member

    members = [batch_member(m) for m in range(args.molecules)]
    ctx = rid.Context(0)
    t0 = time.time()
    probs = [None] * len(members)
    for m in sorted(range(len(members)), key=lambda i: -members[i]["no"]):
        probs[m], _ = f32_problem(rid, ctx, members[m])
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    log("%d molecules generated in %.1f s (FP32 tensors %.1f GB; device memory free %.1f of %.1f GB)"
        % (len(members), time.time() - t0, sum(p._keep[0].numel() + p._keep[1].numel() + p._keep[2].numel()
                                               for p in probs) * 4e-9, free / 1e9, total / 1e9))
    opts = rid.default_opts("ris", "mixed")
    reqs = [rid.make_request("eigen", opts, k=d["k"], mode="rpa")[0] for d in members]
    roots = sum(d["k"] for d in members)

    def run():
        ts = time.perf_counter()
        st, out = rid.batch_solve(ctx, probs, reqs)
        el = time.perf_counter() - ts
        if st != 0:
            raise RuntimeError("batch status %d: %s; %s" % (st, [o["status"] for o in out], ctx.last_error()))
        return el, out

    for w in range(args.warmup):
        el, _ = run()
        log("warmup batch %d: %.2f s" % (w, el))
    ctx.profile(True)
    ctx.profile_read()
    lats, last, total = [], None, 0.0
    for s in range(args.steps):
        el, last = run()
        total += el
        lats += [o["t_done_ms"] * 1e-3 for o in last]
        log("batch %d: %.2f s" % (s, el))
    prof = ctx.profile_read()
    ctx.profile(False)
    value = roots * args.steps / total
    out = {
        "metric": "converged roots/sec + p50/p99 solve latency, mixed-precision vs FP64 Davidson",
        "value": round(value, 4), "unit": "roots/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch of %d molecules, no log-uniform in [20, 200], nv=4no, Naux=20no, "
                               "Naux_ris=4.5no, full-TDDFT k in {5,10,20}, rid preconditioner, mixed precision, "
                               "one rid_batch_solve per step" % len(members), "roots_per_step": roots},
        "latency_s": {"p50": round(float(np.percentile(lats, 50)), 3),
                      "p99": round(float(np.percentile(lats, 99)), 3)},
        "kernels": {kf: {"launches": v["launches"], "ms": round(v["ms"], 1),
                         "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 1)}
                    for kf, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:8]},
        "iterations": {"mean": float(np.mean([o["stats"]["n_iter"] for o in last])),
                       "max": int(max(o["stats"]["n_iter"] for o in last))},
        "members": [[d["no"], d["k"], o["stats"]["n_iter"], o["stats"]["n_mv"], round(o["t_start_ms"] * 1e-3, 2),
                     round(o["t_done_ms"] * 1e-3, 2)] for d, o in zip(members, last)],
    }
    if args.sequential:
        ts = time.perf_counter()
        for p, r in zip(probs, reqs):
            st, o = rid.batch_solve(ctx, [p], [r])
            if st != 0:
                raise RuntimeError("sequential status %d" % st)
        seq = time.perf_counter() - ts
        out["sequential"] = {"value": round(roots / seq, 4), "unit": "roots/s", "seconds": round(seq, 2),
                             "speedup_batched_vs_sequential": round(value / (roots / seq), 3)}
        log("sequential: %.2f s" % seq)
    ctx.close()
    print(json.dumps(out), flush=True)


def f64_problem(rid, ctx, d, dipoles=False):
    """A synthetic molecule lent to the library as FP64 tensors: FP64 solves
    use them directly, mixed-precision solves through the FP32/BF16 copies the
    library makes.  Returns (problem, dipole block or None)."""
    from synth import make_dipoles, make_problem

    p = make_problem(d["no"], d["nv"], d["naux"], d["naux_ris"], naux_ris_k=d["naux_ris_k"], seed=d["seed"],
                     device="cuda:0")
    dip = make_dipoles(p, 3) if dipoles else None
    return rid.Problem.from_synth(ctx, p), dip


def bench_serve(args):
    """Served stream: requests of synth.serve_trace (no log-uniform in
    [20, no_max], 70% TDA/RPA eigen k 5..20, 30% polarizability 3 RHS x 3
    frequencies), mixed precision, rid preconditioner.  First all requests
    arrive at once (saturated throughput), then the same requests arrive as a
    Poisson stream at each of `loads` times that throughput (latency
    percentiles).  With --fp64 the molecules are kept in FP64 and the same
    requests are also served by the FP64 path: saturated, and replaying the
    arrival times of the mixed run at the first load."""
    import numpy as np
    import torch

    import paper_2404_17133_amd as rid
    from synth import serve_trace

    loads = [float(x) for x in args.loads.split(",")] if args.loads else [args.load]
    trace = serve_trace(args.requests, no_max=args.no_max)
    ctx = rid.Context(0)
    t0 = time.time()
    probs, dips = [None] * len(trace), [None] * len(trace)
    make = f64_problem if args.fp64 else f32_problem
    for r in sorted(range(len(trace)), key=lambda i: -trace[i]["no"]):
        probs[r], dips[r] = make(rid, ctx, trace[r], dipoles=trace[r]["kind"] != "eigen")
    torch.cuda.synchronize()
    log("%d requests' molecules generated in %.1f s" % (len(trace), time.time() - t0))

    def requests(opts):
        reqs, keeps, roots = [], [], 0
        for d, dp in zip(trace, dips):
            if d["kind"] == "eigen":
                r, kp = rid.make_request("eigen", opts, k=d["k"], mode=d["mode"])
                roots += d["k"]
            else:
                r, kp = rid.make_request("polarizability", opts, p=dp, omegas=d["omegas"])
                roots += 3 * len(d["omegas"])
            reqs.append(r)
            keeps.append(kp)
        return reqs, keeps, roots

    def serve(reqs, keeps, gaps):
        srv = rid.Server(ctx, hbm_budget_bytes=args.hbm_budget_gb << 30, max_slots=args.slots)
        tick = []
        ts = time.perf_counter()
        tnext = ts
        for i, (p, r) in enumerate(zip(probs, reqs)):
            tnext += gaps[i]
            delay = tnext - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tick.append(srv.submit(p, r, keep=keeps[i]))
        res = [srv.wait(t) for t in tick]
        srv.close()
        bad = [x["status"] for x in res if x["status"] != 0]
        if bad:
            raise RuntimeError("served requests failed: %s" % bad)
        lat = np.array([(x["t_done_ms"] - x["t_arrival_ms"]) * 1e-3 for x in res])
        span = (max(x["t_done_ms"] for x in res) - min(x["t_arrival_ms"] for x in res)) * 1e-3
        return lat, span, res

    def pct(lat):
        return {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3)}

    reqs, keeps, roots = requests(rid.default_opts("ris", "mixed"))
    lat_s, span_s, res_mixed = serve(reqs, keeps, [0.0] * len(trace))
    rate = len(trace) / span_s
    log("saturated: %.2f s for %d requests (%.3f req/s)" % (span_s, len(trace), rate))
    runs = []
    for load in loads:
        gaps = [d["gap"] / (load * rate) for d in trace]
        lat_p, span_p, _ = serve(reqs, keeps, gaps)
        log("Poisson at %.2f x saturation: %.2f s, p50 %.2f s, p99 %.2f s"
            % (load, span_p, np.percentile(lat_p, 50), np.percentile(lat_p, 99)))
        runs.append({"load": load, "rate_req_per_s": round(load * rate, 4), "roots_per_s": round(roots / span_p, 4),
                     "latency_s": pct(lat_p), "gaps": gaps})
    first = runs[0]
    out = {
        "metric": "converged roots/sec + p50/p99 solve latency, mixed-precision vs FP64 Davidson",
        "value": round(roots / span_s, 4), "unit": "roots/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(1e3 * span_s, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "served stream of %d requests, no log-uniform in [20, %d], 70%% TDA/RPA eigen "
                               "k 5..20, 30%% polarizability 3 RHS x 3 frequencies, rid preconditioner, mixed "
                               "precision, %d slots" % (len(trace), args.no_max, args.slots),
                   "roots_per_pass": roots},
        "latency_s": dict(first["latency_s"], arrivals="Poisson at %.2f x the saturated request rate (%.4f req/s)"
                          % (first["load"], first["rate_req_per_s"])),
        "poisson_roots_per_s": first["roots_per_s"],
        "loads": [{k: v for k, v in r.items() if k != "gaps"} for r in runs],
        "saturated_latency_s": pct(lat_s),
    }
    if args.fp64:
        reqs64, keeps64, _ = requests(rid.default_opts("ris", "fp64"))
        lat64, span64, res64 = serve(reqs64, keeps64, [0.0] * len(trace))
        log("FP64 saturated: %.2f s" % span64)
        lat64p, span64p, _ = serve(reqs64, keeps64, first["gaps"])
        log("FP64 replay of the mixed arrivals at %.2f x: %.2f s" % (first["load"], span64p))
        dom, dal = 0.0, 0.0
        for a, b in zip(res_mixed, res64):
            if "omega" in a:
                dom = max(dom, float(np.max(np.abs(a["omega"] - b["omega"]))))
            if "alpha" in a:
                dal = max(dal, float(np.max(np.abs(a["alpha"] - b["alpha"]) / np.abs(b["alpha"]).max())))
        out["fp64_gpu"] = {
            "value": round(roots / span64, 4), "unit": "roots/s", "saturated_latency_s": pct(lat64),
            "replay": {"arrivals": "the mixed run's arrival times at %.2f x" % first["load"],
                       "roots_per_s": round(roots / span64p, 4), "latency_s": pct(lat64p)},
            "speedup_mixed_vs_fp64": round(span64 / span_s, 3),
            "max_abs_omega_diff_Ha": dom, "max_rel_alpha_diff": dal,
        }
    ctx.close()
    print(json.dumps(out), flush=True)


def served_leg(n_req=12, no_max=100, slots=8, load=0.7, budget_gb=96):
    """A short served stream beside the single-molecule step: n_req requests
    of synth.serve_trace (no log-uniform in [20, no_max]), kept in FP64 so
    that both paths serve the very same molecules.  Mixed precision first
    with all requests at once (saturated rate), then as Poisson arrivals at
    `load` x that rate; FP64 saturated, then replaying the mixed run's
    arrival times.  Returns roots/s and latency percentiles of each."""
    import numpy as np
    import torch

    import paper_2404_17133_amd as rid
    from synth import serve_trace

    trace = serve_trace(n_req, no_max=no_max)
    ctx = rid.Context(0)
    probs, dips = [], []
    for d in trace:
        pr, dp = f64_problem(rid, ctx, d, dipoles=d["kind"] != "eigen")
        probs.append(pr)
        dips.append(dp)
    torch.cuda.synchronize()

    def requests(precision):
        opts = rid.default_opts("ris", precision)
        reqs, keeps, roots = [], [], 0
        for d, dp in zip(trace, dips):
            if d["kind"] == "eigen":
                r, kp = rid.make_request("eigen", opts, k=d["k"], mode=d["mode"])
                roots += d["k"]
            else:
                r, kp = rid.make_request("polarizability", opts, p=dp, omegas=d["omegas"])
                roots += 3 * len(d["omegas"])
            reqs.append(r)
            keeps.append(kp)
        return reqs, keeps, roots

    def serve(reqs, keeps, gaps):
        srv = rid.Server(ctx, hbm_budget_bytes=budget_gb << 30, max_slots=slots)
        tick = []
        tnext = time.perf_counter()
        for i, (pr, r) in enumerate(zip(probs, reqs)):
            tnext += gaps[i]
            delay = tnext - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tick.append(srv.submit(pr, r, keep=keeps[i]))
        res = [srv.wait(t) for t in tick]
        srv.close()
        bad = [x["status"] for x in res if x["status"] != 0]
        if bad:
            raise RuntimeError("served requests failed: %s" % bad)
        lat = np.array([(x["t_done_ms"] - x["t_arrival_ms"]) * 1e-3 for x in res])
        span = (max(x["t_done_ms"] for x in res) - min(x["t_arrival_ms"] for x in res)) * 1e-3
        return lat, span, res

    def pct(lat):
        return {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3)}

    out = {"workload": "%d served requests, no log-uniform in [20, %d], 70%% TDA/RPA eigen k 5..20, 30%% "
                       "polarizability 3 RHS x 3 frequencies, rid preconditioner, %d slots; molecules in FP64, "
                       "served by both paths" % (n_req, no_max, slots)}
    legs = {}
    for precision in ("mixed", "fp64"):
        reqs, keeps, roots = requests(precision)
        serve(reqs, keeps, [0.0] * n_req)  # warm: tensor copies and tuned shapes
        lat_s, span_s, res_s = serve(reqs, keeps, [0.0] * n_req)
        if precision == "mixed":
            rate = n_req / span_s
            gaps = [d["gap"] / (load * rate) for d in trace]
        lat_p, span_p, _ = serve(reqs, keeps, gaps)
        legs[precision] = res_s
        out[precision] = {"saturated_roots_per_s": round(roots / span_s, 4), "saturated_s": round(span_s, 3),
                          "saturated_latency_s": pct(lat_s),
                          "poisson_roots_per_s": round(roots / span_p, 4), "poisson_latency_s": pct(lat_p)}
        log("served %s: saturated %.2f s (%.2f roots/s), arrivals p50 %.2f s p99 %.2f s" % (
            precision, span_s, roots / span_s, np.percentile(lat_p, 50), np.percentile(lat_p, 99)))
    out["roots_per_pass"] = roots
    out["arrivals"] = "Poisson at %.2f x the mixed saturated request rate (%.4f req/s), the same times for both" % (
        load, load * rate)
    out["speedup_mixed_vs_fp64_saturated"] = round(out["mixed"]["saturated_roots_per_s"]
                                                   / out["fp64"]["saturated_roots_per_s"], 3)
    dom, dal = 0.0, 0.0
    for a, b in zip(legs["mixed"], legs["fp64"]):
        if "omega" in a:
            dom = max(dom, float(np.max(np.abs(a["omega"] - b["omega"]))))
        if "alpha" in a:
            dal = max(dal, float(np.max(np.abs(a["alpha"] - b["alpha"]) / np.abs(b["alpha"]).max())))
    out["max_abs_omega_diff_Ha"] = dom
    out["max_rel_alpha_diff"] = dal
    ctx.close()
    return out


SWEEP = [
    # label, preconditioner, Naux_ris (None: config value), exchange rows (None: Naux_ris/9), source, noise, window
    ("diagonal", "diag", None, None, "svd", 0.05, True),
    ("rid (s,s): J and K on the s rows", "ris", "s", "s", "svd", 0.05, True),
    ("rid (d,s): J on all rows, K on the s rows", "ris", None, None, "svd", 0.05, True),
    ("rid (d,d): J and K on all rows", "ris", None, "all", "svd", 0.05, True),
    ("rid (d,s), twice the auxiliary rows", "ris", "x2", None, "svd", 0.05, True),
    ("full auxiliary basis, 5% noise, window", "ris", "full", "all", "full", 0.05, True),
    ("exact model: T = A (no noise, no window)", "ris", "full", "all", "full", 0.0, False),
]


def bench_sweep(args):
    """Preconditioner richness sweep (Sec. 3.2, Fig. 2 analogue) on the
    no=100 workload: iterations and products of the full-TDDFT solve for the
    ris model with more or fewer auxiliary rows in its Coulomb (J) and
    exchange (K) parts, up to the exact model T = A; the roots are checked
    against the stored FP64 oracle results."""
    import numpy as np
    import torch

    import paper_2404_17133_amd as rid
    from synth import config_sizes, make_problem

    no, nv, naux, nris, seed = config_sizes("c1")
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_c1.json")))
    ref = np.array(gold["rpa_omega"])
    k = gold["k"]
    rows = []
    for label, pc, nr, nk, src, noise, window in SWEEP:
        n_ris = {None: nris, "s": int(round(nris / 9)), "x2": 2 * nris, "full": naux}[nr]
        n_k = {None: None, "s": int(round(nris / 9)), "all": n_ris}[nk]
        kw = {} if window else {"t_cut": float("inf")}
        p = make_problem(no, nv, naux, n_ris, naux_ris_k=n_k, seed=seed, device="cuda:0", ris_source=src,
                         noise=noise, **kw)
        ctx = rid.Context(0)
        prob = rid.Problem.from_synth(ctx, p)
        prob.eigen(k, "rpa", pc, "mixed", vectors=False)  # warm (tuning, casts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = prob.eigen(k, "rpa", pc, "mixed", vectors=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = out["stats"]
        rows.append({"preconditioner": label, "naux_ris_j": n_ris if pc == "ris" else 0,
                     "naux_ris_k": p.naux_ris_k if pc == "ris" else 0, "status": out["status"],
                     "n_iter": st["n_iter"], "n_mv": st["n_mv"], "n_inner_mv": st["n_inner_mv"],
                     "seconds": round(el, 3), "max_abs_omega_err_Ha": float(np.abs(out["omega"] - ref).max())})
        log("%-45s iters %3d  products %4d  inner %5d  %.2f s  err %.1e" % (
            label, st["n_iter"], st["n_mv"], st["n_inner_mv"], el, rows[-1]["max_abs_omega_err_Ha"]))
        ctx.close()
        del p, prob
        torch.cuda.empty_cache()
    # warm start (NEXT-2): the X, Y of the default problem seed the solve on a
    # neighbour (every tensor perturbed by 1 %, as after a geometry step)
    from synth import related_problem
    p1 = make_problem(no, nv, naux, nris, seed=seed, device="cuda:0")
    p2 = related_problem(p1, step=0.01)
    ctx = rid.Context(0)
    g1, g2 = rid.Problem.from_synth(ctx, p1), rid.Problem.from_synth(ctx, p2)
    first = g1.eigen(k, "rpa", "ris", "mixed")
    guess = torch.cat([first["x"], first["y"]]).contiguous()
    g2.eigen(k, "rpa", "ris", "mixed", vectors=False)  # warm-up of the new shapes
    warm_rows = {}
    for name, kw in (("cold", {}), ("warm", {"guess": guess})):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = g2.eigen(k, "rpa", "ris", "mixed", vectors=False, **kw)
        torch.cuda.synchronize()
        warm_rows[name] = {"status": out["status"], "n_iter": out["stats"]["n_iter"], "n_mv": out["stats"]["n_mv"],
                           "n_inner_mv": out["stats"]["n_inner_mv"], "seconds": round(time.perf_counter() - t0, 3),
                           "omega": out["omega"]}
        log("%s start on the neighbour: iters %d products %d  %.2f s" % (
            name, out["stats"]["n_iter"], out["stats"]["n_mv"], warm_rows[name]["seconds"]))
    diff = float(np.abs(warm_rows["warm"]["omega"] - warm_rows["cold"]["omega"]).max())
    for v in warm_rows.values():
        v.pop("omega")
    ctx.close()
    print(json.dumps({"workload": "preconditioner sweep: full TDDFT, 10 roots, no=100 nv=400 Naux=2000, mixed "
                                  "precision, tolerance 1e-5", "rows": rows,
                      "warm_start": {"neighbour": "every tensor x (1 + 0.01 Z), energies moved by 0.001 U[-1,1]",
                                     "cold": warm_rows["cold"], "warm": warm_rows["warm"],
                                     "max_abs_omega_diff_Ha": diff}}), flush=True)


def bench_rsh(args):
    """Global vs range-separated hybrid (NEXT-3; Sec. 4, wB97X vs PBE0) on
    the no=100 molecule: TDA, 10 roots, mixed precision, diagonal and rid
    preconditioners.  The range-separated problem adds b_x (pq|rs)^LR
    through a second tensor with Naux rows (a_x = 0.157706, b_x = 1 - a_x);
    the global hybrid has a_x = 0.25.  Roots are checked against the FP64
    oracle's products through their residuals (each converged root's
    residual norm is reported by the solver)."""
    import numpy as np
    import torch

    import paper_2404_17133_amd as rid
    from synth import config_sizes, make_problem

    no, nv, naux, nris, seed = config_sizes("c1")
    rows = []
    for name, kw in (("global hybrid (a_x = 0.25)", dict(a_x=0.25)),
                     ("range-separated (a_x = 0.157706, b_x = 0.842294)",
                      dict(a_x=0.157706, b_x=0.842294, naux_lr=naux))):
        p = make_problem(no, nv, naux, nris, seed=seed, device="cuda:0", **kw)
        ctx = rid.Context(0)
        prob = rid.Problem.from_synth(ctx, p)
        for mode in ("tda", "rpa"):
            for pc in ("diag", "ris"):
                prob.eigen(10, mode, pc, "mixed", vectors=False)  # warm
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = prob.eigen(10, mode, pc, "mixed", vectors=False)
                torch.cuda.synchronize()
                st = out["stats"]
                rows.append({"functional": name, "mode": mode, "preconditioner": pc, "status": out["status"],
                             "n_iter": st["n_iter"], "n_mv": st["n_mv"], "n_inner_mv": st["n_inner_mv"],
                             "seconds": round(time.perf_counter() - t0, 3),
                             "max_resid": float(np.max(out["resid"]))})
                log("%-50s %s %-4s iters %3d products %4d  %.2f s" % (name, mode, pc, st["n_iter"], st["n_mv"],
                                                                      rows[-1]["seconds"]))
        ctx.close()
        del p, prob
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "global vs range-separated hybrid: no=100 nv=400 Naux=2000 Naux_ris=450, "
                                  "10 roots, mixed precision, tolerance 1e-5", "rows": rows}), flush=True)


def bench_molecule(args):
    """rid against the diagonal preconditioner on a molecule-derived problem
    (the minimal auxiliary basis of Sec. 2.2.2 built from integrals): a
    50-atom synthetic molecule with no=100, nv=400 (N = 40000), a full
    fitting basis of 950 functions for A and the minimal s, p, d basis of 450
    functions (theta = 0.6; exchange on the 50 s functions) for the ris
    model, both built on the device; full TDDFT and TDA, 10 roots, mixed
    precision, tolerance 1e-5."""
    import numpy as np
    import torch

    import paper_2404_17133_amd as rid
    from synth import make_molecule

    mol = make_molecule(50, 100, 400, seed=500)
    ctx = rid.Context(0)
    t0 = time.perf_counter()
    prob = rid.molecule_problem(ctx, mol)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    log("tensors built on the device in %.2f s (nao %d, full %d, minimal %d auxiliary functions)" % (
        t_build, mol.nao, prob.naux, prob.naux_ris))
    rows = []
    for mode in ("rpa", "tda"):
        omegas = {}
        for pc in ("diag", "ris"):
            prob.eigen(10, mode, pc, "mixed", vectors=False)  # warm (tuning, casts)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            out = prob.eigen(10, mode, pc, "mixed", vectors=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - ts
            st = out["stats"]
            omegas[pc] = out["omega"]
            rows.append({"mode": mode, "preconditioner": pc, "status": out["status"], "n_iter": st["n_iter"],
                         "n_mv": st["n_mv"], "n_inner_mv": st["n_inner_mv"], "seconds": round(el, 3),
                         "precond_time_share": round(st["t_precond_ms"] / max(st["t_total_ms"], 1e-9), 4),
                         "omega": [round(float(x), 10) for x in out["omega"]]})
            log("%s %-4s iterations %3d products %4d inner %5d  %.2f s" % (mode, pc, st["n_iter"], st["n_mv"],
                                                                         st["n_inner_mv"], el))
        rows[-1]["max_abs_omega_diff_vs_diag_Ha"] = float(np.abs(omegas["ris"] - omegas["diag"]).max())
    ctx.close()
    print(json.dumps({"workload": "molecule-derived problem: 50 atoms, no=100 nv=400 (N=40000), nao %d, full "
                                  "auxiliary basis %d functions (s, p, d shells), minimal basis %d (theta 0.6, "
                                  "s/p/d; exchange on the s rows), kappa %.3g, 10 roots, mixed precision, "
                                  "tolerance 1e-5" % (mol.nao, prob.naux, prob.naux_ris, mol.kappa),
                      "tensor_build_s": round(t_build, 3), "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=2,
                    help="untimed steps; the first tunes the GEMM shapes, the last times every kernel family")
    ap.add_argument("--precond", default="ris", choices=["ris", "diag"])
    ap.add_argument("--fp64-steps", type=int, default=2, help="timed steps of the FP64 GPU comparison (0 = skip)")
    ap.add_argument("--fp64-warmup", type=int, default=1, help="untimed FP64 steps before those")
    ap.add_argument("--serve-requests", type=int, default=12,
                    help="single: requests of the short served leg, mixed and FP64 (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serve", action="store_true", help="single: skip the served leg")
    ap.add_argument("--tune-file", default=None,
                    help="single: load GEMM tuning decisions from this file if it exists, save them after")
    ap.add_argument("--no-profile", action="store_true",
                    help="single: no per-kernel event timing in the timed steps (no roofline)")
    ap.add_argument("--graphs", type=int, default=0,
                    help="single: 1 = operator products replayed from captured HIP graphs (timed steps only; "
                         "profiling is off there)")
    ap.add_argument("--cpu-no100", action="store_true",
                    help="also time one oracle step on the no=100 molecule (minutes of CPU time)")
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--m-max", type=int, default=0,
                    help="single: subspace size that triggers a restart (0: the library default)")
    ap.add_argument("--size", default="c2", choices=["c1", "c2"],
                    help="single: molecule of the no=100 (c1) or the no=200 (c2, default) workload")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="MiB of a plain device copy (x * 1.0 on float32) run before timing, so that "
                         "hardware-counter runs can calibrate byte counters against a known size")
    ap.add_argument("--workload", default="single", choices=["single", "batch", "serve", "sweep", "rsh", "molecule"],
                    help="single: one no=200 molecule (default); batch: many molecules in one batched "
                         "solve; serve: a request stream through the server; sweep: ris-model richness "
                         "sweep on the no=100 molecule; rsh: global vs range-separated hybrid; molecule: rid "
                         "vs diagonal on a problem built from a molecule's integrals")
    ap.add_argument("--molecules", type=int, default=64, help="batch: number of molecules")
    ap.add_argument("--sequential", action="store_true", help="batch: also solve the molecules one by one")
    ap.add_argument("--requests", type=int, default=24, help="serve: number of requests")
    ap.add_argument("--no-max", type=int, default=300, help="serve: largest number of occupied orbitals")
    ap.add_argument("--load", type=float, default=0.7, help="serve: arrival rate / saturated rate")
    ap.add_argument("--loads", default=None, help="serve: comma-separated list of loads (overrides --load)")
    ap.add_argument("--fp64", action="store_true", help="serve: also serve the same requests in FP64")
    ap.add_argument("--concurrent", action="store_true",
                    help="single: submit the eigen and the polarizability request of a step together")
    ap.add_argument("--slots", type=int, default=8, help="serve: concurrent requests")
    ap.add_argument("--hbm-budget-gb", type=int, default=96, help="serve: admission budget")
    args = ap.parse_args()
    if args.no_serve:
        args.serve_requests = 0
    if args.workload in ("batch", "serve") or args.serve_requests > 0:
        # many concurrent solve streams: more hardware queues keep them from
        # queueing behind each other (set before the HIP runtime starts)
        os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "sweep":
        return bench_sweep(args)
    if args.workload == "rsh":
        return bench_rsh(args)
    if args.workload == "molecule":
        return bench_molecule(args)

    import numpy as np
    import torch

    import paper_2404_17133_amd as rid
    from synth import config_sizes, make_dipoles, make_problem

    no, nv, naux, nris, seed = config_sizes(args.size)
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
    if args.tune_file and os.path.exists(args.tune_file):
        try:
            log("tuning decisions loaded: %d" % ctx.tune_load(args.tune_file))
        except rid.RidError as e:
            log("tuning file not used: %s" % e)
    prob = rid.Problem.from_synth(ctx, p)
    k = args.k
    roots_per_step = k + pm.shape[0]

    def step(precision):
        if args.concurrent:
            # both requests in one rid_batch_solve: their products share
            # grouped launches and each one's latency-bound phases overlap
            # the other's contractions
            opts = rid.default_opts(args.precond, precision, **({"m_max": args.m_max} if args.m_max > 0 else {}))
            re_, ke = rid.make_request("eigen", opts, k=k, mode="rpa")
            ra, ka = rid.make_request("polarizability", opts, p=pm, omegas=[0.0])
            st_, (e, a) = rid.batch_solve(ctx, [prob, prob], [re_, ra])
            if st_ != 0 or e["status"] != 0 or a["status"] != 0:
                raise RuntimeError("batch status %d: %d %d" % (st_, e["status"], a["status"]))
            return e, a
        kw = {"m_max": args.m_max} if args.m_max > 0 else {}
        kw["graphs"] = 1 if args.graphs else 0
        e = prob.eigen(k, "rpa", args.precond, precision, vectors=False, **kw)
        a = prob.polarizability(pm, [0.0], args.precond, precision, **kw)
        if e["status"] != 0 or a["status"] != 0:
            raise RuntimeError("solve did not converge: %d %d" % (e["status"], a["status"]))
        return e, a

    profiling = not (args.graphs or args.no_profile)  # graph replays are not bracketed by events
    warm_prof = {}
    for w in range(args.warmup):
        if profiling and w == args.warmup - 1:
            # every family timed in the last (untimed) warmup step: the
            # kernel table, and which contraction dominates
            ctx.profile(True)
            ctx.profile_read()
        step("mixed")
        log("warmup step %d done" % w)
    torch.cuda.synchronize()
    if profiling and args.warmup > 0:
        warm_prof = ctx.profile_read()
        ctx.profile(False)
    # the timed steps bracket only the dominant contraction family with
    # events (for its roofline); timing every family would cost ~4 % of the
    # step time
    dom = "exch_w"
    flop_fams = [(k, v) for k, v in warm_prof.items() if v["flops"] > 0]
    if flop_fams:
        dom = max(flop_fams, key=lambda kv: kv[1]["ms"])[0]
    if profiling:
        ctx.profile_only(dom)
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
    prof = ctx.profile_read() if profiling else {}
    ctx.profile(False)
    ctx.profile_only(None)
    value = roots_per_step * args.steps / elapsed

    # dominant kernel: the contraction family (algorithmic FLOPs counted)
    # with the largest summed event time; at this size the exchange W
    # product.  (On smaller molecules the latency-bound dense inner systems
    # can take longer in total, but they have no FLOP roofline.)
    if dom not in prof:
        prof = {dom: {"launches": 1, "ms": 1e-9, "flops": 0.0, "bytes": 0.0}}
    fam, st = dom, prof[dom]
    avg_ms = st["ms"] / st["launches"]
    dtype = "f32" if not fam.startswith("ris_") else "bf16"
    achieved = st["flops"] / st["launches"] / (avg_ms * 1e-3) / 1e12
    traffic = measured_traffic(fam, dtype, args.size)
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
            "workload": "full-TDDFT %d lowest roots + static polarizability (3 RHS), no=%d nv=%d "
                        "(N=%d) Naux=%d Naux_ris=%d, %s preconditioner, mixed precision "
                        "(FP32 outer products, BF16 ris products, FP64 subspace)"
                        % (k, no, nv, no * nv, naux, nris, "rid" if args.precond == "ris" else "diagonal"),
            "precond": args.precond,
            "roots_per_step": roots_per_step,
        },
        "latency_s": {"p50": round(float(np.percentile(lat, 50)), 3),
                      "p99": round(float(np.percentile(lat, 99)), 3)},
        "roofline": roofline,
        "kernels": {kf: {"launches": v["launches"], "ms": round(v["ms"], 1),
                         "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 1)}
                    for kf, v in sorted(warm_prof.items(), key=lambda kv: -kv[1]["ms"])[:12]},
        "kernels_from": "the last warmup step (untimed), every family bracketed by events",
        "solve": {"eigen_iters": last[0]["stats"]["n_iter"], "eigen_n_mv": last[0]["stats"]["n_mv"],
                  "eigen_inner_mv": last[0]["stats"]["n_inner_mv"],
                  "alpha_iters": last[1]["stats"]["n_iter"],
                  "omega": [round(float(x), 10) for x in last[0]["omega"]],
                  # share of the solve time spent in the preconditioner and
                  # the ris initial guess (the paper's cost target: 1-2 %)
                  "precond_time_share": {
                      "eigen": round(last[0]["stats"]["t_precond_ms"] / max(last[0]["stats"]["t_total_ms"], 1e-9), 4),
                      "alpha": round(last[1]["stats"]["t_precond_ms"] / max(last[1]["stats"]["t_total_ms"], 1e-9),
                                     4)},
                  "residual_log10_slope_per_iter": {"eigen": residual_slope(last[0]["stats"]["history"]),
                                                    "alpha": residual_slope(last[1]["stats"]["history"])},
                  # largest residual norm after each outer iteration
                  "residual_history": {"eigen": ["%.3e" % v for v in last[0]["stats"]["history"] if v > 0],
                                       "alpha": ["%.3e" % v for v in last[1]["stats"]["history"] if v > 0]}},
    }
    err = per_root_error(args.size, last[0]["omega"], last[1]["alpha"][0])
    if err is not None:
        out["per_root_err_vs_oracle"] = {"mixed": err}

    if args.fp64_steps > 0:
        # untimed FP64 steps first: the FP64 launch shapes are tuned there,
        # not inside the timed steps
        for w in range(args.fp64_warmup):
            step("fp64")
            torch.cuda.synchronize()
            log("fp64 warmup step %d done" % w)
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
        out["fp64_gpu"] = {"value": round(v64, 4), "unit": "roots/s", "steps": len(lat64),
                           "warmup": args.fp64_warmup,
                           "latency_s": {"p50": round(float(np.percentile(lat64, 50)), 3),
                                         "p99": round(float(np.percentile(lat64, 99)), 3)},
                           "speedup_mixed_vs_fp64": round(value / v64, 3),
                           "max_abs_omega_diff_Ha": dom, "max_rel_alpha_diff": dal}
        err64 = per_root_error(args.size, e64["omega"], a64["alpha"][0])
        if err64 is not None:
            out["per_root_err_vs_oracle"]["fp64"] = err64
    if args.tune_file:
        log("tuning decisions saved: %d" % ctx.tune_save(args.tune_file))
    ctx.close()
    del prob
    if args.serve_requests > 0:
        out["served"] = served_leg(args.serve_requests)
    if not args.no_cpu:
        cb = cpu_baseline(p, n_mv, roots_per_step)
        del p
        torch.cuda.empty_cache()
        cb["solves"] = oracle_solves(args.precond, no100=args.cpu_no100)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
