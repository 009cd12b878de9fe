"""Write oracle results for the GPU parity tests at the no=20, no=100 and
no=200 sizes (tests/golden/oracle_c0.json, oracle_c1.json, oracle_c2.json).

Calls only oracle/ and synth/: the FP64 CPU Davidson (Sec. 2.1; Eq. TDA and
Eq. Casida) and the polarizability solve (Eq. TDDFT_polar), run to a
residual tolerance of 1e-8 so that they serve as the reference the GPU path
must match within 1e-6 Ha (roots) and 1e-5 relative (alpha).

At no=200 (N = 160 000, 27 GB of FP64 tensors, hours of CPU time) only the
workload the benchmark times is stored: the 10 lowest full-TDDFT roots and
the static polarizability of the 3 dipole right-hand sides.

Usage: python tests/golden/make_golden.py c0 c1 c2
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import OracleProblem, eigen_rpa, eigen_tda, polarizability  # noqa: E402
from synth import config_sizes, make_dipoles, make_problem  # noqa: E402

K = {"c0": 5, "c1": 10, "c2": 10}
OMEGAS = [0.0, 0.0569542]  # static and 800 nm (Sec. 4.2)


def run(name):
    no, nv, naux, nris, seed = config_sizes(name)
    t0 = time.time()
    if name == "c2":
        return run_c2(no, nv, naux, seed, t0)
    p = make_problem(no, nv, naux, nris, seed=seed)
    op = OracleProblem.from_arrays(p.numpy())
    pm = make_dipoles(p, 3).numpy().T
    k = K[name]
    out = {"config": name, "sizes": dict(no=no, nv=nv, naux=naux, naux_ris=nris, seed=seed), "k": k,
           "tol": 1e-8, "source": "tests/golden/make_golden.py (oracle/, FP64 CPU)"}
    r = eigen_tda(op, k, "diag", tol=1e-8, max_iter=200)
    out["tda_omega"] = r.omega.tolist()
    out["tda_status"] = r.status
    print(name, "tda", r.status, r.n_iter, time.time() - t0, flush=True)
    r = eigen_rpa(op, k, "diag", tol=1e-8, max_iter=200)
    out["rpa_omega"] = r.omega.tolist()
    out["rpa_status"] = r.status
    print(name, "rpa", r.status, r.n_iter, time.time() - t0, flush=True)
    a = polarizability(op, pm, OMEGAS, "diag", tol=1e-8, max_iter=200)
    out["alpha_omegas"] = OMEGAS
    out["alpha"] = a.alpha.tolist()
    out["alpha_status"] = a.status
    print(name, "alpha", a.status, a.n_iter, time.time() - t0, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_%s.json" % name)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


def run_c2(no, nv, naux, seed, t0):
    # the diagonal preconditioner needs no ris tensor: leave it out (6 GB)
    p = make_problem(no, nv, naux, 0, seed=seed, ris_source="none")
    op = OracleProblem.from_arrays(p.numpy())
    pm = make_dipoles(p, 3).numpy().T
    print("c2 inputs", time.time() - t0, flush=True)
    out = {"config": "c2", "sizes": dict(no=no, nv=nv, naux=naux, seed=seed), "k": 10,
           "tol": 1e-8, "source": "tests/golden/make_golden.py (oracle/, FP64 CPU)"}
    r = eigen_rpa(op, 10, "diag", tol=1e-8, max_iter=200)
    out["rpa_omega"] = r.omega.tolist()
    out["rpa_resid"] = r.resid.tolist()
    out["rpa_status"] = r.status
    out["rpa_n_iter"] = r.n_iter
    out["rpa_n_mv"] = r.n_mv
    print("c2 rpa", r.status, r.n_iter, r.n_mv, time.time() - t0, flush=True)
    a = polarizability(op, pm, [0.0], "diag", tol=1e-8, max_iter=200)
    out["alpha_omegas"] = [0.0]
    out["alpha"] = a.alpha.tolist()
    out["alpha_status"] = a.status
    out["alpha_n_iter"] = a.n_iter
    print("c2 alpha", a.status, a.n_iter, time.time() - t0, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_c2.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    for name in sys.argv[1:]:
        run(name)
