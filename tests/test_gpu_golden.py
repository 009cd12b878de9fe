"""GPU parity at the config-1 size (no=100, nv=400, Naux=2000, Naux_ris=450)
against stored oracle results (tests/golden/oracle_c1.json, written by
tests/golden/make_golden.py, which calls only oracle/ and synth/).

Roots must agree within 1e-6 Ha and polarizabilities within 1e-5 relative,
for the FP64 and the mixed-precision path and for both preconditioners.
"""

import json
import os

import numpy as np
import pytest

from synth import config_sizes, make_dipoles, make_problem

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_c1.json")


@pytest.fixture(scope="module")
def c1():
    import paper_2404_17133_amd as rid

    with open(GOLDEN) as f:
        g = json.load(f)
    no, nv, naux, nris, seed = config_sizes("c1")
    assert g["sizes"] == dict(no=no, nv=nv, naux=naux, naux_ris=nris, seed=seed)
    p = make_problem(no, nv, naux, nris, seed=seed, device="cuda:0")
    ctx = rid.Context(0)
    prob = rid.Problem.from_synth(ctx, p)
    yield g, p, prob
    ctx.close()


CASES = [("diag", "fp64"), ("ris", "fp64"), ("ris", "mixed"), ("diag", "mixed")]


@pytest.mark.parametrize("precond,precision", CASES)
def test_c1_tda_roots(c1, precond, precision):
    g, p, prob = c1
    print("c1 tda", precond, precision, flush=True)
    out = prob.eigen(g["k"], "tda", precond, precision, vectors=False)
    assert out["status"] == 0
    err = np.abs(out["omega"] - np.array(g["tda_omega"])).max()
    print("max |omega - oracle| =", err, flush=True)
    assert err < 1e-6


@pytest.mark.parametrize("precond,precision", CASES)
def test_c1_rpa_roots(c1, precond, precision):
    g, p, prob = c1
    print("c1 rpa", precond, precision, flush=True)
    out = prob.eigen(g["k"], "rpa", precond, precision, vectors=False)
    assert out["status"] == 0
    err = np.abs(out["omega"] - np.array(g["rpa_omega"])).max()
    print("max |omega - oracle| =", err, flush=True)
    assert err < 1e-6


@pytest.mark.parametrize("precond,precision", CASES)
def test_c1_polarizability(c1, precond, precision):
    g, p, prob = c1
    print("c1 alpha", precond, precision, flush=True)
    pm = make_dipoles(p, 3)
    out = prob.polarizability(pm, g["alpha_omegas"], precond, precision)
    assert out["status"] == 0
    ref = np.array(g["alpha"])
    rel = np.abs(out["alpha"] - ref).max() / np.abs(ref).max()
    print("relative alpha error =", rel, flush=True)
    assert rel < 1e-5
