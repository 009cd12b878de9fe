"""Batched and served solves at the sizes of the batched workload (GPU).

The no=100 molecule whose FP64 oracle results are stored
(tests/golden/oracle_c1.json: 10 full-TDDFT roots and alpha at two
frequencies, tolerance 1e-8) is solved inside a batch of molecules of the
batched workload's recipe (no 63..125, nv = 4 no, Naux = 20 no, k from the
recipe), rid preconditioner, mixed precision.  Its roots and polarizability
must match the oracle, and every member's result must equal the same request
solved alone; the continuous-batching server must give the same results for
the same requests.
"""

import json
import os

import numpy as np
import pytest

from synth import batch_member, config_sizes, make_dipoles, make_problem

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_c1.json")
MEMBERS = [6, 10, 13, 28, 31]  # no = 82, 63, 114, 125, 123 with k = 5, 20, 20, 10, 5


@pytest.fixture(scope="module")
def setup():
    import paper_2404_17133_amd as rid

    g = json.load(open(GOLDEN))
    no, nv, naux, nris, seed = config_sizes("c1")
    ctx = rid.Context(0)
    mols = [make_problem(no, nv, naux, nris, seed=seed, device="cuda:0")]
    ks = [g["k"]]
    for m in MEMBERS:
        d = batch_member(m)
        mols.append(make_problem(d["no"], d["nv"], d["naux"], d["naux_ris"], naux_ris_k=d["naux_ris_k"],
                                 seed=d["seed"], device="cuda:0"))
        ks.append(d["k"])
    probs = [rid.Problem.from_synth(ctx, p) for p in mols]
    dip = make_dipoles(mols[0], 3)
    o = rid.default_opts("ris", "mixed")
    reqs, keep = [], []
    for k in ks:
        r, kp = rid.make_request("eigen", o, k=k, mode="rpa")
        reqs.append(r)
        keep.append(kp)
    r, kp = rid.make_request("polarizability", o, p=dip, omegas=g["alpha_omegas"])
    reqs.append(r)
    keep.append(kp)
    owners = probs + [probs[0]]
    yield rid, ctx, g, probs, dip, reqs, keep, owners
    ctx.close()


def _check_against_oracle(g, res):
    err = np.abs(np.asarray(res[0]["omega"]) - np.array(g["rpa_omega"])).max()
    a = np.asarray(res[-1]["alpha"])
    ref = np.array(g["alpha"])
    rel = np.abs(a - ref).max() / np.abs(ref).max()
    print("no=100 member: max |dOmega| %.2e Ha, alpha max rel %.2e" % (err, rel), flush=True)
    assert err < 1e-6
    assert rel < 1e-5


def test_batch_at_workload_sizes(setup):
    rid, ctx, g, probs, dip, reqs, keep, owners = setup
    print("alone", flush=True)
    alone = [probs[m].eigen(reqs[m].k, "rpa", "ris", "mixed", vectors=False)["omega"] for m in range(len(probs))]
    alone.append(probs[0].polarizability(dip, g["alpha_omegas"], "ris", "mixed")["alpha"])
    print("batch of", len(reqs), "requests", flush=True)
    s, out = rid.batch_solve(ctx, owners, reqs)
    assert s == 0, [o["status"] for o in out]
    _check_against_oracle(g, out)
    worst = 0.0
    for m, o in enumerate(out):
        v = o["omega"] if "omega" in o else o["alpha"]
        scale = 1.0 if m < len(probs) else np.abs(alone[m]).max()
        worst = max(worst, np.abs(np.asarray(v) - np.asarray(alone[m])).max() / scale)
    print("largest batch-vs-alone difference", worst, flush=True)
    assert worst < 1e-9


def test_server_at_workload_sizes(setup):
    rid, ctx, g, probs, dip, reqs, keep, owners = setup
    s, ref = rid.batch_solve(ctx, owners, reqs)
    assert s == 0
    srv = rid.Server(ctx, hbm_budget_bytes=96 << 30, max_slots=4)
    tickets = [srv.submit(owners[m], reqs[m], keep=keep[m]) for m in range(len(reqs))]
    res = [srv.wait(t, 300000) for t in tickets]
    srv.close()
    assert all(r["status"] == 0 for r in res), [r["status"] for r in res]
    _check_against_oracle(g, res)
    for m, (a, b) in enumerate(zip(res, ref)):
        va = a["omega"] if "omega" in a else a["alpha"]
        vb = b["omega"] if "omega" in b else b["alpha"]
        np.testing.assert_allclose(va, vb, rtol=0, atol=1e-9 * max(1.0, np.abs(vb).max()))
