"""Variants of the ris model on the config-0 molecule (GPU): J and K on the
s rows only, J and K on all rows, and the exact model T = A (ris tensor =
full tensor, no noise, no window).  Every preconditioner reaches the
oracle's roots (Sec. 2.1: the preconditioner changes the path, not the
answer); with T = A the outer solve needs only a few iterations (Sec. 2.1:
the closer T is to A, the fewer iterations)."""

import numpy as np
import pytest

from oracle import OracleProblem, eigen_rpa, eigen_tda
from synth import config_sizes, make_problem

pytestmark = pytest.mark.gpu

VARIANTS = [
    ("ss", dict(naux_ris=10, naux_ris_k=10)),
    ("dd", dict(naux_ris=90, naux_ris_k=90)),
    ("exact", dict(naux_ris=400, naux_ris_k=400, ris_source="full", noise=0.0, t_cut=float("inf"))),
]


@pytest.fixture(scope="module")
def reference():
    no, nv, naux, nris, seed = config_sizes("c0")
    p = make_problem(no, nv, naux, nris, seed=seed)
    op = OracleProblem.from_arrays(p.numpy())
    return eigen_tda(op, 5, "diag", tol=1e-8).omega, eigen_rpa(op, 5, "diag", tol=1e-8).omega


@pytest.mark.parametrize("name,kw", VARIANTS, ids=[v[0] for v in VARIANTS])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_variant_reaches_oracle_roots(reference, name, kw, precision):
    import paper_2404_17133_amd as rid

    no, nv, naux, _, seed = config_sizes("c0")
    kw = dict(kw)
    nris = kw.pop("naux_ris")
    p = make_problem(no, nv, naux, nris, seed=seed, device="cuda:0", **kw)
    ctx = rid.Context(0)
    prob = rid.Problem.from_synth(ctx, p)
    print("variant", name, precision, flush=True)
    tda = prob.eigen(5, "tda", "ris", precision, vectors=False)
    rpa = prob.eigen(5, "rpa", "ris", precision, vectors=False)
    assert tda["status"] == 0 and rpa["status"] == 0
    assert np.abs(tda["omega"] - reference[0]).max() < 1e-6
    assert np.abs(rpa["omega"] - reference[1]).max() < 1e-6
    if name == "exact":
        assert tda["stats"]["n_iter"] <= 4 and rpa["stats"]["n_iter"] <= 4, (tda["stats"], rpa["stats"])
    ctx.close()
