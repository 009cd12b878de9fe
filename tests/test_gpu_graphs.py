"""Operator products replayed from captured HIP graphs (GPU).

With rid_solve_opts.graphs = 1 a solve that has the device to itself runs
each product shape once directly, then captures it as a graph and replays
it whenever the shape recurs -- also in later solves on the same problem.
Every replay sits between the solver's own direct work (projections,
orthonormalisation, small dense problems, read-backs), so a replay that
went wrong would change the iterates.  The same kernels run with the same
plans, so the roots, vectors and iteration counts must be bit-identical to
the direct path, solve after solve, and also after the problem's scratch
has been reallocated by a larger block (the graphs are captured again).
"""

import numpy as np
import pytest

from synth import make_dipoles, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c0():
    import paper_2404_17133_amd as rid

    p = make_problem(20, 80, 400, 90, seed=0).to("cuda:0")
    ctx = rid.Context(0)
    prob = rid.Problem.from_synth(ctx, p)
    yield p, ctx, prob
    ctx.close()


@pytest.mark.parametrize("mode,precond,precision", [("rpa", "ris", "mixed"), ("tda", "diag", "fp64"),
                                                     ("rpa", "diag", "fp64"), ("tda", "ris", "mixed")])
def test_graph_replays_equal_direct_products(c0, mode, precond, precision):
    p, ctx, prob = c0
    print("graphs", mode, precond, precision, flush=True)
    ref = prob.eigen(5, mode, precond, precision, graphs=0)
    assert ref["status"] == 0
    for rep in range(3):  # capture in the first solve, replays in all
        out = prob.eigen(5, mode, precond, precision, graphs=1)
        assert out["status"] == 0
        assert np.array_equal(out["omega"], ref["omega"]), (rep, out["omega"] - ref["omega"])
        assert out["stats"]["n_iter"] == ref["stats"]["n_iter"] and out["stats"]["n_mv"] == ref["stats"]["n_mv"]
        assert bool((out["x"] == ref["x"]).all())


def test_graphs_recaptured_after_scratch_grows(c0):
    p, ctx, prob = c0
    small = prob.eigen(4, "rpa", "diag", "fp64", graphs=0)
    big = prob.eigen(12, "rpa", "diag", "fp64", graphs=0)
    for k, ref in ((4, small), (12, big), (4, small), (12, big)):
        out = prob.eigen(k, "rpa", "diag", "fp64", graphs=1)
        assert np.array_equal(out["omega"], ref["omega"]), k


def test_graph_replays_in_polarizability(c0):
    p, ctx, prob = c0
    pm = make_dipoles(p, 3).contiguous()
    ref = prob.polarizability(pm, [0.0, 0.1], "ris", "mixed", graphs=0)
    for _ in range(2):
        out = prob.polarizability(pm, [0.0, 0.1], "ris", "mixed", graphs=1)
        assert np.array_equal(out["alpha"], ref["alpha"])


def test_graphs_flag_is_validated(c0):
    import paper_2404_17133_amd as rid

    p, ctx, prob = c0
    with pytest.raises(rid.RidError) as e:
        prob.eigen(3, "tda", "diag", "fp64", graphs=2)
    assert e.value.status == -1
