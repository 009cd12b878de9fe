"""Degenerate and edge cases of the GPU solvers against the oracle (GPU).

* zero coupling (B = 0): A = A+B = A-B = diag(de), so the roots are the
  smallest orbital-energy differences and the diagonal preconditioner
  converges at the first iteration;
* one occupied orbital, and pure Coulomb coupling (a_x = 0) through a
  single auxiliary function;
* every root of a tiny problem (k = N), against dense diagonalisation;
* prime-sized (ragged) dimensions in both precisions.
"""

import numpy as np
import pytest

from oracle import OracleProblem, eigen_rpa, eigen_tda
from oracle import operators as ops
from synth import make_problem

pytestmark = pytest.mark.gpu


def _gpu(p):
    import paper_2404_17133_amd as rid

    ctx = rid.Context(0)
    return ctx, rid.Problem.from_synth(ctx, p.to("cuda:0"))


def _dense_roots(op):
    eye = np.eye(op.n)
    a = ops.apply_a(op, eye)
    apb, amb = ops.apply_apb_amb(op, eye)
    tda = np.linalg.eigvalsh(0.5 * (a + a.T))
    lam, u = np.linalg.eigh(amb)
    s = u @ np.diag(np.sqrt(lam)) @ u.T
    rpa = np.sqrt(np.linalg.eigvalsh(s @ apb @ s))
    return tda, rpa


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_coupling(precision):
    p = make_problem(6, 20, 40, 9, seed=4, coupling=0.0)
    de = np.sort((p.eps_vir.numpy()[None, :] - p.eps_occ.numpy()[:, None]).ravel())
    ctx, prob = _gpu(p)
    print("zero coupling", precision, flush=True)
    for mode in ("tda", "rpa"):
        out = prob.eigen(5, mode, "diag", precision, vectors=False)
        assert out["status"] == 0
        np.testing.assert_allclose(out["omega"], de[:5], rtol=0, atol=1e-12)
        assert out["stats"]["n_iter"] == 1
    ctx.close()


@pytest.mark.parametrize("case", ["one_occupied", "coulomb_rank_one"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_special_cases(case, precision):
    if case == "one_occupied":
        p = make_problem(1, 24, 30, 6, seed=7)
    else:
        p = make_problem(5, 12, 1, 1, seed=8, a_x=0.0)
    op = OracleProblem.from_arrays(p.numpy())
    tda_ref, rpa_ref = _dense_roots(op)
    ctx, prob = _gpu(p)
    print(case, precision, flush=True)
    for mode, ref in (("tda", tda_ref), ("rpa", rpa_ref)):
        for precond in ("diag", "ris"):
            out = prob.eigen(4, mode, precond, precision, vectors=False)
            assert out["status"] == 0, (mode, precond)
            np.testing.assert_allclose(out["omega"], ref[:4], rtol=0, atol=1e-6)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_all_roots_of_a_tiny_problem(precision):
    p = make_problem(2, 3, 8, 3, seed=11)
    op = OracleProblem.from_arrays(p.numpy())
    tda_ref, rpa_ref = _dense_roots(op)
    ctx, prob = _gpu(p)
    print("k = N", precision, flush=True)
    tda = prob.eigen(6, "tda", "diag", precision)
    rpa = prob.eigen(6, "rpa", "diag", precision)
    assert tda["status"] == 0 and rpa["status"] == 0
    np.testing.assert_allclose(tda["omega"], tda_ref, rtol=0, atol=1e-6)
    np.testing.assert_allclose(rpa["omega"], rpa_ref, rtol=0, atol=1e-6)
    x = tda["x"].cpu().numpy()
    np.testing.assert_allclose(x @ x.T, np.eye(6), atol=1e-8)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_prime_sizes(precision):
    p = make_problem(7, 31, 53, 13, seed=12)
    op = OracleProblem.from_arrays(p.numpy())
    ref_t = eigen_tda(op, 3, "diag", tol=1e-8).omega
    ref_r = eigen_rpa(op, 3, "diag", tol=1e-8).omega
    ctx, prob = _gpu(p)
    print("prime sizes", precision, flush=True)
    for mode, ref in (("tda", ref_t), ("rpa", ref_r)):
        out = prob.eigen(3, mode, "ris", precision, vectors=False)
        assert out["status"] == 0
        np.testing.assert_allclose(out["omega"], ref, rtol=0, atol=1e-6)
    ctx.close()
