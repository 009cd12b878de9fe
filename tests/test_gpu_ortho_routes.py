"""Both orthonormalisation routes (GPU).

New directions that stay well apart are orthonormalised within their block
by two Cholesky-QR passes; a block with a (nearly) dependent direction takes
modified Gram-Schmidt, which drops it (below 1e-8 of its length).  A start
subspace that repeats a vector forces the second route; the roots must be
the oracle's either way, and the solve statistics report the routes taken.
"""

import numpy as np
import pytest
import torch

from oracle import OracleProblem, eigen_tda
from synth import make_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_dependent_start_block_takes_gram_schmidt(precision):
    import paper_2404_17133_amd as rid

    p = make_problem(20, 80, 400, 90, seed=0)
    ref = eigen_tda(OracleProblem.from_arrays(p.numpy()), 5, "diag", tol=1e-8).omega
    ctx = rid.Context(0)
    prob = rid.Problem.from_synth(ctx, p.to("cuda:0"))
    print("ortho routes", precision, flush=True)
    plain = prob.eigen(5, "tda", "diag", precision)
    assert plain["status"] == 0
    assert plain["stats"]["n_blocks_cholqr"] > 0, plain["stats"]
    x = plain["x"]
    # the first two start vectors are the same direction (scaled): one is dropped
    guess = torch.cat([x[:1], 2.0 * x[:1], x[1:3]]).contiguous()
    out = prob.eigen(5, "tda", "diag", precision, guess=guess)
    assert out["status"] == 0
    np.testing.assert_allclose(out["omega"], ref, rtol=0, atol=1e-6)
    assert out["stats"]["n_blocks_mgs"] >= 1, out["stats"]
    xo = out["x"].cpu().numpy()
    np.testing.assert_allclose(xo @ xo.T, np.eye(5), atol=1e-8)
    ctx.close()
