"""Operator products through the C ABI against the FP64 oracle (GPU).

Shapes span several GEMM tiles with ragged edges (sizes that are not
multiples of the 16/32/64/128 tile sizes, a prime auxiliary count) and an
exchange window that cuts both orbital ranges.

Tolerances, relative to the largest magnitude of the two-electron part
(y - de x) of the exact product:
* FP64: 1e-12 (reordered sums of ~1e4 terms at unit round-off 1.1e-16);
* FP32 operands, FP32 accumulation within a split, FP64 across splits:
  2e-5 (unit round-off 6e-8 times a few hundred for the operand rounding and
  the within-split sums of up to ~1e4 terms);
* BF16 operands (8 significant bits, round-off 3.9e-3), FP32 accumulation:
  3e-2.
"""

import numpy as np
import pytest
import torch

from oracle import operators as ops
from oracle.operators import OracleProblem
from synth import make_block, make_problem

pytestmark = pytest.mark.gpu

CASES = [
    # no, nv, naux, naux_ris, nk, t_cut, nvec
    (7, 29, 37, 11, 3, 1.0, 5),      # ragged everywhere, window cuts i and a
    (20, 80, 400, 90, 10, None, 13),  # config-0 shapes
    (16, 64, 128, 32, 4, float("inf"), 1),  # aligned sizes, no window
    (33, 131, 97, 23, 5, 1.3, 19),   # more tiles, odd strides
]


def _setup(no, nv, naux, nris, nk, tcut, seed=5):
    import paper_2404_17133_amd as rid

    kw = {} if tcut is None else {"t_cut": tcut}
    if nris == 0:
        kw["ris_source"] = "none"
    p = make_problem(no, nv, naux, nris, naux_ris_k=nk or None, seed=seed, **kw)
    op = OracleProblem.from_arrays(p.numpy())
    ctx = rid.Context(0)
    prob = rid.Problem.from_synth(ctx, p.to("cuda:0"))
    return p, op, ctx, prob


def _rel(got, ref, de_x):
    scale = np.abs(ref - de_x).max()
    return np.abs(got - ref).max() / scale


@pytest.mark.parametrize("case", CASES)
def test_outer_operator_fp64_fp32(case):
    no, nv, naux, nris, nk, tcut, nvec = case
    p, op, ctx, prob = _setup(no, nv, naux, nris, nk, tcut)
    print("case", case, flush=True)
    x = make_block(3, 1, nvec, op.n)
    xc = x.numpy().T
    de_x = op.delta_eps()[:, None] * xc
    ref_a = ops.apply_a(op, xc)
    ref_p, ref_m = ops.apply_apb_amb(op, xc)
    xd = x.to("cuda:0").contiguous()
    errs = {}
    try:
        for dt, tol in (("f64", 1e-12), ("f32", 2e-5)):
            ya = prob.apply("A", xd, dt).cpu().numpy().T
            yp, ym = prob.apply("APB_AMB", xd, dt)
            yp, ym = yp.cpu().numpy().T, ym.cpu().numpy().T
            errs[dt] = (_rel(ya, ref_a, de_x), _rel(yp, ref_p, de_x), _rel(ym, ref_m, de_x), tol)
    finally:
        ctx.close()
    print("relative errors (A, A+B, A-B, tol):", errs, flush=True)
    for dt, e in errs.items():
        assert max(e[:3]) < e[3], (dt, e)


@pytest.mark.parametrize("case", CASES)
def test_ris_operator_fp64_bf16(case):
    no, nv, naux, nris, nk, tcut, nvec = case
    p, op, ctx, prob = _setup(no, nv, naux, nris, nk, tcut)
    print("case", case, flush=True)
    i0, na = prob.window()
    assert (i0, na) == op.active_ranges()
    x = make_block(4, 2, nvec, op.n)
    xc = x.numpy().T
    de_x = op.delta_eps()[:, None] * xc
    ref_t = ops.apply_t(op, xc)
    ref_p, ref_m = ops.apply_tpm(op, xc)
    xd = x.to("cuda:0").contiguous()
    errs = {}
    try:
        for dt, tol in (("f64", 1e-12), ("bf16", 3e-2)):
            yt = prob.apply("T", xd, dt).cpu().numpy().T
            yp, ym = prob.apply("TPM", xd, dt)
            yp, ym = yp.cpu().numpy().T, ym.cpu().numpy().T
            errs[dt] = (_rel(yt, ref_t, de_x), _rel(yp, ref_p, de_x), _rel(ym, ref_m, de_x), tol)
    finally:
        ctx.close()
    print("relative errors (T, T+, T-, tol):", errs, flush=True)
    for dt, e in errs.items():
        assert max(e[:3]) < e[3], (dt, e)


def test_operator_error_paths():
    import paper_2404_17133_amd as rid

    p, op, ctx, prob = _setup(5, 12, 17, 0, 0, None)
    x = make_block(1, 1, 2, op.n).to("cuda:0")
    with pytest.raises(rid.RidError) as e:
        prob.apply("T", x, "f64")  # no ris tensor
    assert e.value.status == -1
    with pytest.raises(rid.RidError) as e:
        prob.apply("A", x, "bf16")  # BF16 only for the ris model
    assert e.value.status == -3
    # empty block is a no-op
    y = prob.apply("A", x[:0].contiguous(), "f64")
    assert y.shape == (0, op.n)
    prob.close()
    ctx.close()
