"""The allocation-free operator product (rid_apply_operator_noalloc) against
rid_apply_operator and the FP64 oracle (GPU).

Every intermediate of the product lives in the library's fixed device region
of RID_NOALLOC_SCRATCH_BYTES per GPU.  Two calls in a row -- a larger block,
then a smaller one, so that the second reads a region holding the first
call's data -- must each match the allocating entry point and the oracle to
the same tolerances as the operator parity tests (relative to the largest
two-electron part |y - de x|): FP64 1e-12, FP32 2e-5, BF16 3e-2.  Neither
call may take device memory from the allocator.
"""

import ctypes

import numpy as np
import pytest
import torch

from oracle import operators as ops
from oracle.operators import OracleProblem
from synth import make_block, make_problem

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5, "bf16": 3e-2}
# (no, nv, naux, naux_ris, nk, t_cut): the no=20 shapes and a ragged case
# whose exchange window cuts both orbital ranges
CASES = [(20, 80, 400, 90, 10, None), (7, 29, 37, 11, 3, 1.0)]


def _outputs(op, x):
    pair = op in ("APB_AMB", "TPM")
    return torch.empty_like(x), (torch.empty_like(x) if pair else None)


def _noalloc(prob, op, dt, x, out=None):
    """Call the allocation-free entry point; outputs are made here unless
    given (give them when device allocations are being counted)."""
    from paper_2404_17133_amd import _binding as B
    from paper_2404_17133_amd.solver import _DTYPES, _OPS

    y, y2 = out if out is not None else _outputs(op, x)
    pair = y2 is not None
    s = B.lib.rid_apply_operator_noalloc(prob.handle, _OPS[op], _DTYPES[dt], x.shape[0], ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(y.data_ptr()),
                                         ctypes.c_void_p(y2.data_ptr()) if pair else None)
    return s, ((y, y2) if pair else y)


def _rel(got, ref, de_x):
    return np.abs(got - ref).max() / np.abs(ref - de_x).max()


def _setup(case):
    import paper_2404_17133_amd as rid

    no, nv, naux, nris, nk, tcut = case
    kw = {} if tcut is None else {"t_cut": tcut}
    p = make_problem(no, nv, naux, nris, naux_ris_k=nk, seed=5, **kw)
    op = OracleProblem.from_arrays(p.numpy())
    ctx = rid.Context(0)
    prob = rid.Problem.from_synth(ctx, p.to("cuda:0"))
    return op, ctx, prob


def _oracle(op, name, xc):
    if name == "A":
        return (ops.apply_a(op, xc),)
    if name == "APB_AMB":
        return ops.apply_apb_amb(op, xc)
    if name == "T":
        return (ops.apply_t(op, xc),)
    return ops.apply_tpm(op, xc)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("opname,dt", [("A", "f64"), ("APB_AMB", "f64"), ("A", "f32"), ("APB_AMB", "f32"),
                                       ("T", "f64"), ("TPM", "f64"), ("T", "bf16"), ("TPM", "bf16")])
def test_noalloc_matches_allocating_product_twice(case, opname, dt):
    from paper_2404_17133_amd import _binding as B

    op, ctx, prob = _setup(case)
    print("noalloc", case, opname, dt, flush=True)
    try:
        # the allocating entry point makes the tensor copies of this precision
        for nvec, seed in ((24, 1), (5, 2)):
            x = make_block(seed, 7, nvec, op.n)
            xc = x.numpy().T
            de_x = op.delta_eps()[:, None] * xc
            refs = _oracle(op, opname, xc)
            xd = x.to("cuda:0").contiguous()
            ya = prob.apply(opname, xd, dt)
            ya = ya if isinstance(ya, tuple) else (ya,)
            out = _outputs(opname, xd)
            torch.cuda.synchronize()
            before = torch.cuda.memory_allocated()
            s, yn = _noalloc(prob, opname, dt, xd, out)
            torch.cuda.synchronize()
            assert s == B.RID_OK, (s, ctx.last_error())
            assert torch.cuda.memory_allocated() == before  # nothing taken from the allocator
            yn = yn if isinstance(yn, tuple) else (yn,)
            for a, n, r in zip(ya, yn, refs):
                a, n = a.cpu().numpy().T, n.cpu().numpy().T
                e_alloc, e_fixed, e_pair = _rel(a, r, de_x), _rel(n, r, de_x), _rel(n, a, de_x)
                print("  nvec %d: oracle err alloc %.2e fixed %.2e; fixed vs alloc %.2e" % (nvec, e_alloc, e_fixed,
                                                                                              e_pair), flush=True)
                assert e_fixed < TOL[dt] and e_pair < TOL[dt]
            del ya, yn, out  # so that the next call's allocation count starts clean
    finally:
        ctx.close()


def test_noalloc_refuses_missing_copies_and_oversized_products():
    from paper_2404_17133_amd import _binding as B

    op, ctx, prob = _setup(CASES[0])
    try:
        x = make_block(3, 7, 4, op.n).to("cuda:0").contiguous()
        # no FP32 product has run on this problem: its FP32 copies do not exist
        s, _ = _noalloc(prob, "A", "f32", x)
        assert s == B.RID_ERR_INVALID_ARG
        assert "copies" in ctx.last_error()
        prob.apply("A", x, "f64")  # makes the FP64 copies
        big = make_block(4, 7, 3000, op.n).to("cuda:0").contiguous()  # intermediates far above 128 MiB
        mark = torch.full_like(big, 7.0)
        from paper_2404_17133_amd.solver import _DTYPES, _OPS

        s = B.lib.rid_apply_operator_noalloc(prob.handle, _OPS["A"], _DTYPES["f64"], big.shape[0],
                                             ctypes.c_void_p(big.data_ptr()), ctypes.c_void_p(mark.data_ptr()), None)
        torch.cuda.synchronize()
        assert s == B.RID_ERR_SHAPE
        assert "scratch" in ctx.last_error()
        assert torch.equal(mark, torch.full_like(big, 7.0))  # output untouched
        del big, mark
        torch.cuda.synchronize()
        # the region still serves a product that fits
        out = _outputs("A", x)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        s, y = _noalloc(prob, "A", "f64", x, out)
        torch.cuda.synchronize()
        assert s == B.RID_OK
        assert torch.cuda.memory_allocated() == before
        ref = ops.apply_a(op, x.cpu().numpy().T)
        de_x = op.delta_eps()[:, None] * x.cpu().numpy().T
        assert _rel(y.cpu().numpy().T, ref, de_x) < 1e-12
    finally:
        ctx.close()
