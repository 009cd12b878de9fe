"""Pins of the oracle's response operators (CPU only).

The factored products of the oracle are checked against routes that share no
arithmetic with them: Hessians written element by element from explicit
four-index integrals (Eq. hessian, Eq. pqrs_approx), closed forms of special
cases, and symmetry.  A test at the end plants plausible mistakes in the oracle
and checks that these pins catch each one.
"""

import numpy as np
import pytest

from oracle import operators as ops
from oracle.operators import OracleProblem
from synth import make_problem


def tiny(no=3, nv=4, naux=5, naux_ris=4, nk=2, seed=7, a_x=0.25, t_cut=None):
    kw = {} if t_cut is None else {"t_cut": t_cut}
    naux_ris = min(naux_ris, naux)
    p = make_problem(no, nv, naux, naux_ris, naux_ris_k=min(nk, naux_ris), a_x=a_x, seed=seed, **kw)
    return OracleProblem.from_arrays(p.numpy())


def dense_from_eri(op: OracleProblem, ris=False):
    if ris:
        b = ops.full_three_index(op.bris_ia[:], op.bris_ij, op.bris_ab)
        bk = ops.full_three_index(op.bris_ia[:op.naux_ris_k], op.bris_ij[:op.naux_ris_k],
                                  op.bris_ab[:op.naux_ris_k])
        eri_j = ops.dense_eri(b)
        eri_k = ops.dense_eri(bk)
        i0, na = op.active_ranges()
        occ = np.arange(op.no) >= i0
        vir = np.arange(op.nv) < na
        # Coulomb from all rows, exchange from the leading rows on the active block
        a_j, b_j = ops.dense_hessians(op.eps_occ, op.eps_vir, eri_j, 0.0)
        a_jk, b_jk = ops.dense_hessians(op.eps_occ, op.eps_vir, eri_k, op.a_x, occ, vir)
        a_k0, b_k0 = ops.dense_hessians(op.eps_occ, op.eps_vir, eri_k, 0.0)
        return a_j + (a_jk - a_k0), b_j + (b_jk - b_k0)
    eri = ops.dense_eri(ops.full_three_index(op.b_ia, op.b_ij, op.b_ab))
    return ops.dense_hessians(op.eps_occ, op.eps_vir, eri, op.a_x)


def test_apply_a_matches_eri_definition():
    op = tiny()
    amat, _ = dense_from_eri(op)
    x = np.random.default_rng(1).standard_normal((op.n, 3))
    np.testing.assert_allclose(ops.apply_a(op, x), amat @ x, rtol=0, atol=1e-13)


def test_apb_amb_match_eri_definition():
    op = tiny(no=2, nv=5, naux=3, naux_ris=3)
    amat, bmat = dense_from_eri(op)
    x = np.random.default_rng(2).standard_normal((op.n, 4))
    apb, amb = ops.apply_apb_amb(op, x)
    np.testing.assert_allclose(apb, (amat + bmat) @ x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(amb, (amat - bmat) @ x, rtol=0, atol=1e-13)


def test_ris_operator_matches_eri_definition_with_cutoff():
    # t_cut small enough that some occupied and some virtual orbitals are inactive
    op = tiny(no=4, nv=5, naux=6, naux_ris=5, nk=2, t_cut=1.0, seed=11)
    i0, na = op.active_ranges()
    assert 0 < i0 < op.no and 0 < na < op.nv
    tmat, tb = dense_from_eri(op, ris=True)
    x = np.random.default_rng(3).standard_normal((op.n, 3))
    np.testing.assert_allclose(ops.apply_t(op, x), tmat @ x, rtol=0, atol=1e-13)
    tp, tm = ops.apply_tpm(op, x)
    np.testing.assert_allclose(tp, (tmat + tb) @ x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(tm, (tmat - tb) @ x, rtol=0, atol=1e-13)


def test_operators_are_symmetric():
    op = tiny(no=4, nv=6, naux=7, naux_ris=5, nk=2, t_cut=1.2, seed=5)
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal((op.n, 1)), rng.standard_normal((op.n, 1))
    for f in (lambda x: ops.apply_a(op, x), lambda x: ops.apply_t(op, x),
              lambda x: ops.apply_apb_amb(op, x)[0], lambda x: ops.apply_apb_amb(op, x)[1],
              lambda x: ops.apply_tpm(op, x)[0], lambda x: ops.apply_tpm(op, x)[1]):
        assert abs((u.T @ f(v)).item() - (v.T @ f(u)).item()) < 1e-12


def test_zero_tensor_gives_orbital_energy_differences():
    op = tiny()
    op.b_ia[:] = 0.0
    op.b_ij[:] = 0.0
    op.b_ab[:] = 0.0
    x = np.eye(op.n)
    de = (op.eps_vir[None, :] - op.eps_occ[:, None]).reshape(-1)
    np.testing.assert_array_equal(ops.apply_a(op, x), np.diag(de))


def _secular_roots(d, b, k):
    """k lowest roots of 1 + 2 sum b^2/(d - lam) = 0 by bisection (pure Python)."""
    order = sorted(range(len(d)), key=lambda t: d[t])
    ds = [d[t] for t in order]
    f = lambda lam: 1.0 + 2.0 * sum(bb * bb / (dd - lam) for dd, bb in zip(d, b))
    roots = []
    for j in range(k):
        lo, hi = ds[j], ds[j + 1]
        lo_, hi_ = lo + 1e-15 * (1 + abs(lo)), hi - 1e-15 * (1 + abs(hi))
        for _ in range(200):
            mid = 0.5 * (lo_ + hi_)
            if f(mid) < 0.0:
                lo_ = mid
            else:
                hi_ = mid
        roots.append(0.5 * (lo_ + hi_))
    return roots


def test_rank_one_coulomb_secular_equation():
    # a_x = 0 and one auxiliary function: A = diag(de) + 2 b b^T
    op = tiny(no=3, nv=5, naux=1, a_x=0.0, seed=21)
    de = op.delta_eps()
    b = op.b_ia.reshape(-1)
    lam = np.linalg.eigvalsh(ops.apply_a(op, np.eye(op.n)))
    ref = _secular_roots(list(de), list(b), 4)
    np.testing.assert_allclose(lam[:4], ref, rtol=0, atol=1e-12)


def test_single_occupied_exchange_closed_form():
    # no = 1: (W x)_{0a} = sum_P B^P_00 sum_b x_0b B^P_ba
    op = tiny(no=1, nv=6, naux=4, seed=3)
    x = np.random.default_rng(5).standard_normal((op.n, 1))
    ref = np.zeros(op.nv)
    for a in range(op.nv):
        for p in range(op.b_ij.shape[0]):
            for bb in range(op.nv):
                ref[a] += op.b_ij[p, 0, 0] * x[bb, 0] * op.b_ab[p, bb, a]
    np.testing.assert_allclose(ops.exchange_w(op.b_ij, op.b_ab, x, 1, op.nv)[:, 0], ref,
                               rtol=0, atol=1e-14)


def test_planted_mistakes_are_caught(monkeypatch):
    """Plausible slips in the factored products must fail the ERI pin."""
    op = tiny(no=3, nv=4, naux=5)
    amat, bmat = dense_from_eri(op)
    x = np.random.default_rng(6).standard_normal((op.n, 2))

    def pins_pass():
        apb, amb = ops.apply_apb_amb(op, x)
        return (np.allclose(ops.apply_a(op, x), amat @ x, atol=1e-12)
                and np.allclose(apb, (amat + bmat) @ x, atol=1e-12)
                and np.allclose(amb, (amat - bmat) @ x, atol=1e-12))

    assert pins_pass()
    good_w, good_wp, good_c = ops.exchange_w, ops.exchange_wp, ops.coulomb

    def wp_transposed(b_ia, x_, no, nv):  # (ia|jb) instead of (ib|ja)
        return good_c(b_ia, x_)

    def w_dropped(b_ij, b_ab, x_, no, nv):
        return np.zeros_like(x_)

    def coul_half(b_ia, x_):
        return 0.5 * good_c(b_ia, x_)

    def w_wrong_sign(b_ij, b_ab, x_, no, nv):  # exchange added instead of subtracted
        return -good_w(b_ij, b_ab, x_, no, nv)

    for name, bad in (("exchange_wp", wp_transposed), ("exchange_w", w_dropped),
                      ("coulomb", coul_half), ("exchange_w", w_wrong_sign)):
        monkeypatch.setattr(ops, name, bad)
        assert not pins_pass(), name
        monkeypatch.setattr(ops, "exchange_w", good_w)
        monkeypatch.setattr(ops, "exchange_wp", good_wp)
        monkeypatch.setattr(ops, "coulomb", good_c)
    assert pins_pass()


@pytest.mark.parametrize("ris", [False, True])
def test_a_minus_b_and_a_plus_b_positive_definite_at_small_config(ris):
    # definiteness of A +- B (imaginary frequencies otherwise), on a scaled-down
    # instance of the generator
    p = make_problem(6, 24, 120, 27, seed=3)
    op = OracleProblem.from_arrays(p.numpy())
    eye = np.eye(op.n)
    apb, amb = (ops.apply_tpm if ris else ops.apply_apb_amb)(op, eye)
    assert np.linalg.eigvalsh(apb).min() > 0.0
    assert np.linalg.eigvalsh(amb).min() > 0.0


def test_sampled_entries_match_full_products():
    op = tiny(no=4, nv=7, naux=9)
    rng = np.random.default_rng(8)
    x = rng.standard_normal((op.n, 1))
    apb, amb = ops.apply_apb_amb(op, x)
    xc = x[:, 0].reshape(op.no, op.nv)
    de = op.delta_eps().reshape(op.no, op.nv)
    for i, a in ((0, 0), (3, 6), (2, 1)):
        p, m = ops.sampled_entries(op.b_ia[:, i, :], op.b_ia[:, :, a], op.b_ij[:, i, :], op.b_ab[:, :, a],
                                   op.b_ia, op.a_x, de[i, a], xc, i, a)
        assert abs(p - apb[i * op.nv + a, 0]) < 1e-13
        assert abs(m - amb[i * op.nv + a, 0]) < 1e-13


def tiny_lr(no=3, nv=4, naux=5, naux_ris=4, nk=2, naux_lr=4, b_x=0.6, seed=13, t_cut=None):
    kw = {} if t_cut is None else {"t_cut": t_cut}
    p = make_problem(no, nv, naux, naux_ris, naux_ris_k=nk, a_x=0.16, seed=seed, b_x=b_x, naux_lr=naux_lr, **kw)
    return OracleProblem.from_arrays(p.numpy())


def test_range_separated_operators_match_eri_definition():
    """A and B with a_x (pq|rs) + b_x (pq|rs)^LR, element by element."""
    op = tiny_lr()
    eri = ops.dense_eri(ops.full_three_index(op.b_ia, op.b_ij, op.b_ab))
    eri_lr = ops.dense_eri(ops.full_three_index(op.blr_ia, op.blr_ij, op.blr_ab))
    amat, bmat = ops.dense_hessians(op.eps_occ, op.eps_vir, eri, op.a_x, eri_lr=eri_lr, b_x=op.b_x)
    x = np.random.default_rng(5).standard_normal((op.n, 3))
    np.testing.assert_allclose(ops.apply_a(op, x), amat @ x, rtol=0, atol=1e-13)
    p, m = ops.apply_apb_amb(op, x)
    np.testing.assert_allclose(p, (amat + bmat) @ x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(m, (amat - bmat) @ x, rtol=0, atol=1e-13)


def test_range_separated_ris_model_matches_eri_definition():
    """T with both exchange parts on the active block (Sec. 3.1)."""
    op = tiny_lr(no=4, nv=5, naux=6, naux_ris=5, nk=2, naux_lr=4, t_cut=1.0, seed=17)
    i0, na = op.active_ranges()
    assert 0 < i0 < op.no and 0 < na < op.nv
    occ = np.arange(op.no) >= i0
    vir = np.arange(op.nv) < na
    b = ops.full_three_index(op.bris_ia, op.bris_ij, op.bris_ab)
    bk = ops.full_three_index(op.bris_ia[:op.naux_ris_k], op.bris_ij[:op.naux_ris_k], op.bris_ab[:op.naux_ris_k])
    bl = ops.full_three_index(op.brislr_ia, op.brislr_ij, op.brislr_ab)
    eri_j, eri_k, eri_l = ops.dense_eri(b), ops.dense_eri(bk), ops.dense_eri(bl)
    a_j, b_j = ops.dense_hessians(op.eps_occ, op.eps_vir, eri_j, 0.0)
    a_k, b_k = ops.dense_hessians(op.eps_occ, op.eps_vir, eri_k, op.a_x, occ, vir, eri_lr=eri_l, b_x=op.b_x)
    a_0, b_0 = ops.dense_hessians(op.eps_occ, op.eps_vir, eri_k, 0.0)
    tmat, tb = a_j + (a_k - a_0), b_j + (b_k - b_0)
    x = np.random.default_rng(6).standard_normal((op.n, 3))
    np.testing.assert_allclose(ops.apply_t(op, x), tmat @ x, rtol=0, atol=1e-13)
    tp, tm = ops.apply_tpm(op, x)
    np.testing.assert_allclose(tp, (tmat + tb) @ x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(tm, (tmat - tb) @ x, rtol=0, atol=1e-13)


def test_long_range_tensor_equal_to_full_tensor_adds_the_weights():
    """With C = B the two exchange terms merge: a_x W + b_x W = (a_x + b_x) W."""
    op = tiny_lr(naux_lr=5)
    op.blr_ia, op.blr_ij, op.blr_ab = op.b_ia.copy(), op.b_ij.copy(), op.b_ab.copy()
    plain = OracleProblem(no=op.no, nv=op.nv, eps_occ=op.eps_occ, eps_vir=op.eps_vir, b_ia=op.b_ia, b_ij=op.b_ij,
                          b_ab=op.b_ab, a_x=op.a_x + op.b_x)
    x = np.random.default_rng(7).standard_normal((op.n, 2))
    np.testing.assert_allclose(ops.apply_a(op, x), ops.apply_a(plain, x), rtol=0, atol=1e-13)
    for u, v in zip(ops.apply_apb_amb(op, x), ops.apply_apb_amb(plain, x)):
        np.testing.assert_allclose(u, v, rtol=0, atol=1e-13)
