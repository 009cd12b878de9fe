"""Pins of the oracle's preconditioners (Eq. precondition; Sec. 2.1, Sec. 3.1).

Converged roots do not depend on the preconditioner, so a slip in one would
change only the iteration and product counts -- the paper's figures of
merit.  These tests therefore check the preconditioners themselves against
what fixes them:

* the diagonal step solves (de - Omega) v = r: multiplying back must give r,
  including the guarded denominators;
* the diagonal pair step solves [[de, -s], [-s, de]] (d1; d2) = (r1; r2)
  (the diagonal stand-in for [[A+B, -Omega], [-Omega, A-B]] of Eq. Casida):
  the 2 x 2 product per element, and a library solve of the explicit
  2N x 2N system, must give the right-hand sides back;
* the inner ris solves at the method's loose tolerance: each right-hand side
  stops at the first inner iterate whose residual, relative to the
  right-hand side (unit-normalised), is below 1e-2, or after the iteration
  budget; scaling a right-hand side scales its solution and leaves the
  counts unchanged (a relative, not absolute, threshold);
* the full-TDDFT T = A limit: with the ris model equal to A the initial
  guess already holds the eigenvectors and the solve stops at iteration 1.

Each check is written as a function of the preconditioner so that planted
mistakes (a flipped off-diagonal sign, a de + Omega denominator, an absolute
inner threshold) are shown to fail it.
"""

import numpy as np
import pytest

from oracle import eigen_rpa
from oracle import operators as ops
from oracle import precond as pc
from oracle.operators import OracleProblem
from synth import make_problem


def _rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# diagonal step
# ---------------------------------------------------------------------------

def check_diag_tda(fn):
    """Multiply back: (de - Omega_n) * v_n = r_n elementwise, and the guard
    replaces |de - Omega| < 1e-8 by +-1e-8 with the sign of de - Omega."""
    g = _rng(1)
    de = np.sort(g.uniform(0.3, 2.5, 40))
    r = g.normal(size=(40, 3))
    om = np.array([0.1, 0.4123, 3.0])
    v = fn(de, r, om)
    back = (de[:, None] - om[None, :]) * v
    if not np.allclose(back, r, rtol=1e-14, atol=0):
        return False
    # guarded entries: one exact zero denominator (+1e-8) and one tiny negative (-1e-8)
    de2 = np.array([0.5, 0.7, 0.9])
    om2 = np.array([0.7])
    de2[2] = 0.7 - 3e-9
    r2 = np.array([[1.0], [2.0], [3.0]])
    v2 = fn(de2, r2, om2)
    return (np.isclose(v2[0, 0], 1.0 / (0.5 - 0.7), rtol=1e-14) and v2[1, 0] == 2.0 / 1e-8
            and v2[2, 0] == 3.0 / -1e-8)


def test_diag_tda_solves_the_shifted_diagonal_system():
    assert check_diag_tda(pc.diag_tda)


def test_diag_tda_pin_rejects_planted_mistakes():
    assert not check_diag_tda(lambda de, r, om: r / (de[:, None] + om[None, :]))          # de + Omega
    assert not check_diag_tda(lambda de, r, om: r / (de[:, None] - om[None, :] + 1e-30))  # no guard
    assert not check_diag_tda(lambda de, r, om: r * (de[:, None] - om[None, :]))           # multiplied


# ---------------------------------------------------------------------------
# diagonal pair step (full TDDFT and the polarizability)
# ---------------------------------------------------------------------------

def check_diag_pair(fn):
    g = _rng(2)
    n = 30
    de = np.sort(g.uniform(0.3, 2.5, n))
    om = np.array([0.05, 0.29, 1.1])
    r1 = g.normal(size=(n, 3))
    r2 = g.normal(size=(n, 3))
    d1, d2 = fn(de, r1, r2, om)
    # element by element: [[de, -s], [-s, de]] (d1; d2) = (r1; r2)
    b1 = de[:, None] * d1 - om[None, :] * d2
    b2 = -om[None, :] * d1 + de[:, None] * d2
    if not (np.allclose(b1, r1, rtol=1e-12, atol=1e-12) and np.allclose(b2, r2, rtol=1e-12, atol=1e-12)):
        return False
    # the explicit 2N x 2N block system through a library solve, per column
    for c in range(3):
        big = np.block([[np.diag(de), -om[c] * np.eye(n)], [-om[c] * np.eye(n), np.diag(de)]])
        sol = np.linalg.solve(big, np.concatenate([r1[:, c], r2[:, c]]))
        if not (np.allclose(sol[:n], d1[:, c], rtol=1e-12, atol=1e-13)
                and np.allclose(sol[n:], d2[:, c], rtol=1e-12, atol=1e-13)):
            return False
    return True


def test_diag_pair_solves_the_two_by_two_system():
    assert check_diag_pair(pc.diag_pair)


def test_diag_pair_pin_rejects_planted_mistakes():
    def flipped(de, r1, r2, s):  # sign of the off-diagonal term
        den = (de[:, None] - s[None, :]) * (de[:, None] + s[None, :])
        return ((de[:, None] * r1 - s[None, :] * r2) / den, (de[:, None] * r2 - s[None, :] * r1) / den)

    def swapped(de, r1, r2, s):  # d1 and d2 exchanged
        a, b = pc.diag_pair(de, r1, r2, s)
        return b, a

    def decoupled(de, r1, r2, s):  # each component alone, (de - s)^(-1) r
        return pc.diag_tda(de, r1, s), pc.diag_tda(de, r2, s)

    for bad in (flipped, swapped, decoupled):
        assert not check_diag_pair(bad), bad.__name__


def test_diag_pair_guard_keeps_the_sign():
    """A denominator de - s within 1e-8 of zero is replaced by +-1e-8 (reading
    of Sec. 2.1 where the paper is silent); the other factor de + s stays."""
    de = np.array([0.4, 0.6])
    s = np.array([0.6])
    r1 = np.array([[1.0], [1.0]])
    r2 = np.array([[0.0], [0.0]])
    d1, _ = pc.diag_pair(de, r1, r2, s)
    assert d1[1, 0] == pytest.approx(0.6 / (1e-8 * 1.2), rel=1e-12)
    assert d1[0, 0] == pytest.approx(0.4 / ((0.4 - 0.6) * (0.4 + 0.6)), rel=1e-12)


# ---------------------------------------------------------------------------
# inner ris solves at the method's loose tolerance
# ---------------------------------------------------------------------------

def _ris_problem():
    p = make_problem(6, 24, 120, 27, seed=5)
    op = OracleProblem.from_arrays(p.numpy())
    eye = np.eye(op.n)
    t = ops.apply_t(op, eye)
    tp, tm = ops.apply_tpm(op, eye)
    return op, 0.5 * (t + t.T), 0.5 * (tp + tp.T), 0.5 * (tm + tm.T)


def _rel_resid_tda(t, v, r, s):
    res = t @ v - v * s[None, :] - r
    return np.linalg.norm(res, axis=0) / np.linalg.norm(r, axis=0)


def _rel_resid_pair(tp, tm, d1, d2, r1, r2, s):
    a = tp @ d1 - d2 * s[None, :] - r1
    b = tm @ d2 - d1 * s[None, :] - r2
    return np.sqrt(np.sum(a * a, axis=0) + np.sum(b * b, axis=0)) / np.sqrt(
        np.sum(r1 * r1, axis=0) + np.sum(r2 * r2, axis=0))


def check_inner_tda(solve, op, t, tol=1e-2):
    """Every column meets tol relative to its right-hand side (checked with
    the explicit T), the solve stops at the first iteration where all did,
    and scaling the right-hand sides by 1e6 changes nothing but the scale."""
    g = _rng(7)
    de = op.delta_eps()
    r = g.normal(size=(op.n, 4)) * np.array([1e-3, 1.0, 30.0, 0.2])[None, :]
    s = np.array([0.35, 0.41, 0.44, 0.5])
    v, nmv, nit = solve(lambda x: ops.apply_t(op, x), de, r, s, tol, 20)
    if nit >= 20 or not np.all(_rel_resid_tda(t, v, r, s) < tol):
        return False
    if nit > 1:
        v1, _, _ = solve(lambda x: ops.apply_t(op, x), de, r, s, tol, nit - 1)
        if np.all(_rel_resid_tda(t, v1, r, s) < tol):  # it could have stopped earlier
            return False
    v6, nmv6, nit6 = solve(lambda x: ops.apply_t(op, x), de, 1e6 * r, s, tol, 20)
    return nit6 == nit and nmv6 == nmv and np.allclose(v6, 1e6 * v, rtol=1e-8, atol=0)


def test_inner_tda_stops_at_the_relative_threshold():
    op, t, _, _ = _ris_problem()
    assert check_inner_tda(pc.inner_solve_tda, op, t)


def test_inner_tda_pin_rejects_an_absolute_threshold():
    op, t, _, _ = _ris_problem()

    def absolute_threshold(apply_t, de, r, shifts, tol=1e-2, max_iter=20):
        # a threshold on the raw residual: the same as a relative one of
        # tol / ||r||, which the largest right-hand side would meet too late
        big = np.linalg.norm(r, axis=0).max()
        return pc.inner_solve_tda(apply_t, de, r, shifts, tol / big, max_iter)

    assert not check_inner_tda(absolute_threshold, op, t)


def test_inner_tda_respects_the_iteration_budget():
    op, t, _, _ = _ris_problem()
    de = op.delta_eps()
    r = _rng(3).normal(size=(op.n, 3))
    s = np.array([0.3, 0.4, 0.5])
    for budget in (1, 2, 5):
        v, nmv, nit = pc.inner_solve_tda(lambda x: ops.apply_t(op, x), de, r, s, 1e-30, budget)
        assert nit == budget
        assert v.shape == r.shape and np.all(np.isfinite(v))


def test_inner_pair_stops_at_the_relative_threshold():
    op, _, tp, tm = _ris_problem()
    de = op.delta_eps()
    g = _rng(11)
    r1 = g.normal(size=(op.n, 3)) * np.array([1e-2, 1.0, 5.0])[None, :]
    r2 = g.normal(size=(op.n, 3)) * np.array([1e-2, 1.0, 5.0])[None, :]
    s = np.array([0.0, 0.2, 0.3])
    f = lambda x: ops.apply_tpm(op, x)
    d1, d2, nmv, nit = pc.inner_solve_pair(f, de, r1, r2, s, 1e-2, 20)
    assert nit < 20
    assert np.all(_rel_resid_pair(tp, tm, d1, d2, r1, r2, s) < 1e-2)
    if nit > 1:
        e1, e2, _, _ = pc.inner_solve_pair(f, de, r1, r2, s, 1e-2, nit - 1)
        assert not np.all(_rel_resid_pair(tp, tm, e1, e2, r1, r2, s) < 1e-2)
    g1, g2, nmv6, nit6 = pc.inner_solve_pair(f, de, 1e6 * r1, 1e6 * r2, s, 1e-2, 20)
    assert (nit6, nmv6) == (nit, nmv)
    np.testing.assert_allclose(g1, 1e6 * d1, rtol=1e-8)
    np.testing.assert_allclose(g2, 1e6 * d2, rtol=1e-8)


def test_inner_pair_at_tight_tolerance_solves_the_block_system():
    """With a tight threshold the pair solve reaches the dense solution of
    [[T+, -s], [-s, T-]] (d1; d2) = (r1; r2)."""
    op, _, tp, tm = _ris_problem()
    de = op.delta_eps()
    g = _rng(12)
    r1, r2 = g.normal(size=(op.n, 2)), g.normal(size=(op.n, 2))
    s = np.array([0.1, 0.25])
    d1, d2, _, _ = pc.inner_solve_pair(lambda x: ops.apply_tpm(op, x), de, r1, r2, s, 1e-12, 200)
    n = op.n
    for c in range(2):
        big = np.block([[tp, -s[c] * np.eye(n)], [-s[c] * np.eye(n), tm]])
        sol = np.linalg.solve(big, np.concatenate([r1[:, c], r2[:, c]]))
        np.testing.assert_allclose(d1[:, c], sol[:n], atol=1e-9 * np.abs(sol).max())
        np.testing.assert_allclose(d2[:, c], sol[n:], atol=1e-9 * np.abs(sol).max())


# ---------------------------------------------------------------------------
# full-TDDFT T = A limit
# ---------------------------------------------------------------------------

def test_rpa_t_equal_a_limit_converges_at_once():
    """ris tensor = full tensor, no noise, no energy window, every row in the
    exchange: T+- = A+-B, so the ris initial guess (solved tightly) already
    spans the eigenvectors and the full-TDDFT solve stops at iteration 1."""
    p = make_problem(5, 20, 80, 0, seed=2, ris_source="full", noise=0.0, t_cut=np.inf, naux_ris_k=80)
    op = OracleProblem.from_arrays(p.numpy())
    eye = np.eye(op.n)
    apb, amb = ops.apply_apb_amb(op, eye)
    tp, tm = ops.apply_tpm(op, eye)
    np.testing.assert_allclose(tp, apb, atol=1e-13)
    np.testing.assert_allclose(tm, amb, atol=1e-13)
    ev, u = np.linalg.eigh(0.5 * (amb + amb.T))
    sq = (u * np.sqrt(ev)) @ u.T
    ref = np.sqrt(np.linalg.eigvalsh(sq @ apb @ sq))
    res = eigen_rpa(op, 4, "ris", tol=1e-6, init_tol=1e-9, init_max=60)
    assert res.converged and res.n_iter == 1, (res.status, res.n_iter)
    np.testing.assert_allclose(res.omega, ref[:4], atol=1e-12)
