"""Pins of the oracle's Davidson and polarizability solvers (CPU only).

The converged results of a preconditioned Davidson run have plain definitions
(Sec. 2.1: any preconditioner reaches the exact eigenpairs, only faster), so
they are checked against dense LAPACK diagonalisation and dense solves, the
non-symmetric Casida matrix (Eq. Casida), the sum-over-states form of
Eq. TDDFT_polar, the Kato-Temple error bound, Cauchy interlacing of Ritz
values, preconditioner invariance, and the T = A limit of Sec. 2.1.
"""

import numpy as np
import pytest

from oracle import eigen_rpa, eigen_tda, polarizability
from oracle import operators as ops
from oracle.davidson import davidson_sym, diag_guess, n_init_rule
from oracle.linalg import orthonormalize
from oracle.operators import OracleProblem
from oracle.precond import diag_tda, inner_solve_pair, inner_solve_tda
from synth import make_dipoles, make_problem


def small(no=6, nv=24, naux=120, naux_ris=27, seed=3, **kw):
    p = make_problem(no, nv, naux, naux_ris, seed=seed, **kw)
    return p, OracleProblem.from_arrays(p.numpy())


def dense(op):
    eye = np.eye(op.n)
    a = ops.apply_a(op, eye)
    apb, amb = ops.apply_apb_amb(op, eye)
    return a, apb, amb


def rpa_dense_roots(apb, amb):
    lam, u = np.linalg.eigh(amb)
    s = u @ np.diag(np.sqrt(lam)) @ u.T
    w2, f = np.linalg.eigh(s @ apb @ s)
    return np.sqrt(w2), s, f


@pytest.mark.parametrize("precond", ["diag", "ris"])
def test_tda_matches_dense_eigh(precond):
    _, op = small()
    a, _, _ = dense(op)
    ref, vec = np.linalg.eigh(a)
    res = eigen_tda(op, 5, precond, tol=1e-8)
    assert res.converged
    np.testing.assert_allclose(res.omega, ref[:5], rtol=0, atol=1e-10)
    # eigenvectors up to sign: |overlap| = 1
    ov = np.abs(np.sum(res.x * vec[:, :5], axis=0))
    np.testing.assert_allclose(ov, 1.0, atol=1e-7)
    np.testing.assert_allclose(np.linalg.norm(res.x, axis=0), 1.0, atol=1e-12)


@pytest.mark.parametrize("precond", ["diag", "ris"])
def test_rpa_matches_dense_and_casida(precond):
    _, op = small()
    _, apb, amb = dense(op)
    ref, _, _ = rpa_dense_roots(apb, amb)
    # the non-symmetric Casida matrix [[A, B], [-B, -A]] has eigenvalues +-Omega
    amat, bmat = 0.5 * (apb + amb), 0.5 * (apb - amb)
    cas = np.block([[amat, bmat], [-bmat, -amat]])
    ev = np.sort(np.linalg.eigvals(cas).real)
    pos = ev[ev > 0][:5]
    np.testing.assert_allclose(ref[:5], pos, rtol=0, atol=1e-9)
    res = eigen_rpa(op, 5, precond, tol=1e-8)
    assert res.converged
    np.testing.assert_allclose(res.omega, ref[:5], rtol=0, atol=1e-10)
    # X^T X - Y^T Y = 1 and the Casida equations hold
    norm = np.sum(res.x * res.x, axis=0) - np.sum(res.y * res.y, axis=0)
    np.testing.assert_allclose(norm, 1.0, atol=1e-10)
    lhs = amat @ res.x + bmat @ res.y
    np.testing.assert_allclose(lhs, res.x * res.omega[None, :], atol=1e-7)
    lhs2 = bmat @ res.x + amat @ res.y
    np.testing.assert_allclose(lhs2, -res.y * res.omega[None, :], atol=1e-7)


def test_preconditioner_invariance_tight_tolerance():
    _, op = small(seed=8)
    r_d = eigen_tda(op, 4, "diag", tol=1e-8)
    r_r = eigen_tda(op, 4, "ris", tol=1e-8)
    np.testing.assert_allclose(r_d.omega, r_r.omega, rtol=0, atol=1e-10)
    q_d = eigen_rpa(op, 4, "diag", tol=1e-8)
    q_r = eigen_rpa(op, 4, "ris", tol=1e-8)
    np.testing.assert_allclose(q_d.omega, q_r.omega, rtol=0, atol=1e-10)


def test_kato_temple_and_interlacing():
    _, op = small(seed=4)
    a, _, _ = dense(op)
    lam = np.linalg.eigvalsh(a)
    de = op.delta_eps()
    # stop early on purpose so that residuals are not tiny
    res = davidson_sym(lambda x: a @ x, de, 3, diag_guess(de, 11),
                       lambda r, om: (diag_tda(de, r, om), 0), tol=1e-3, max_iter=3)
    for n in range(3):
        # Rayleigh-Ritz values are upper bounds (Cauchy interlacing)
        assert res.omega[n] >= lam[n] - 1e-12
        gap = lam[n + 1] - res.omega[n]
        if gap > 0:
            assert res.omega[n] - lam[n] <= res.resid[n] ** 2 / gap + 1e-12
    # Ritz values do not increase as the subspace grows
    prev = None
    for it in range(1, 6):
        r = davidson_sym(lambda x: a @ x, de, 3, diag_guess(de, 11),
                         lambda r_, om: (diag_tda(de, r_, om), 0), tol=1e-14, max_iter=it)
        if prev is not None:
            assert np.all(r.omega <= prev + 1e-13)
        prev = r.omega


def test_t_equal_a_limit_converges_at_once():
    # ris tensor = full tensor, no noise, no cutoff, every row in exchange:
    # then T = A and the initial guess already holds the eigenvectors (Sec. 2.1)
    p = make_problem(5, 20, 80, 0, seed=2, ris_source="full", noise=0.0, t_cut=np.inf,
                     naux_ris_k=80)
    op = OracleProblem.from_arrays(p.numpy())
    a, _, _ = dense(op)
    ref = np.linalg.eigvalsh(a)
    res = eigen_tda(op, 4, "ris", tol=1e-6, init_tol=1e-9, init_max=60)
    assert res.converged and res.n_iter == 1
    assert res.history[0] <= 1e-6
    np.testing.assert_allclose(res.omega, ref[:4], atol=1e-12)


def test_zero_coupling_gives_orbital_energy_differences_in_one_iteration():
    p, op = small()
    op.b_ia[:] = 0.0
    op.b_ij[:] = 0.0
    op.b_ab[:] = 0.0
    res = eigen_tda(op, 5, "diag")
    assert res.converged and res.n_iter == 1
    np.testing.assert_allclose(res.omega, np.sort(op.delta_eps())[:5], atol=1e-15)


def test_not_converged_status_and_n_init_rule():
    _, op = small()
    res = eigen_tda(op, 5, "diag", max_iter=1)
    assert res.status == "not_converged" and res.n_iter == 1
    assert res.n_mv == n_init_rule(5, "diag", op.n) == 13
    assert n_init_rule(5, "ris", op.n) == 8
    assert n_init_rule(1, "ris", op.n) == 2
    assert n_init_rule(20, "ris", op.n) == 23


def test_inner_solvers_converge_to_exact_shifted_solution():
    _, op = small(seed=9)
    de = op.delta_eps()
    t = ops.apply_t(op, np.eye(op.n))
    rng = np.random.default_rng(0)
    r = rng.standard_normal((op.n, 3))
    sh = np.array([0.2, 0.3, 0.35])
    sol, nmv, it = inner_solve_tda(lambda x: t @ x, de, r, sh, tol=1e-10, max_iter=200)
    for n in range(3):
        ref = np.linalg.solve(t - sh[n] * np.eye(op.n), r[:, n])
        np.testing.assert_allclose(sol[:, n], ref, rtol=0, atol=1e-8 * np.abs(ref).max())
    tp, tm = ops.apply_tpm(op, np.eye(op.n))
    r2 = rng.standard_normal((op.n, 3))
    d1, d2, _, _ = inner_solve_pair(lambda x: (tp @ x, tm @ x), de, r, r2, sh, tol=1e-10,
                                    max_iter=200)
    for n in range(3):
        big = np.block([[tp, -sh[n] * np.eye(op.n)], [-sh[n] * np.eye(op.n), tm]])
        ref = np.linalg.solve(big, np.concatenate([r[:, n], r2[:, n]]))
        np.testing.assert_allclose(np.concatenate([d1[:, n], d2[:, n]]), ref,
                                   atol=1e-8 * np.abs(ref).max())


@pytest.mark.parametrize("precond", ["diag", "ris"])
def test_polarizability_matches_dense_and_sum_over_states(precond):
    p, op = small(seed=5)
    a, apb, amb = dense(op)
    pm = make_dipoles(p, 3).numpy().T
    om = [0.0, 0.0569542, 0.2]
    res = polarizability(op, pm, om, precond, tol=1e-9)
    assert res.converged
    # static: 2 P^T (A+B)^-1 P
    a0 = 2.0 * pm.T @ np.linalg.solve(apb, pm)
    np.testing.assert_allclose(res.alpha[0], a0, rtol=1e-8)
    assert np.allclose(res.alpha[0], res.alpha[0].T, rtol=1e-8)
    assert np.linalg.eigvalsh(0.5 * (res.alpha[0] + res.alpha[0].T)).min() > 0.0
    # dynamic: the sandwich of Eq. TDDFT_polar with mu_vo = mu_ov = P
    bm = 0.5 * (apb - amb)
    n = op.n
    for f, w in enumerate(om):
        big = np.block([[a - w * np.eye(n), bm], [bm, a + w * np.eye(n)]])
        mu = np.vstack([pm, pm])
        ref = mu.T @ np.linalg.solve(big, mu)
        np.testing.assert_allclose(res.alpha[f], ref, rtol=1e-8)
    # sum over states: alpha_uv(w) = sum_n 2 (P_u^T S F_n)(P_v^T S F_n) / (Omega_n^2 - w^2)
    omg, s, fv = rpa_dense_roots(apb, amb)
    t = pm.T @ s @ fv
    for f, w in enumerate(om):
        sos = 2.0 * (t / (omg ** 2 - w ** 2)[None, :]) @ t.T
        np.testing.assert_allclose(res.alpha[f], sos, rtol=1e-8)
    # alpha(w) grows with w below the first pole (diagonal elements)
    assert np.all(np.diag(res.alpha[2]) > np.diag(res.alpha[1]))
    assert np.all(np.diag(res.alpha[1]) > np.diag(res.alpha[0]))


def test_gram_schmidt_orthonormal_and_drops_dependent_directions():
    rng = np.random.default_rng(1)
    v = orthonormalize(rng.standard_normal((50, 6)))
    np.testing.assert_allclose(v.T @ v, np.eye(6), atol=1e-14)
    w = np.hstack([rng.standard_normal((50, 3)), v[:, :2] @ rng.standard_normal((2, 2))])
    w = np.hstack([w, w[:, :1] * 3.0])
    out = orthonormalize(w, v)
    assert out.shape[1] == 3
    np.testing.assert_allclose(out.T @ out, np.eye(3), atol=1e-14)
    np.testing.assert_allclose(v.T @ out, 0.0, atol=1e-14)


@pytest.mark.slow
def test_config0_both_preconditioners_reach_dense_roots():
    p = make_problem(20, 80, 400, 90, seed=0)
    op = OracleProblem.from_arrays(p.numpy())
    a, apb, amb = dense(op)
    ref = np.linalg.eigvalsh(a)[:5]
    for pc in ("diag", "ris"):
        res = eigen_tda(op, 5, pc)
        assert res.converged
        # converged to 1e-5 in the residual: Kato-Temple gives ~1e-9 here
        np.testing.assert_allclose(res.omega, ref, atol=1e-8)


@pytest.mark.parametrize("mode", ["tda", "rpa"])
def test_restart_reaches_dense_roots(mode):
    """A subspace limit far below the iteration count forces restarts onto the
    leading Ritz vectors (k + n_extra of them; for full TDDFT their Z and Z');
    the roots still converge to the dense ones."""
    _, op = small(no=8, nv=32, naux=160, naux_ris=36, seed=5)
    a, apb, amb = dense(op)
    if mode == "tda":
        ref = np.linalg.eigh(a)[0][:5]
        res = eigen_tda(op, 5, "diag", tol=1e-8, m_max=30)
        full = eigen_tda(op, 5, "diag", tol=1e-8)
    else:
        ref = rpa_dense_roots(apb, amb)[0][:5]
        res = eigen_rpa(op, 5, "diag", tol=1e-8, m_max=40)
        full = eigen_rpa(op, 5, "diag", tol=1e-8)
    assert res.converged
    assert res.n_mv > 40  # more products than the subspace holds: it restarted
    np.testing.assert_allclose(res.omega, ref, rtol=0, atol=1e-10)
    np.testing.assert_allclose(full.omega, ref, rtol=0, atol=1e-10)
