"""Davidson eigensolvers for TDDFT (Sec. 2.1 and Fig. 1; test infrastructure only).

TDA (Eq. TDA): the k lowest eigenpairs of the symmetric A.  Each iteration
projects A on the orthonormal subspace V (a = V^T A V), diagonalises it,
forms Ritz vectors X = V x and residuals R_n = A X_n - Omega_n X_n
(Eq. residual), stops when every ||R_n|| is below the threshold, and
otherwise expands V with preconditioned residuals of the unconverged roots
(Eq. precondition), orthonormalised against V and each other.

Full TDDFT (Eq. Casida): with Z = X+Y and Z' = X-Y the problem reads
(A+B) Z = Omega Z', (A-B) Z' = Omega Z.  The oracle uses one subspace V for
both components: a_+ = V^T (A+B) V and a_- = V^T (A-B) V; with a_- = L L^T,
the eigenpairs (Omega^2, w) of L^T a_+ L give z = L w / sqrt(Omega) (w unit)
and z' = a_+ z / Omega, normalised so that z^T z' = X^T X - Y^T Y = 1.  The
residual pair is R = (A+B) V z - Omega V z', R' = (A-B) V z' - Omega V z, its
norm sqrt(||R||^2 + ||R'||^2).  (The paper's own full-TDDFT algorithm is in
its supporting information, which is not available; this Galerkin form
converges to the same roots.)

Initial subspace (Sec. 2.1, Sec. 3.2): N_init = k + min(k, 3) vectors for
the ris preconditioner and k + 8 for the diagonal one.  The diagonal guess is
the unit vectors of the N_init smallest de (stable order); the ris guess is
the N_init lowest Ritz vectors of a Davidson run on T itself (diagonal
preconditioner, tolerance 1e-3, at most 20 iterations, Sec. 3.1).

Counting (Sec. 3, Sec. 4): n_iter counts products of A with a block of
vectors, the initial block included; n_mv counts vectors multiplied by A
(for full TDDFT one vector's (A+B, A-B) pair counts once); n_inner_mv counts
vectors multiplied by T in the preconditioner and in the initial guess.
"""

from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np

from . import operators as ops
from .linalg import orthonormalize
from .precond import diag_pair, diag_tda, inner_solve_pair, inner_solve_tda


@dataclasses.dataclass
class SolveResult:
    omega: np.ndarray
    x: np.ndarray
    y: Optional[np.ndarray]
    resid: np.ndarray
    n_iter: int
    n_mv: int
    n_inner_mv: int
    history: List[float]
    status: str  # "ok", "not_converged", "breakdown", "indefinite"

    @property
    def converged(self) -> bool:
        return self.status == "ok"


class IndefiniteError(RuntimeError):
    pass


def n_init_rule(k: int, precond: str, n: int, n_extra: Optional[int] = None) -> int:
    """N_init = k + min(k, 3) for rid, k + 8 otherwise (Sec. 3.2), capped at N."""
    if n_extra is None:
        n_extra = min(k, 3) if precond == "ris" else 8
    return min(n, k + n_extra)


def diag_guess(de: np.ndarray, count: int) -> np.ndarray:
    """Unit vectors e_ia of the `count` smallest de_ia, ties by index."""
    idx = np.argsort(de, kind="stable")[:count]
    v = np.zeros((de.shape[0], len(idx)))
    v[idx, np.arange(len(idx))] = 1.0
    return v


def _sym(a):
    return 0.5 * (a + a.T)


def davidson_sym(apply_op: Callable, de: np.ndarray, k: int, v0: np.ndarray,
                 precond: Callable, tol: float, max_iter: int,
                 m_max: Optional[int] = None, keep: Optional[int] = None) -> SolveResult:
    """Davidson for the k lowest eigenpairs of a symmetric operator.

    precond(R, omegas) -> (new directions (N, n), inner products counted).
    """
    v = orthonormalize(v0)
    av = apply_op(v)
    n_iter, n_mv, n_inner = 1, v.shape[1], 0
    m_max = m_max or max(200, 40 * k)
    keep = keep or k
    history = []
    while True:
        a = _sym(v.T @ av)
        w, x = np.linalg.eigh(a)
        kk = min(k, len(w))
        w, xk = w[:kk], x[:, :kk]
        xv = v @ xk
        r = av @ xk - xv * w[None, :]
        rn = np.linalg.norm(r, axis=0)
        history.append(float(rn.max()))
        if np.all(rn < tol):
            return SolveResult(w, xv, None, rn, n_iter, n_mv, n_inner, history, "ok")
        if n_iter >= max_iter:
            return SolveResult(w, xv, None, rn, n_iter, n_mv, n_inner, history, "not_converged")
        act = np.where(rn >= tol)[0]
        new, ninner = precond(r[:, act], w[act])
        n_inner += ninner
        if v.shape[1] + new.shape[1] > m_max:
            # restart: collapse onto the leading Ritz vectors (exact, by linearity)
            c = x[:, :min(keep, x.shape[1])]
            v, av = v @ c, av @ c
        vn = orthonormalize(new, v)
        if vn.shape[1] == 0:
            return SolveResult(w, xv, None, rn, n_iter, n_mv, n_inner, history, "breakdown")
        v = np.hstack([v, vn])
        av = np.hstack([av, apply_op(vn)])
        n_iter += 1
        n_mv += vn.shape[1]


def davidson_rpa(apply_pm: Callable, de: np.ndarray, k: int, v0: np.ndarray,
                 precond: Callable, tol: float, max_iter: int,
                 m_max: Optional[int] = None, keep: Optional[int] = None) -> SolveResult:
    """Shared-subspace Davidson for (A+B) Z = Omega Z', (A-B) Z' = Omega Z.

    precond(RZ, RZ', omegas) -> (new directions (N, n), inner products counted).
    Returns x = X = (Z+Z')/2 and y = Y = (Z-Z')/2.
    """
    v = orthonormalize(v0)
    pv, mv = apply_pm(v)
    n_iter, n_mv, n_inner = 1, v.shape[1], 0
    m_max = m_max or max(200, 40 * k)
    keep = keep or k
    history = []
    while True:
        ap = _sym(v.T @ pv)
        am = _sym(v.T @ mv)
        try:
            lo = np.linalg.cholesky(am)
        except np.linalg.LinAlgError as e:
            raise IndefiniteError("projected A-B is not positive definite") from e
        w2all, wvall = np.linalg.eigh(_sym(lo.T @ ap @ lo))
        kk = min(k, len(w2all))
        w2, wv = w2all[:kk], wvall[:, :kk]
        if np.any(w2 <= 0.0):
            raise IndefiniteError("non-positive Omega^2 in the projected problem")
        om = np.sqrt(w2)
        z = (lo @ wv) / np.sqrt(om)[None, :]
        zp = (ap @ z) / om[None, :]
        zv, zpv = v @ z, v @ zp
        rz = pv @ z - zpv * om[None, :]
        rzp = mv @ zp - zv * om[None, :]
        rn = np.sqrt(np.sum(rz * rz, axis=0) + np.sum(rzp * rzp, axis=0))
        history.append(float(rn.max()))
        xo, yo = 0.5 * (zv + zpv), 0.5 * (zv - zpv)
        if np.all(rn < tol):
            return SolveResult(om, xo, yo, rn, n_iter, n_mv, n_inner, history, "ok")
        if n_iter >= max_iter:
            return SolveResult(om, xo, yo, rn, n_iter, n_mv, n_inner, history, "not_converged")
        act = np.where(rn >= tol)[0]
        new, ninner = precond(rz[:, act], rzp[:, act], om[act])
        n_inner += ninner
        if v.shape[1] + new.shape[1] > m_max:
            # restart on the Z and Z' of the `keep` lowest positive Ritz pairs
            nk = int(min(max(keep, kk), len(w2all)))
            while nk > kk and w2all[nk - 1] <= 0.0:
                nk -= 1
            omk = np.sqrt(w2all[:nk])
            zk = (lo @ wvall[:, :nk]) / np.sqrt(omk)[None, :]
            zpk = (ap @ zk) / omk[None, :]
            c = orthonormalize(np.hstack([zk, zpk]))
            v, pv, mv = v @ c, pv @ c, mv @ c
        vn = orthonormalize(new, v)
        if vn.shape[1] == 0:
            return SolveResult(om, xo, yo, rn, n_iter, n_mv, n_inner, history, "breakdown")
        v = np.hstack([v, vn])
        a, b = apply_pm(vn)
        pv, mv = np.hstack([pv, a]), np.hstack([mv, b])
        n_iter += 1
        n_mv += vn.shape[1]


def eigen_tda(prob: ops.OracleProblem, k: int, precond: str = "diag", tol: float = 1e-5,
              max_iter: int = 100, n_extra: Optional[int] = None, inner_tol: float = 1e-2,
              inner_max: int = 20, init_tol: float = 1e-3, init_max: int = 20,
              m_max: Optional[int] = None) -> SolveResult:
    """k lowest TDA roots of A (Eq. TDA) with the diagonal or the ris preconditioner."""
    de = prob.delta_eps()
    n_init = n_init_rule(k, precond, prob.n, n_extra)
    apply_a = lambda x: ops.apply_a(prob, x)
    if precond == "diag":
        v0, inner0 = diag_guess(de, n_init), 0

        def pc(r, om):
            return diag_tda(de, r, om), 0
    elif precond == "ris":
        apply_t = lambda x: ops.apply_t(prob, x)
        guess = davidson_sym(apply_t, de, n_init, diag_guess(de, n_init_rule(n_init, "diag", prob.n)),
                             lambda r, om: (diag_tda(de, r, om), 0), init_tol, init_max)
        v0, inner0 = guess.x, guess.n_mv

        def pc(r, om):
            sol, nmv, _ = inner_solve_tda(apply_t, de, r, om, inner_tol, inner_max)
            return sol, nmv
    else:
        raise ValueError(precond)
    res = davidson_sym(apply_a, de, k, v0, pc, tol, max_iter, m_max, keep=n_init)
    res.n_inner_mv += inner0
    return res


def eigen_rpa(prob: ops.OracleProblem, k: int, precond: str = "diag", tol: float = 1e-5,
              max_iter: int = 100, n_extra: Optional[int] = None, inner_tol: float = 1e-2,
              inner_max: int = 20, init_tol: float = 1e-3, init_max: int = 20,
              m_max: Optional[int] = None) -> SolveResult:
    """k lowest full-TDDFT roots (Eq. Casida) with the diagonal or the ris preconditioner."""
    de = prob.delta_eps()
    n_init = n_init_rule(k, precond, prob.n, n_extra)
    apply_pm = lambda x: ops.apply_apb_amb(prob, x)

    def diag_pc(rz, rzp, om):
        d1, d2 = diag_pair(de, rz, rzp, om)
        return np.hstack([d1, d2]), 0

    if precond == "diag":
        v0, inner0 = diag_guess(de, n_init), 0
        pc = diag_pc
    elif precond == "ris":
        apply_tpm = lambda x: ops.apply_tpm(prob, x)
        guess = davidson_rpa(apply_tpm, de, n_init, diag_guess(de, n_init_rule(n_init, "diag", prob.n)),
                             diag_pc, init_tol, init_max)
        zg = guess.x + guess.y
        zpg = guess.x - guess.y
        v0, inner0 = np.hstack([zg, zpg]), guess.n_mv

        def pc(rz, rzp, om):
            d1, d2, nmv, _ = inner_solve_pair(apply_tpm, de, rz, rzp, om, inner_tol, inner_max)
            return np.hstack([d1, d2]), nmv
    else:
        raise ValueError(precond)
    res = davidson_rpa(apply_pm, de, k, v0, pc, tol, max_iter, m_max, keep=n_init)
    res.n_inner_mv += inner0
    return res
