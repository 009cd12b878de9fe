"""Preconditioners of the Davidson step (Eq. precondition; test infrastructure only).

v_n = (T - Omega_n)^(-1) R_n.  With the diagonal T this is an elementwise
division (Sec. 2.1).  With the ris model the shifted system is solved by an
inner Krylov method (Sec. 2.1) to a loose tolerance of 1e-2 and at most 20
iterations (Sec. 3.1).

Readings taken where the paper is silent:
* the diagonal T is de_ia = eps_a - eps_i; a denominator smaller than 1e-8 in
  magnitude is replaced by +-1e-8 (its sign kept, + for zero);
* the inner method is a block Galerkin (Davidson-type) solver: all right-hand
  sides of one outer iteration share one subspace U, each is solved from its
  own projected shifted system, and U is expanded with the diagonally
  preconditioned inner residuals of the unconverged right-hand sides;
* the inner tolerance is relative: right-hand sides are scaled to unit norm
  before the solve (an absolute 1e-2 would be met trivially once the outer
  residual drops below it, contradicting the fast outer rate of Sec. 4.1);
* the full-TDDFT (and polarizability) form solves the 2x2 block system
  [[T+, -s], [-s, T-]] (d; d') = (r1; r2) for the pair of residual components,
  with T+ / T- the ris models of A+B / A-B; the diagonal version of that
  system is solved in closed form.
"""

from __future__ import annotations

import numpy as np

from .linalg import orthonormalize

DENOM_GUARD = 1e-8


def _guard(d: np.ndarray) -> np.ndarray:
    small = np.abs(d) < DENOM_GUARD
    out = d.copy()
    out[small] = np.where(d[small] < 0.0, -DENOM_GUARD, DENOM_GUARD)
    return out


def diag_tda(de: np.ndarray, r: np.ndarray, shifts: np.ndarray) -> np.ndarray:
    """(de - Omega_n)^(-1) R_n for each column n.  r: (N, n), shifts: (n,)."""
    return r / _guard(de[:, None] - shifts[None, :])


def diag_pair(de: np.ndarray, r1: np.ndarray, r2: np.ndarray, shifts: np.ndarray):
    """Solve [[de, -s], [-s, de]] (d1; d2) = (r1; r2) elementwise, per column.

    d1 = (de r1 + s r2) / (de^2 - s^2), d2 = (s r1 + de r2) / (de^2 - s^2).
    """
    dm = _guard(de[:, None] - shifts[None, :])
    dp = de[:, None] + shifts[None, :]
    den = dm * dp
    d1 = (de[:, None] * r1 + shifts[None, :] * r2) / den
    d2 = (shifts[None, :] * r1 + de[:, None] * r2) / den
    return d1, d2


def _small_solve(mat: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    try:
        return np.linalg.solve(mat, rhs)
    except np.linalg.LinAlgError:
        return np.linalg.lstsq(mat, rhs, rcond=None)[0]


def inner_solve_tda(apply_t, de, r, shifts, tol=1e-2, max_iter=20):
    """Approximately solve (T - s_n) v_n = r_n for all columns n together.

    Returns (v, n_mv, n_iter): v (N, nrhs) approximates (T - s_n)^(-1) r_n,
    n_mv counts the columns multiplied by T, n_iter the block products.
    """
    nrm = np.linalg.norm(r, axis=0)
    nrm[nrm == 0.0] = 1.0
    rh = r / nrm[None, :]
    nrhs = r.shape[1]
    u = orthonormalize(diag_tda(de, rh, shifts))
    tu = apply_t(u)
    n_mv, n_iter = u.shape[1], 1
    sol = np.zeros_like(rh)
    done = np.zeros(nrhs, dtype=bool)
    while True:
        t = u.T @ tu
        t = 0.5 * (t + t.T)
        g = u.T @ rh
        rho = np.zeros_like(rh)
        for n in range(nrhs):
            if done[n]:
                continue
            y = _small_solve(t - shifts[n] * np.eye(t.shape[0]), g[:, n])
            sol[:, n] = u @ y
            rho[:, n] = tu @ y - shifts[n] * sol[:, n] - rh[:, n]
            if np.linalg.norm(rho[:, n]) < tol:
                done[n] = True
        if done.all() or n_iter >= max_iter:
            break
        act = np.where(~done)[0]
        un = orthonormalize(diag_tda(de, rho[:, act], shifts[act]), u)
        if un.shape[1] == 0:
            break
        u = np.hstack([u, un])
        tu = np.hstack([tu, apply_t(un)])
        n_mv += un.shape[1]
        n_iter += 1
    return sol * nrm[None, :], n_mv, n_iter


def inner_solve_pair(apply_tpm, de, r1, r2, shifts, tol=1e-2, max_iter=20):
    """Approximately solve [[T+, -s_n], [-s_n, T-]] (d1; d2) = (r1; r2) per column.

    apply_tpm(x) -> (T+ x, T- x).  Returns (d1, d2, n_mv, n_iter).
    """
    nrm = np.sqrt(np.sum(r1 * r1, axis=0) + np.sum(r2 * r2, axis=0))
    nrm[nrm == 0.0] = 1.0
    h1, h2 = r1 / nrm[None, :], r2 / nrm[None, :]
    nrhs = r1.shape[1]
    e1, e2 = diag_pair(de, h1, h2, shifts)
    u = orthonormalize(np.hstack([e1, e2]))
    tp, tm = apply_tpm(u)
    n_mv, n_iter = u.shape[1], 1
    s1 = np.zeros_like(h1)
    s2 = np.zeros_like(h2)
    done = np.zeros(nrhs, dtype=bool)
    while True:
        m = u.shape[1]
        ap = u.T @ tp
        ap = 0.5 * (ap + ap.T)
        am = u.T @ tm
        am = 0.5 * (am + am.T)
        g1, g2 = u.T @ h1, u.T @ h2
        rho1 = np.zeros_like(h1)
        rho2 = np.zeros_like(h2)
        for n in range(nrhs):
            if done[n]:
                continue
            s = shifts[n]
            big = np.block([[ap, -s * np.eye(m)], [-s * np.eye(m), am]])
            yy = _small_solve(big, np.concatenate([g1[:, n], g2[:, n]]))
            y, yp = yy[:m], yy[m:]
            s1[:, n], s2[:, n] = u @ y, u @ yp
            rho1[:, n] = tp @ y - s * s2[:, n] - h1[:, n]
            rho2[:, n] = tm @ yp - s * s1[:, n] - h2[:, n]
            if np.sqrt(rho1[:, n] @ rho1[:, n] + rho2[:, n] @ rho2[:, n]) < tol:
                done[n] = True
        if done.all() or n_iter >= max_iter:
            break
        act = np.where(~done)[0]
        d1, d2 = diag_pair(de, rho1[:, act], rho2[:, act], shifts[act])
        un = orthonormalize(np.hstack([d1, d2]), u)
        if un.shape[1] == 0:
            break
        u = np.hstack([u, un])
        a, b = apply_tpm(un)
        tp, tm = np.hstack([tp, a]), np.hstack([tm, b])
        n_mv += un.shape[1]
        n_iter += 1
    return s1 * nrm[None, :], s2 * nrm[None, :], n_mv, n_iter
