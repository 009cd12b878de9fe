"""Dynamic polarizability by a preconditioned Krylov linear solve (Eq. TDDFT_polar).

With dipole right-hand sides mu_vo = mu_ov = P, the polarizability of
Eq. TDDFT_polar reduces, through Z = X + Y and Z' = X - Y, to

    alpha_uv(w) = -2 P_u^T U_v,   (A+B) U - w U' = -P_v,   (A-B) U' - w U = 0,

and for w = 0 to alpha_uv(0) = 2 P_u^T (A+B)^(-1) P_v.  All right-hand sides
and frequencies of one request share one subspace V (both components of every
solution are expanded in it).  Each iteration solves the projected 2m x 2m
system [[a_+, -w], [-w, a_-]] (y; y') = (-V^T P_v; 0) per (rhs, frequency)
pair, forms the residual pair R = (A+B) V y - w V y' + P_v,
R' = (A-B) V y' - w V y, and stops when sqrt(||R||^2 + ||R'||^2) / ||P_v||
is below the threshold for every pair.  Unconverged pairs add their
preconditioned residual pair (the diagonal 2x2 form, or the inner ris solve of
the 2x2 system with shift w).  The initial subspace is the diagonal (or ris,
solved to 1e-3) solution of the same 2x2 system with right-hand side (-P, 0).
"""

from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from . import operators as ops
from .linalg import orthonormalize
from .precond import diag_pair, inner_solve_pair


@dataclasses.dataclass
class ResponseResult:
    alpha: np.ndarray    # (nfreq, nrhs, nrhs): alpha[f, u, v]
    u: np.ndarray        # (N, nrhs, nfreq)
    resid: np.ndarray    # (nrhs, nfreq) relative residuals
    n_iter: int
    n_mv: int
    n_inner_mv: int
    history: List[float]
    status: str

    @property
    def converged(self) -> bool:
        return self.status == "ok"


def _sym(a):
    return 0.5 * (a + a.T)


def polarizability(prob: ops.OracleProblem, p: np.ndarray, omegas, precond: str = "diag",
                   tol: float = 1e-5, max_iter: int = 100, inner_tol: float = 1e-2,
                   inner_max: int = 20, init_tol: float = 1e-3, init_max: int = 20) -> ResponseResult:
    """alpha(w) for dipole right-hand sides p (N, nrhs) at frequencies `omegas`."""
    omegas = np.asarray(omegas, dtype=np.float64)
    nrhs, nf = p.shape[1], len(omegas)
    de = prob.delta_eps()
    apply_pm = lambda x: ops.apply_apb_amb(prob, x)
    apply_tpm = lambda x: ops.apply_tpm(prob, x)
    # one column per (rhs, frequency) pair, rhs fastest
    rhs = np.ascontiguousarray(np.concatenate([p for _ in range(nf)], axis=1))
    sh = np.repeat(omegas, nrhs)
    pn = np.linalg.norm(rhs, axis=0)
    zero = np.zeros_like(rhs)

    n_inner = 0
    if precond == "diag":
        u0, u0p = diag_pair(de, -rhs, zero, sh)
    elif precond == "ris":
        u0, u0p, n_inner, _ = inner_solve_pair(apply_tpm, de, -rhs, zero, sh, init_tol, init_max)
    else:
        raise ValueError(precond)
    v = orthonormalize(np.hstack([u0, u0p]))
    pv, mv = apply_pm(v)
    n_iter, n_mv = 1, v.shape[1]
    history = []
    npair = rhs.shape[1]
    while True:
        m = v.shape[1]
        ap, am = _sym(v.T @ pv), _sym(v.T @ mv)
        g = v.T @ rhs
        sol = np.zeros((m, npair))
        solp = np.zeros((m, npair))
        for c in range(npair):
            w = sh[c]
            if w == 0.0:
                sol[:, c] = np.linalg.solve(ap, -g[:, c])
            else:
                big = np.block([[ap, -w * np.eye(m)], [-w * np.eye(m), am]])
                yy = np.linalg.solve(big, np.concatenate([-g[:, c], np.zeros(m)]))
                sol[:, c], solp[:, c] = yy[:m], yy[m:]
        uu, uup = v @ sol, v @ solp
        r1 = pv @ sol - uup * sh[None, :] + rhs
        r2 = mv @ solp - uu * sh[None, :]
        rn = np.sqrt(np.sum(r1 * r1, axis=0) + np.sum(r2 * r2, axis=0)) / pn
        history.append(float(rn.max()))
        status = None
        if np.all(rn < tol):
            status = "ok"
        elif n_iter >= max_iter:
            status = "not_converged"
        if status is None:
            act = np.where(rn >= tol)[0]
            if precond == "diag":
                d1, d2 = diag_pair(de, r1[:, act], r2[:, act], sh[act])
            else:
                d1, d2, nmv, _ = inner_solve_pair(apply_tpm, de, r1[:, act], r2[:, act], sh[act],
                                                  inner_tol, inner_max)
                n_inner += nmv
            vn = orthonormalize(np.hstack([d1, d2]), v)
            if vn.shape[1] == 0:
                status = "breakdown"
            else:
                v = np.hstack([v, vn])
                a, b = apply_pm(vn)
                pv, mv = np.hstack([pv, a]), np.hstack([mv, b])
                n_iter += 1
                n_mv += vn.shape[1]
                continue
        ucube = uu.reshape(p.shape[0], nf, nrhs).transpose(0, 2, 1)  # (N, nrhs, nf)
        alpha = np.empty((nf, nrhs, nrhs))
        for f in range(nf):
            alpha[f] = -2.0 * p.T @ ucube[:, :, f]
        return ResponseResult(alpha, ucube, rn.reshape(nf, nrhs).T, n_iter, n_mv, n_inner,
                              history, status)
