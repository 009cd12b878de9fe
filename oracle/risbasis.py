"""Auxiliary-basis RI tensors from a molecule (test infrastructure only).

Sec. 2.2.2 and Eq. TDDFT-ris_approx: the ris model approximates the
electron-repulsion integrals by resolution of the identity in a minimal
auxiliary basis, (pq|rs) ~ sum_PQ (pq|P) [(P|Q)^-1]_PQ (Q|rs), with one
Gaussian shell of each angular momentum up to l_max on every atom and the
exponent alpha_A = theta / R_A^2 of the atom's radius R_A (the paper's best
preconditioner, rid, uses s, p and d shells with theta = 0.6 for the Coulomb
part and only the s shells for exchange, Sec. 3.2).  The same construction
with a larger auxiliary basis gives the "full" tensor of the operator A.

The integrals here follow McMurchie and Davidson (J. Comput. Phys. 26, 218
(1978)): every function is expanded in Hermite Gaussians
Lambda_tuv = d^t/dA_x^t d^u/dA_y^u d^v/dA_z^v exp(-a |r - A|^2), and the
Coulomb integral of two Hermite Gaussians (exponents a, c at A, C) is
  2 pi^(5/2) / (a c sqrt(a + c)) (-1)^(tau+nu+phi) R_{t+tau, u+nu, v+phi},
with R_tuv the Hermite integrals of the Boys function F_n built by the
recursion R^(n)_{t+1,u,v} = t R^(n+1)_{t-1,u,v} + X R^(n+1)_{t,u,v} from
R^(n)_000 = (-2 omega)^n F_n(omega |A - C|^2), omega = a c / (a + c).
Atomic orbitals are s Gaussians, so a pair mu nu is one Gaussian (exponent
a + b at the weighted centre, Gaussian product theorem) and a three-centre
integral (mu nu|P) is a two-centre integral of that product with P.

The tensor is factored with the Cholesky factor of the metric: with
(P|Q) = L L^T, B = L^-1 K, K^P_pq = (pq|P), so that B^T B = K^T (P|Q)^-1 K
(Eq. pqrs_approx with the metric folded in).  The auxiliary functions are
ordered s shells first; because L is lower triangular, the leading rows of
B are then exactly the tensor of the s functions alone -- the exchange part
of the (d, s) design -- while all rows give the s, p, d tensor of the
Coulomb part.  Finally B is multiplied by sqrt(kappa) (the molecule's scale
of the Coulomb operator).

Readings: real solid-harmonic d functions in the (unnormalised) order xy,
xz, yz, x^2 - y^2, 2 z^2 - x^2 - y^2 (five per shell, so s, p, d give the
nine functions per atom of the (d, s) design); functions are not normalised
(B does not depend on the scale of an auxiliary function, only on the
space the functions span and their order); atomic orbitals are normalised
s Gaussians.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import gammainc, gamma

# Cartesian monomials (powers of x, y, z) and coefficients of the real
# functions of one shell, in the order used for the auxiliary index
SHELL_FUNCS = {
    0: [[((0, 0, 0), 1.0)]],
    1: [[((1, 0, 0), 1.0)], [((0, 1, 0), 1.0)], [((0, 0, 1), 1.0)]],
    2: [[((1, 1, 0), 1.0)], [((1, 0, 1), 1.0)], [((0, 1, 1), 1.0)],
        [((2, 0, 0), 1.0), ((0, 2, 0), -1.0)],
        [((0, 0, 2), 2.0), ((2, 0, 0), -1.0), ((0, 2, 0), -1.0)]],
}


def boys(nmax: int, t: np.ndarray) -> np.ndarray:
    """F_n(t) = int_0^1 u^(2n) exp(-t u^2) du for n = 0..nmax (rows)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty((nmax + 1,) + t.shape)
    small = t < 1e-8
    ts = np.where(small, 1.0, t)
    for n in range(nmax + 1):
        a = n + 0.5
        # lower incomplete gamma: gamma(a) * P(a, t) = 2 t^a F_n(t)
        big = gamma(a) * gammainc(a, ts) / (2.0 * ts ** a)
        # series for tiny t: sum_k (-t)^k / (k! (2n + 2k + 1))
        ser = 1.0 / (2 * n + 1) - t / (2 * n + 3) + t * t / (2.0 * (2 * n + 5))
        out[n] = np.where(small, ser, big)
    return out


def hermite_r(lmax: int, omega: np.ndarray, x: np.ndarray) -> dict:
    """R_tuv(omega, X) for t + u + v <= lmax; x: (..., 3) separation A - C.

    Returns {(t, u, v): array}.  Built by the McMurchie-Davidson recursion
    (module docstring)."""
    omega = np.asarray(omega, dtype=np.float64)
    r2 = np.sum(x * x, axis=-1)
    f = boys(lmax, omega * r2)
    # r[n][(t, u, v)] = R^(n)_tuv
    r = [{(0, 0, 0): (-2.0 * omega) ** n * f[n]} for n in range(lmax + 1)]
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    for order in range(1, lmax + 1):
        for n in range(lmax - order + 1):
            for t in range(order + 1):
                for u in range(order - t + 1):
                    v = order - t - u
                    if t > 0:
                        val = X * r[n + 1][(t - 1, u, v)]
                        if t > 1:
                            val = val + (t - 1) * r[n + 1][(t - 2, u, v)]
                    elif u > 0:
                        val = Y * r[n + 1][(t, u - 1, v)]
                        if u > 1:
                            val = val + (u - 1) * r[n + 1][(t, u - 2, v)]
                    else:
                        val = Z * r[n + 1][(t, u, v - 1)]
                        if v > 1:
                            val = val + (v - 1) * r[n + 1][(t, u, v - 2)]
                    r[n][(t, u, v)] = val
    return r[0]


def hermite_1d(i: int, a: float) -> list:
    """E^i_t with x_A^i exp(-a x_A^2) = sum_t E^i_t Lambda_t(a, A)."""
    e = [1.0]
    for _ in range(i):
        nxt = [0.0] * (len(e) + 1)
        for t, c in enumerate(e):
            nxt[t + 1] += c / (2.0 * a)      # x_A Lambda_t = Lambda_{t+1} / (2a) + t Lambda_{t-1}
            if t > 0:
                nxt[t - 1] += t * c
        e = nxt
    return e


def hermite_expansion(terms, a: float) -> dict:
    """{(t, u, v): coefficient} of sum_k c_k x^i y^j z^k exp(-a r_A^2)."""
    out = {}
    for (i, j, k), c in terms:
        ex, ey, ez = hermite_1d(i, a), hermite_1d(j, a), hermite_1d(k, a)
        for t, cx in enumerate(ex):
            for u, cy in enumerate(ey):
                for v, cz in enumerate(ez):
                    # structural zeros stay the scalar 0.0 (exponents may be arrays)
                    if not any(isinstance(w, float) and w == 0.0 for w in (cx, cy, cz)):
                        out[(t, u, v)] = out.get((t, u, v), 0.0) + c * cx * cy * cz
    return out


def coulomb_hermite(ha: dict, a, A, hc: dict, c: float, C) -> np.ndarray:
    """Coulomb integral of sum ha Lambda(a, A) and sum hc Lambda(c, C).

    a and A may be arrays (a batch of first functions, A of shape (n, 3))."""
    a = np.asarray(a, dtype=np.float64)
    lmax = max(sum(k) for k in ha) + max(sum(k) for k in hc)
    omega = a * c / (a + c)
    x = np.asarray(A, dtype=np.float64) - np.asarray(C, dtype=np.float64)
    r = hermite_r(lmax, omega, x)
    acc = 0.0
    for (t, u, v), ca in ha.items():
        for (tt, uu, vv), cc in hc.items():
            acc = acc + ca * cc * (-1.0) ** (tt + uu + vv) * r[(t + tt, u + uu, v + vv)]
    return 2.0 * math.pi ** 2.5 / (a * c * np.sqrt(a + c)) * acc


def aux_functions(mol, shells):
    """The auxiliary functions of a list of shells (atom, l, exponent),
    ordered: all s shells, then all p, then all d (shells in list order,
    functions in SHELL_FUNCS order).  Returns a list of (centre, exponent,
    Hermite expansion, l) and the kind (l, index in shell) of each."""
    out, kinds = [], []
    for l in (0, 1, 2):
        for atom, ll, e in shells:
            if ll != l:
                continue
            for i, terms in enumerate(SHELL_FUNCS[l]):
                out.append((np.asarray(mol.coords[atom], dtype=np.float64), float(e), hermite_expansion(terms, e), l))
                kinds.append((l, i))
    return out, kinds


def minimal_shells(mol, theta: float = 0.6, lmax: int = 2):
    """One shell of each l <= lmax per atom, exponent theta / R_A^2 (Sec. 2.2.2)."""
    return [(a, l, theta / mol.radius[a] ** 2) for a in range(mol.natom) for l in range(lmax + 1)]


def full_shells(mol):
    return [(int(a), int(l), float(e)) for a, l, e in zip(mol.shell_atom, mol.shell_l, mol.shell_exp)]


def ao_pairs(mol):
    """Exponent, centre and prefactor of every AO product mu nu (Gaussian
    product theorem; normalised s functions), arrays of shape (nao, nao)."""
    nao = mol.nao
    atom_of = np.repeat(np.arange(mol.natom), mol.ao_count)
    cen = mol.coords[atom_of]
    a = mol.ao_exp[:, None]
    b = mol.ao_exp[None, :]
    p = a + b
    centre = (a[..., None] * cen[:, None, :] + b[..., None] * cen[None, :, :]) / p[..., None]
    d2 = np.sum((cen[:, None, :] - cen[None, :, :]) ** 2, axis=-1)
    norm = (2.0 * mol.ao_exp / np.pi) ** 0.75
    pref = norm[:, None] * norm[None, :] * np.exp(-a * b / p * d2)
    assert p.shape == (nao, nao)
    return p, centre, pref


def three_center(mol, funcs) -> np.ndarray:
    """(mu nu|P) for every AO pair and auxiliary function: (naux, nao, nao)."""
    p, centre, pref = ao_pairs(mol)
    out = np.empty((len(funcs), mol.nao, mol.nao))
    s = {(0, 0, 0): 1.0}
    for q, (C, c, hc, _) in enumerate(funcs):
        out[q] = pref * coulomb_hermite(s, p, centre, hc, c, C)
    return out


def metric(funcs, kinds) -> np.ndarray:
    """(P|Q): (naux, naux).  kinds[r] = (l, index in its shell) of function r;
    the second functions of one kind are taken together (their Hermite
    coefficients as arrays over the exponents)."""
    n = len(funcs)
    j = np.empty((n, n))
    groups = {}
    for r, kd in enumerate(kinds):
        groups.setdefault(kd, []).append(r)
    for (l, i), idx in groups.items():
        idx = np.array(idx)
        cen = np.array([funcs[r][0] for r in idx])
        ex = np.array([funcs[r][1] for r in idx])
        hc = hermite_expansion(SHELL_FUNCS[l][i], ex)
        for q, (A, a, ha, _) in enumerate(funcs):
            # (f_q | g_r) with the roles swapped: (g_r | f_q), batch first
            j[q, idx] = coulomb_hermite(hc, ex, cen, ha, a, A)
    return j


def ri_tensor(mol, shells):
    """B = sqrt(kappa) L^-1 K with (P|Q) = L L^T and K^P_pq = (pq|P), over
    the molecular orbitals.  Returns (b (naux, nmo, nmo), number of s
    functions)."""
    funcs, kinds = aux_functions(mol, shells)
    x = three_center(mol, funcs)
    k = np.einsum("mp,Pmn,nq->Ppq", mol.mo, x, mol.mo, optimize=True)
    j = metric(funcs, kinds)
    l = np.linalg.cholesky(0.5 * (j + j.T))
    naux, nmo = k.shape[0], k.shape[1]
    b = np.linalg.solve(l, k.reshape(naux, nmo * nmo)).reshape(naux, nmo, nmo)
    n_s = sum(1 for f in funcs if f[3] == 0)
    return math.sqrt(mol.kappa) * b, n_s


def blocks(mol, b):
    """(b_ia, b_ij, b_ab) of a tensor over all orbitals (occupied first)."""
    no = mol.no
    return (np.ascontiguousarray(b[:, :no, no:]), np.ascontiguousarray(b[:, :no, :no]),
            np.ascontiguousarray(b[:, no:, no:]))


def molecule_problem(mol, theta: float = 0.6, lmax: int = 2, a_x: float = 0.25, t_cut: float = np.inf):
    """The response problem of a molecule: A from the full auxiliary basis,
    the ris model T from the minimal one (Coulomb: all functions; exchange:
    the s functions).  Returns an OracleProblem."""
    from .operators import OracleProblem

    bf, _ = ri_tensor(mol, full_shells(mol))
    br, n_s = ri_tensor(mol, minimal_shells(mol, theta, lmax))
    fia, fij, fab = blocks(mol, bf)
    ria, rij, rab = blocks(mol, br)
    return OracleProblem(no=mol.no, nv=mol.nv, eps_occ=mol.eps_occ, eps_vir=mol.eps_vir, b_ia=fia, b_ij=fij,
                         b_ab=fab, a_x=a_x, bris_ia=ria, bris_ij=rij, bris_ab=rab, naux_ris_k=n_s, t_cut=t_cut)
