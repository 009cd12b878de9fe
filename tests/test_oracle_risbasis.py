"""Pins of the oracle's auxiliary-basis tensors built from a molecule
(Sec. 2.2.2, Eq. TDDFT-ris_approx and the exponent rule alpha_A = theta /
R_A^2; the (d, s) design of Sec. 3.2).

* Gaussian charge distributions: the Coulomb integral of two normalised s
  Gaussians is erf(sqrt(ab/(a+b)) R) / R (electrostatics, not the Hermite
  recursion under test);
* p and d functions are derivatives of s functions with respect to their
  centre: every p and d integral (three-centre and metric) must equal the
  central finite difference of s integrals;
* (P|Q) is symmetric positive definite;
* one-centre exactness: on a single atom, an auxiliary basis holding every
  product of the atomic orbitals reproduces the exact four-index integrals
  (closed form for one-centre s Gaussians);
* rotational invariance of the RI integrals sum_P B^P_pq B^P_rs (p and d
  shells are only invariant as whole shells);
* the (d, s) split: the leading rows of the s, p, d tensor are the tensor of
  the s functions alone;
* the molecule's response problem: symmetric operators, A +- B positive
  definite, and the rid preconditioner reaching the dense roots.
Planted mistakes in the Hermite expansion and in the sign of the second
centre's derivatives fail the finite-difference pins.  (The lowering term of
the Hermite recursion cancels in every real d function of the chosen set, so
dropping it is not a mistake these functions can show.)
"""

import math

import numpy as np
import pytest

from oracle import eigen_rpa, eigen_tda
from oracle import operators as ops
from oracle import risbasis as rb
from synth import make_molecule


def small_molecule(seed=4):
    return make_molecule(6, 5, 15, seed=seed)


def norm_s(a):
    return (a / math.pi) ** 1.5  # unit charge


def test_s_s_coulomb_is_the_gaussian_charge_interaction():
    s = {(0, 0, 0): 1.0}
    for a, c, dist in ((0.7, 1.3, 2.1), (0.2, 5.0, 0.4), (3.0, 3.0, 1e-12), (0.05, 0.09, 7.5)):
        got = rb.coulomb_hermite(s, a, np.array([0.0, 0.0, 0.0]), s, c, np.array([0.0, 0.0, dist]))
        got *= norm_s(a) * norm_s(c)
        k = math.sqrt(a * c / (a + c))
        ref = math.erf(k * dist) / dist if dist > 1e-9 else 2.0 * k / math.sqrt(math.pi)
        assert abs(float(got) - ref) < 1e-12 * ref, (a, c, dist, float(got), ref)


def _s_three_center(mol, centre, c):
    """(mu nu| s_C) for all AO pairs (the finite-difference building block)."""
    p, pc, pref = rb.ao_pairs(mol)
    s = {(0, 0, 0): 1.0}
    return pref * rb.coulomb_hermite(s, p, pc, s, c, np.asarray(centre, dtype=np.float64))


def check_derivatives(mol, h=1e-4, tol=2e-6):
    """Every p and d three-centre integral, and a p-p and a d-s metric
    element, against central differences of s integrals."""
    C = np.array([0.3, -0.8, 1.1])
    c = 0.9
    f = lambda dC: _s_three_center(mol, C + dC, c)
    e = np.eye(3)
    g = {}
    for i in range(3):
        g[i] = (f(h * e[i]) - f(-h * e[i])) / (2 * h)
    g2 = {}
    for i in range(3):
        for j in range(3):
            g2[i, j] = (f(h * (e[i] + e[j])) - f(h * (e[i] - e[j])) - f(h * (-e[i] + e[j])) + f(-h * (e[i] + e[j]))) / (4 * h * h)
    s0 = f(np.zeros(3))
    scale = np.abs(s0).max()
    q = 1.0 / (2.0 * c)
    fd = {
        (1, 0): q * g[0], (1, 1): q * g[1], (1, 2): q * g[2],
        (2, 0): q * q * g2[0, 1], (2, 1): q * q * g2[0, 2], (2, 2): q * q * g2[1, 2],
        (2, 3): q * q * (g2[0, 0] - g2[1, 1]),
        (2, 4): q * q * (2 * g2[2, 2] - g2[0, 0] - g2[1, 1]),
    }
    p, pc, pref = rb.ao_pairs(mol)
    s = {(0, 0, 0): 1.0}
    for (l, i), ref in fd.items():
        hc = rb.hermite_expansion(rb.SHELL_FUNCS[l][i], c)
        got = pref * rb.coulomb_hermite(s, p, pc, hc, c, C)
        if np.abs(got - ref).max() > tol * scale:
            return False
    # metric: (x_A e^{-a} | x_C e^{-c}) = q_a q_c d/dA_x d/dC_x (s_A|s_C)
    A, a = np.array([-0.4, 0.2, 0.5]), 0.6
    qa = 1.0 / (2.0 * a)
    ss = lambda dA, dC: float(rb.coulomb_hermite(s, a, A + dA, s, c, C + dC))
    mixed = (ss(h * e[0], h * e[0]) - ss(h * e[0], -h * e[0]) - ss(-h * e[0], h * e[0]) + ss(-h * e[0], -h * e[0])) / (4 * h * h)
    px_a, px_c = rb.hermite_expansion(rb.SHELL_FUNCS[1][0], a), rb.hermite_expansion(rb.SHELL_FUNCS[1][0], c)
    got = float(rb.coulomb_hermite(px_a, a, A, px_c, c, C))
    if abs(got - qa * q * mixed) > tol * abs(ss(0 * e[0], 0 * e[0])):
        return False
    # (d_xy at A | s at C) = qa^2 d^2/dA_x dA_y (s_A|s_C)
    dxy = (ss(h * (e[0] + e[1]), 0 * e[0]) - ss(h * (e[0] - e[1]), 0 * e[0]) - ss(h * (e[1] - e[0]), 0 * e[0])
           + ss(-h * (e[0] + e[1]), 0 * e[0])) / (4 * h * h)
    got = float(rb.coulomb_hermite(rb.hermite_expansion(rb.SHELL_FUNCS[2][0], a), a, A, s, c, C))
    return abs(got - qa * qa * dxy) <= tol * abs(ss(0 * e[0], 0 * e[0]))


def test_p_and_d_integrals_are_centre_derivatives_of_s_integrals():
    assert check_derivatives(small_molecule())


def test_derivative_pin_rejects_planted_mistakes(monkeypatch):
    mol = small_molecule()
    good_1d = rb.hermite_1d

    def wrong_step(i, a):  # x_A Lambda_t taken as Lambda_{t+1} / a (factor 2 lost)
        e = [1.0]
        for _ in range(i):
            nxt = [0.0] * (len(e) + 1)
            for t, c in enumerate(e):
                nxt[t + 1] += c / a
                if t > 0:
                    nxt[t - 1] += t * c
            e = nxt
        return e

    monkeypatch.setattr(rb, "hermite_1d", wrong_step)
    assert not check_derivatives(mol)
    monkeypatch.setattr(rb, "hermite_1d", good_1d)
    good = rb.coulomb_hermite

    def no_sign(ha, a, A, hc, c, C):  # second centre's derivatives without (-1)^(tau+nu+phi)
        lmax = max(sum(k) for k in ha) + max(sum(k) for k in hc)
        aa = np.asarray(a, dtype=np.float64)
        r = rb.hermite_r(lmax, aa * c / (aa + c), np.asarray(A, dtype=np.float64) - np.asarray(C, dtype=np.float64))
        acc = 0.0
        for (t, u, v), ca in ha.items():
            for (tt, uu, vv), cc in hc.items():
                acc = acc + ca * cc * r[(t + tt, u + uu, v + vv)]
        return 2.0 * math.pi ** 2.5 / (aa * c * np.sqrt(aa + c)) * acc

    monkeypatch.setattr(rb, "coulomb_hermite", no_sign)
    assert not check_derivatives(mol)
    monkeypatch.setattr(rb, "coulomb_hermite", good)
    assert check_derivatives(mol)


def test_metric_symmetric_positive_definite():
    mol = small_molecule()
    for shells, per_atom in ((rb.minimal_shells(mol), 9), (rb.full_shells(mol), 19)):
        funcs, kinds = rb.aux_functions(mol, shells)
        assert len(funcs) == per_atom * mol.natom  # s, p, d: 9 per atom; the full basis 19
        j = rb.metric(funcs, kinds)
        np.testing.assert_allclose(j, j.T, rtol=1e-12, atol=1e-14 * np.abs(j).max())
        assert np.linalg.eigvalsh(0.5 * (j + j.T)).min() > 0.0


def test_one_centre_products_in_the_basis_make_ri_exact():
    """One atom; the auxiliary s exponents are every sum e_k + e_l of two
    atomic-orbital exponents, so every product of two atomic orbitals lies
    in the auxiliary space and RI is exact.  The four-index integrals of
    one-centre s Gaussians have the closed form N^4 2 pi^(5/2) / (p q
    sqrt(p + q)) (p, q the pair exponent sums)."""
    from synth.molecule import Molecule

    ex = np.array([0.4, 1.1, 3.2])
    pairs = sorted({round(a + b, 12) for a in ex for b in ex})
    mol = Molecule(coords=np.zeros((1, 3)), radius=np.array([1.0]), ao_count=np.array([3], dtype=np.int32),
                   ao_exp=ex, mo=np.eye(3), eps_occ=np.array([-0.5]), eps_vir=np.array([0.5, 0.7]), no=1, nv=2,
                   kappa=1.0, shell_atom=np.zeros(len(pairs), dtype=np.int32),
                   shell_l=np.zeros(len(pairs), dtype=np.int32), shell_exp=np.array(pairs))
    b, _ = rb.ri_tensor(mol, rb.full_shells(mol))
    ri = np.einsum("Ppq,Prs->pqrs", b, b)
    n = (2.0 * ex / math.pi) ** 0.75
    exact = np.empty((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    p, q = ex[i] + ex[j], ex[k] + ex[l]
                    exact[i, j, k, l] = n[i] * n[j] * n[k] * n[l] * 2.0 * math.pi ** 2.5 / (p * q * math.sqrt(p + q))
    np.testing.assert_allclose(ri, exact, rtol=1e-9)


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


@pytest.mark.parametrize("lmax", [1, 2])
def test_ri_integrals_are_rotation_invariant(lmax):
    mol = small_molecule()
    shells = lambda m: rb.minimal_shells(m, 0.6, lmax)
    b, _ = rb.ri_tensor(mol, shells(mol))
    mol2 = mol.rotated(_rotation(3), shift=(0.5, -1.0, 2.0))
    b2, _ = rb.ri_tensor(mol2, shells(mol2))
    nmo = mol.no + mol.nv
    g = b.reshape(b.shape[0], -1).T @ b.reshape(b.shape[0], -1)
    g2 = b2.reshape(b2.shape[0], -1).T @ b2.reshape(b2.shape[0], -1)
    assert g.shape == (nmo * nmo, nmo * nmo)
    np.testing.assert_allclose(g2, g, atol=1e-11 * np.abs(g).max())


def test_rotation_pin_sees_an_incomplete_shell():
    """Dropping one d function of every shell breaks the invariance."""
    mol = small_molecule()
    saved = rb.SHELL_FUNCS[2]
    try:
        rb.SHELL_FUNCS[2] = saved[:4]
        b, _ = rb.ri_tensor(mol, rb.minimal_shells(mol))
        mol2 = mol.rotated(_rotation(3))
        b2, _ = rb.ri_tensor(mol2, rb.minimal_shells(mol2))
    finally:
        rb.SHELL_FUNCS[2] = saved
    g = b.reshape(b.shape[0], -1).T @ b.reshape(b.shape[0], -1)
    g2 = b2.reshape(b2.shape[0], -1).T @ b2.reshape(b2.shape[0], -1)
    assert np.abs(g2 - g).max() > 1e-6 * np.abs(g).max()


def test_leading_rows_are_the_s_only_tensor():
    mol = small_molecule()
    b, n_s = rb.ri_tensor(mol, rb.minimal_shells(mol, 0.6, 2))
    bs, n_s2 = rb.ri_tensor(mol, rb.minimal_shells(mol, 0.6, 0))
    assert n_s == n_s2 == mol.natom
    np.testing.assert_allclose(b[:n_s], bs, atol=1e-12 * np.abs(bs).max())
    assert b.shape[0] == 9 * mol.natom


@pytest.mark.parametrize("mode", ["tda", "rpa"])
def test_molecule_problem_rid_reaches_dense_roots(mode):
    mol = small_molecule()
    op = rb.molecule_problem(mol)
    eye = np.eye(op.n)
    a = ops.apply_a(op, eye)
    apb, amb = ops.apply_apb_amb(op, eye)
    t = ops.apply_t(op, eye)
    for m in (a, apb, amb, t):
        np.testing.assert_allclose(m, m.T, atol=1e-13 * np.abs(m).max())
    assert np.linalg.eigvalsh(0.5 * (amb + amb.T)).min() > 0 and np.linalg.eigvalsh(0.5 * (apb + apb.T)).min() > 0
    if mode == "tda":
        ref = np.linalg.eigvalsh(0.5 * (a + a.T))[:4]
        res = eigen_tda(op, 4, "ris", tol=1e-9)
    else:
        ev, u = np.linalg.eigh(0.5 * (amb + amb.T))
        s = (u * np.sqrt(ev)) @ u.T
        ref = np.sqrt(np.linalg.eigvalsh(s @ apb @ s))[:4]
        res = eigen_rpa(op, 4, "ris", tol=1e-9)
    assert res.converged
    np.testing.assert_allclose(res.omega, ref, atol=1e-10)
