"""Response operators in plain NumPy float64 (test infrastructure only).

Notation (Sec. 2.2): i, j occupied; a, b virtual; response index ia -> i*nv + a.
With the XC kernel set to zero and the ERIs factored through a symmetric
three-index tensor, (pq|rs) = sum_P B^P_pq B^P_rs (Eq. pqrs_approx with the
metric folded into B), the orbital-rotation Hessians of Eq. hessian become

    A   = diag(de) + 2 K - a_x W          (Eq. TDA uses A alone)
    B   =            2 K - a_x W'
    A+B = diag(de) + 4 K - a_x (W + W')
    A-B = diag(de)       - a_x (W - W')

with de_ia = eps_a - eps_i, K_{ia,jb} = (ia|jb), W_{ia,jb} = (ij|ab) and
W'_{ia,jb} = (ib|ja).  The A+B line doubles the Coulomb factor printed in
Eq. hessian (which reads 2(ia|jb) for A+B); this follows from A = de + 2K
(restricted singlet) and B = 2K, and agrees with the printed A-B.

Range-separated hybrids (the paper's second functional, wB97X, Sec. 4):
the exact-exchange integrals become a_x (pq|rs) + b_x (pq|rs)^LR, the
long-range (attenuated) integrals factored through a second tensor C,
(pq|rs)^LR = sum_Q C^Q_pq C^Q_rs, so W -> a_x W + b_x W^LR and likewise W'.

The ris model T (Sec. 2.2.2, Eq. TDDFT-ris_approx) has the same structure,
built from the minimal-auxiliary tensor: the Coulomb part uses all of its
rows, the exchange part only the leading ``naux_ris_k`` rows (the (d, s)
split of Sec. 3.2), and exchange integrals that touch a virtual above
eps_HOMO + t_cut or an occupied below eps_LUMO - t_cut are dropped (Sec. 3.1).

Vectors are columns: a block X has shape (N, nvec) with N = no*nv.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class OracleProblem:
    no: int
    nv: int
    eps_occ: np.ndarray
    eps_vir: np.ndarray
    b_ia: np.ndarray  # (naux, no, nv)
    b_ij: np.ndarray  # (naux, no, no)
    b_ab: np.ndarray  # (naux, nv, nv)
    a_x: float
    bris_ia: Optional[np.ndarray] = None
    bris_ij: Optional[np.ndarray] = None
    bris_ab: Optional[np.ndarray] = None
    naux_ris_k: int = 0
    t_cut: float = np.inf
    # range-separated hybrid: weight and long-range tensors (full and ris)
    b_x: float = 0.0
    blr_ia: Optional[np.ndarray] = None
    blr_ij: Optional[np.ndarray] = None
    blr_ab: Optional[np.ndarray] = None
    brislr_ia: Optional[np.ndarray] = None
    brislr_ij: Optional[np.ndarray] = None
    brislr_ab: Optional[np.ndarray] = None

    @classmethod
    def from_arrays(cls, d: dict) -> "OracleProblem":
        """Build from the dict returned by synth.Problem.numpy()."""
        f = lambda k: None if d.get(k) is None else np.ascontiguousarray(d[k], dtype=np.float64)
        return cls(no=int(d["no"]), nv=int(d["nv"]), eps_occ=f("eps_occ"), eps_vir=f("eps_vir"),
                   b_ia=f("b_ia"), b_ij=f("b_ij"), b_ab=f("b_ab"), a_x=float(d["a_x"]),
                   bris_ia=f("bris_ia"), bris_ij=f("bris_ij"), bris_ab=f("bris_ab"),
                   naux_ris_k=int(d.get("naux_ris_k") or 0),
                   t_cut=float(d.get("t_cut", np.inf)),
                   b_x=float(d.get("b_x") or 0.0), blr_ia=f("blr_ia"), blr_ij=f("blr_ij"), blr_ab=f("blr_ab"),
                   brislr_ia=f("brislr_ia"), brislr_ij=f("brislr_ij"), brislr_ab=f("brislr_ab"))

    @property
    def has_lr(self) -> bool:
        return self.b_x != 0.0 and self.blr_ij is not None

    @property
    def n(self) -> int:
        return self.no * self.nv

    def delta_eps(self) -> np.ndarray:
        """de_ia = eps_a - eps_i, flattened to length N (diagonal of Eq. hessian)."""
        return (self.eps_vir[None, :] - self.eps_occ[:, None]).reshape(-1)

    def active_ranges(self):
        """(i0, nv_act) of the exchange cutoff of Sec. 3.1 (energies sorted).

        Active virtuals: eps_a <= eps_HOMO + t_cut; active occupieds:
        eps_i >= eps_LUMO - t_cut.
        """
        homo, lumo = self.eps_occ[-1], self.eps_vir[0]
        nv_act = int(np.sum(self.eps_vir <= homo + self.t_cut))
        i0 = int(np.sum(self.eps_occ < lumo - self.t_cut))
        return i0, nv_act


def _as_cube(x: np.ndarray, no: int, nv: int) -> np.ndarray:
    """(N, nvec) columns -> (nvec, no, nv)."""
    return np.ascontiguousarray(x.T).reshape(x.shape[1], no, nv)


def _as_cols(y: np.ndarray) -> np.ndarray:
    """(nvec, no, nv) -> (N, nvec) columns."""
    return np.ascontiguousarray(y.reshape(y.shape[0], -1).T)


def coulomb(b_ia: np.ndarray, x: np.ndarray) -> np.ndarray:
    """K x with K_{ia,jb} = sum_P B^P_ia B^P_jb.  x: (N, nvec)."""
    naux = b_ia.shape[0]
    bm = b_ia.reshape(naux, -1)
    t = bm @ x              # (naux, nvec): t^P_v = sum_jb B^P_jb x_jb,v
    return bm.T @ t         # sum_P B^P_ia t^P_v


def exchange_w(b_ij: np.ndarray, b_ab: np.ndarray, x: np.ndarray, no: int, nv: int) -> np.ndarray:
    """W x with W_{ia,jb} = (ij|ab) = sum_P B^P_ij B^P_ab.

    (W x)_ia = sum_P sum_j B^P_ij sum_b x_jb B^P_ba; B^P_ab is symmetric.
    """
    xc = _as_cube(x, no, nv)
    out = np.zeros_like(xc)
    for p in range(b_ij.shape[0]):
        s = np.matmul(b_ij[p], xc)          # (nvec, no, nv): sum_j B^P_ij x_jb
        out += np.matmul(s, b_ab[p])        # sum_b s_ib B^P_ba
    return _as_cols(out)


def exchange_wp(b_ia: np.ndarray, x: np.ndarray, no: int, nv: int) -> np.ndarray:
    """W' x with W'_{ia,jb} = (ib|ja) = sum_P B^P_ib B^P_ja.

    (W' x)_ia = sum_P sum_j q^P_ij B^P_ja with q^P_ij = sum_b B^P_ib x_jb.
    """
    xc = _as_cube(x, no, nv)
    out = np.zeros_like(xc)
    for p in range(b_ia.shape[0]):
        q = np.matmul(b_ia[p], xc.transpose(0, 2, 1))   # (nvec, no, no)
        out += np.matmul(q, b_ia[p])                    # (nvec, no, nv)
    return _as_cols(out)


def apply_a(prob: OracleProblem, x: np.ndarray) -> np.ndarray:
    """A x = de x + 2 K x - a_x W x [- b_x W^LR x]  (Eqs. hessian, TDA; f^xc = 0)."""
    de = prob.delta_eps()[:, None]
    y = de * x + 2.0 * coulomb(prob.b_ia, x)
    if prob.a_x != 0.0:
        y -= prob.a_x * exchange_w(prob.b_ij, prob.b_ab, x, prob.no, prob.nv)
    if prob.has_lr:
        y -= prob.b_x * exchange_w(prob.blr_ij, prob.blr_ab, x, prob.no, prob.nv)
    return y


def apply_apb_amb(prob: OracleProblem, x: np.ndarray):
    """((A+B) x, (A-B) x) from one evaluation of K x, W x and W' x (Eq. hessian)."""
    de = prob.delta_eps()[:, None]
    kx = coulomb(prob.b_ia, x)
    wx = np.zeros_like(x)
    wpx = np.zeros_like(x)
    if prob.a_x != 0.0:
        wx += prob.a_x * exchange_w(prob.b_ij, prob.b_ab, x, prob.no, prob.nv)
        wpx += prob.a_x * exchange_wp(prob.b_ia, x, prob.no, prob.nv)
    if prob.has_lr:
        wx += prob.b_x * exchange_w(prob.blr_ij, prob.blr_ab, x, prob.no, prob.nv)
        wpx += prob.b_x * exchange_wp(prob.blr_ia, x, prob.no, prob.nv)
    apb = de * x + 4.0 * kx - (wx + wpx)
    amb = de * x - (wx - wpx)
    return apb, amb


def _ris_exchange_rows(prob: OracleProblem, b_ia, b_ij, b_ab, nk: int, x: np.ndarray, with_wp: bool):
    """(W x, W' x) from rows [0, nk) of (b_ia, b_ij, b_ab), restricted to the
    active block of Sec. 3.1 (every orbital index of the integral active)."""
    no, nv = prob.no, prob.nv
    i0, na = prob.active_ranges()
    xc = _as_cube(x, no, nv)
    xa = xc[:, i0:, :na]
    w = np.zeros_like(xc)
    wp = np.zeros_like(xc)
    for p in range(nk):
        bij = b_ij[p, i0:, i0:]
        bab = b_ab[p, :na, :na]
        w[:, i0:, :na] += np.matmul(np.matmul(bij, xa), bab)
        if with_wp:
            bia = b_ia[p, i0:, :na]
            q = np.matmul(bia, xa.transpose(0, 2, 1))
            wp[:, i0:, :na] += np.matmul(q, bia)
    return _as_cols(w), _as_cols(wp)


def _ris_exchange(prob: OracleProblem, x: np.ndarray, with_wp: bool):
    """Weighted exchange of the ris model: a_x (W_ris, W'_ris) from the leading
    naux_ris_k rows of the ris tensor (Sec. 3.2) plus, for a range-separated
    hybrid, b_x times the same from every row of the long-range ris tensor."""
    w = np.zeros_like(x)
    wp = np.zeros_like(x)
    if prob.a_x != 0.0 and prob.naux_ris_k > 0:
        a, b = _ris_exchange_rows(prob, prob.bris_ia, prob.bris_ij, prob.bris_ab, prob.naux_ris_k, x, with_wp)
        w += prob.a_x * a
        wp += prob.a_x * b
    if prob.b_x != 0.0 and prob.brislr_ij is not None:
        a, b = _ris_exchange_rows(prob, prob.brislr_ia, prob.brislr_ij, prob.brislr_ab, prob.brislr_ij.shape[0], x,
                                  with_wp)
        w += prob.b_x * a
        wp += prob.b_x * b
    return w, wp


def apply_t(prob: OracleProblem, x: np.ndarray) -> np.ndarray:
    """T x for the TDA ris model: de x + 2 K_ris x - a_x W_ris^(t_cut) x [- b_x W_ris^LR x]."""
    de = prob.delta_eps()[:, None]
    w, _ = _ris_exchange(prob, x, with_wp=False)
    return de * x + 2.0 * coulomb(prob.bris_ia, x) - w


def apply_tpm(prob: OracleProblem, x: np.ndarray):
    """(T_+ x, T_- x): the ris model of A+B and A-B."""
    de = prob.delta_eps()[:, None]
    kx = coulomb(prob.bris_ia, x)
    w, wp = _ris_exchange(prob, x, with_wp=True)
    return de * x + 4.0 * kx - (w + wp), de * x - (w - wp)


# ---------------------------------------------------------------------------
# Dense builders for tiny sizes: the Hessians written element by element from
# explicit four-index integrals (pq|rs) = sum_P B^P_pq B^P_rs over the full
# orbital space.  A different route from the factored products above.
# ---------------------------------------------------------------------------

def full_three_index(b_ia, b_ij, b_ab) -> np.ndarray:
    """Assemble B^P_pq over all orbitals (occupied first, then virtual)."""
    naux, no, nv = b_ia.shape
    nmo = no + nv
    b = np.zeros((naux, nmo, nmo))
    b[:, :no, :no] = b_ij
    b[:, :no, no:] = b_ia
    b[:, no:, :no] = b_ia.transpose(0, 2, 1)
    b[:, no:, no:] = b_ab
    return b


def dense_eri(b_full: np.ndarray) -> np.ndarray:
    """(pq|rs) for every orbital quadruple, by explicit loops (tiny sizes only)."""
    naux, nmo, _ = b_full.shape
    eri = np.zeros((nmo, nmo, nmo, nmo))
    for p in range(nmo):
        for q in range(nmo):
            for r in range(nmo):
                for s in range(nmo):
                    acc = 0.0
                    for aux in range(naux):
                        acc += b_full[aux, p, q] * b_full[aux, r, s]
                    eri[p, q, r, s] = acc
    return eri


def dense_hessians(eps_occ, eps_vir, eri, a_x, occ_active=None, vir_active=None, eri_lr=None, b_x=0.0):
    """Dense A and B (N x N) element by element from (pq|rs) (Eq. hessian, f^xc = 0).

    A_{ia,jb} = de_ia d_ij d_ab + 2 (ia|jb) - a_x (ij|ab) [- b_x (ij|ab)^LR]
    B_{ia,jb} =                   2 (ia|jb) - a_x (ib|ja) [- b_x (ib|ja)^LR]
    If active masks are given, the exchange integrals are kept only when all
    four orbitals are active (Sec. 3.1).
    """
    no, nv = len(eps_occ), len(eps_vir)
    n = no * nv
    amat = np.zeros((n, n))
    bmat = np.zeros((n, n))
    for i in range(no):
        for a in range(nv):
            ia = i * nv + a
            for j in range(no):
                for b in range(nv):
                    jb = j * nv + b
                    A = 2.0 * eri[i, no + a, j, no + b]
                    B = 2.0 * eri[i, no + a, j, no + b]
                    keep = True
                    if occ_active is not None:
                        keep = (occ_active[i] and occ_active[j]
                                and vir_active[a] and vir_active[b])
                    if keep:
                        A -= a_x * eri[i, j, no + a, no + b]
                        B -= a_x * eri[i, no + b, j, no + a]
                        if eri_lr is not None:
                            A -= b_x * eri_lr[i, j, no + a, no + b]
                            B -= b_x * eri_lr[i, no + b, j, no + a]
                    if ia == jb:
                        A += eps_vir[a] - eps_occ[i]
                    amat[ia, jb] = A
                    bmat[ia, jb] = B
    return amat, bmat


def sampled_entries(b_ia_rows_i, b_ia_cols_a, b_ij_rows_i, b_ab_cols_a, b_ia, a_x, de_ia, x_cube, i, a):
    """((A+B) x)_ia and ((A-B) x)_ia for one output entry, from Eq. hessian.

    For full-size checks where the whole product is too costly: every term is
    summed straight from its definition over the auxiliary index.
      b_ia_rows_i = B^P_{i b}  (naux, nv)    b_ia_cols_a = B^P_{j a}  (naux, no)
      b_ij_rows_i = B^P_{i j}  (naux, no)    b_ab_cols_a = B^P_{b a}  (naux, nv)
      b_ia: the full (naux, no, nv) tensor (for the Coulomb term)
      x_cube: (no, nv) vector, de_ia = eps_a - eps_i.
    K x   = sum_P B^P_ia sum_jb B^P_jb x_jb
    W x   = sum_P sum_jb B^P_ij B^P_ba x_jb
    W' x  = sum_P sum_jb B^P_ib B^P_ja x_jb
    """
    naux = b_ia.shape[0]
    t = b_ia.reshape(naux, -1) @ x_cube.reshape(-1)          # sum_jb B^P_jb x_jb
    kx = float(b_ia[:, i, a] @ t)
    wx = float(np.sum((b_ij_rows_i @ x_cube) * b_ab_cols_a))     # sum_P sum_b (sum_j B_ij x_jb) B_ba
    wpx = float(np.sum((b_ia_rows_i @ x_cube.T) * b_ia_cols_a))  # sum_P sum_j (sum_b B_ib x_jb) B_ja
    apb = de_ia * x_cube[i, a] + 4.0 * kx - a_x * (wx + wpx)
    amb = de_ia * x_cube[i, a] - a_x * (wx - wpx)
    return apb, amb
