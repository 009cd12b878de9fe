"""Seeded synthetic molecules for building auxiliary-basis tensors from
integrals (test and benchmark inputs; none of the method's arithmetic).

A molecule is a set of atoms with positions and radii, a basis of s-type
Gaussian atomic orbitals on each atom, molecular-orbital coefficients, the
orbital energies of the response problem, and the shells of a "full"
auxiliary basis that stands in for a standard fitting basis.  The
minimal auxiliary basis of the ris model is not part of the input: its
exponents follow from the radii by the method's rule (theta / R_A^2).

Readings (the paper's molecules, basis sets and radius table are not
available here):
* positions: atoms placed one after another at a bond length of
  2.4-3.0 bohr from a randomly chosen earlier atom, in a random direction,
  rejecting placements closer than 2.2 bohr to any atom (a branched,
  molecule-like cluster); about 30 % of the atoms are light (hydrogen-like);
* radii R_A (bohr), stand-ins for a tabulated radius: 1.30 (heavy) and 0.70
  (light);
* atomic orbitals: even-tempered s Gaussians, exponents 0.12 * 3^k (heavy,
  k = 0..n-1) and 0.25 * 3^k (light), n chosen so that there are at least
  as many atomic orbitals as molecular orbitals;
* molecular orbitals: the first no + nv columns of a random orthogonal
  matrix (QR of a Gaussian matrix) -- orthonormal in the Euclidean sense;
  any set of functions gives a positive semidefinite four-index tensor, so
  the response problem stays well defined;
* full auxiliary basis: per atom, s shells with exponents (0.3, 1.5, 7.5) /
  R_A^2, p shells (0.6, 3.0) / R_A^2 and d shells (0.8, 4.0) / R_A^2 (19
  functions per atom);
* orbital energies as in generate.py (occupied U[-1.0, -0.3] Ha, virtual
  U[0.05, 2.0] Ha, sorted);
* kappa: a scale of the Coulomb operator (the integrals are multiplied by
  kappa); 0.07 gives ||B_ia||_2^2 of about 0.5 Ha on the no=20, nv=80
  molecules, the coupling the synthetic tensors of generate.py have.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .generate import counter_normals, counter_uniforms

HEAVY_RADIUS = 1.30
LIGHT_RADIUS = 0.70
FULL_AUX = ((0, (0.3, 1.5, 7.5)), (1, (0.6, 3.0)), (2, (0.8, 4.0)))  # (l, theta multipliers)

_STREAM_GEOM = 21
_STREAM_MO = 22
_STREAM_EPS_OCC = 1
_STREAM_EPS_VIR = 2


@dataclasses.dataclass
class Molecule:
    coords: np.ndarray       # (natom, 3) bohr
    radius: np.ndarray       # (natom,) bohr
    ao_count: np.ndarray     # (natom,) s functions per atom
    ao_exp: np.ndarray       # (nao,) exponents, atom by atom
    mo: np.ndarray           # (nao, no + nv) coefficients
    eps_occ: np.ndarray
    eps_vir: np.ndarray
    no: int
    nv: int
    kappa: float
    shell_atom: np.ndarray   # full auxiliary basis: atom of each shell
    shell_l: np.ndarray      # angular momentum of each shell
    shell_exp: np.ndarray    # exponent of each shell
    seed: int = 0

    @property
    def natom(self) -> int:
        return len(self.radius)

    @property
    def nao(self) -> int:
        return len(self.ao_exp)

    def rotated(self, rot: np.ndarray, shift=(0.0, 0.0, 0.0)) -> "Molecule":
        """The same molecule with its coordinates rotated (and shifted)."""
        d = dataclasses.asdict(self)
        d["coords"] = self.coords @ rot.T + np.asarray(shift)[None, :]
        return Molecule(**d)


def _uniform(seed, stream, start, count):
    return counter_uniforms(seed, stream, start, count).numpy()


def make_molecule(natom: int, no: int, nv: int, seed: int = 0, kappa: float = 0.07) -> Molecule:
    u = _uniform(seed, _STREAM_GEOM, 0, 8 * natom * 64)
    pos = 0
    coords = np.zeros((natom, 3))
    heavy = np.ones(natom, dtype=bool)
    for a in range(1, natom):
        while True:
            base = int(u[pos] * a)
            bond = 2.4 + 0.6 * u[pos + 1]
            cz = 2.0 * u[pos + 2] - 1.0
            phi = 2.0 * np.pi * u[pos + 3]
            pos += 4
            sz = np.sqrt(max(0.0, 1.0 - cz * cz))
            cand = coords[base] + bond * np.array([sz * np.cos(phi), sz * np.sin(phi), cz])
            if np.min(np.linalg.norm(coords[:a] - cand[None, :], axis=1)) >= 2.2:
                coords[a] = cand
                break
        heavy[a] = u[pos] >= 0.3
        pos += 1
    radius = np.where(heavy, HEAVY_RADIUS, LIGHT_RADIUS)
    nmo = no + nv
    per = int(np.ceil(nmo / natom)) + 1
    ao_count = np.full(natom, per, dtype=np.int32)
    ao_exp = np.concatenate([(0.12 if heavy[a] else 0.25) * 3.0 ** np.arange(per) for a in range(natom)])
    nao = len(ao_exp)
    g = counter_normals(seed, _STREAM_MO, 0, nao * nao).numpy().reshape(nao, nao)
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]  # a deterministic sign per column
    mo = np.ascontiguousarray(q[:, :nmo])
    eps_occ = np.sort(-1.0 + 0.7 * _uniform(seed, _STREAM_EPS_OCC, 0, no))
    eps_vir = np.sort(0.05 + 1.95 * _uniform(seed, _STREAM_EPS_VIR, 0, nv))
    sa, sl, se = [], [], []
    for a in range(natom):
        for l, mult in FULL_AUX:
            for m in mult:
                sa.append(a)
                sl.append(l)
                se.append(m / radius[a] ** 2)
    return Molecule(coords=coords, radius=radius, ao_count=ao_count, ao_exp=ao_exp, mo=mo, eps_occ=eps_occ,
                    eps_vir=eps_vir, no=no, nv=nv, kappa=kappa, shell_atom=np.array(sa, dtype=np.int32),
                    shell_l=np.array(sl, dtype=np.int32), shell_exp=np.array(se), seed=seed)
