"""Seeded, device-independent generator of synthetic TDDFT response inputs.

Random numbers come from a counter-based generator: the value at counter c of
stream s under seed k is splitmix64(key(k, s) + (c + 1) * 0x9E3779B97F4A7C15),
where splitmix64 is the output function of Steele, Lea and Flood's SplitMix64
("Fast splittable pseudorandom number generators", OOPSLA 2014).  Every value is
addressable by its index, so a tensor can be drawn in blocks, in any order, on
the CPU or on a GPU, and come out the same (the integer hashing is exact; the
Box-Muller transform may differ between devices by an ulp).

Shapes and distributions follow the paper's setting (Sec. 2.2, Eq. pqrs_approx:
ERIs written as a contraction of a symmetric three-index tensor, here already
multiplied by the square root of the metric) with these readings:

* orbital energies: occupied U[-1.0, -0.3] Ha, virtual U[0.05, 2.0] Ha, each
  sorted ascending (KS convention; makes the t_cut active sets of Sec. 3.1
  contiguous);
* B^P_pq for the ia, ij and ab blocks: i.i.d. N(0, 1); the ij and ab blocks are
  drawn on their upper triangle and mirrored (real orbitals give B^P_pq =
  B^P_qp); all three blocks share one scale c chosen so that the spectral norm
  of B_ia viewed as Naux x (no*nv) satisfies ||B_ia||_2^2 = 0.5 Ha;
* the ris tensor (the minimal auxiliary basis of Sec. 2.2.2) is one rotation of
  the auxiliary index shared by all blocks: the leading Naux_ris left singular
  vectors U_k of B_cat = [B_ia | B_ij | B_ab], B_ris = U_k^T B, then multiplied
  elementwise by (1 + 0.05 Z), Z ~ N(0, 1) (mirrored for ij/ab); the exchange
  part uses the leading round(Naux_ris / 9) rows (one s function out of the
  nine s, p, d functions per atom of the (d, s) design of Sec. 3.2);
* dipole right-hand sides: P_{ia,u} = g_{ia,u} / (eps_a - eps_i), g ~ N(0, 1).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import torch

HARTREE_PER_EV = 1.0 / 27.211386246
TCUT_HA_DEFAULT = 40.0 * HARTREE_PER_EV  # Sec. 3.1: t_cut = 40 eV

# Stream identifiers.  Each tensor draws from its own stream so that changing
# one size never shifts another tensor's values.
_STREAM_EPS_OCC = 1
_STREAM_EPS_VIR = 2
_STREAM_B_IA = 3
_STREAM_B_IJ = 4
_STREAM_B_AB = 5
_STREAM_RIS_IA = 6
_STREAM_RIS_IJ = 7
_STREAM_RIS_AB = 8
_STREAM_DIPOLE = 9
_STREAM_LR_IA = 10
_STREAM_LR_IJ = 11
_STREAM_LR_AB = 12
_STREAM_RISLR_IA = 13
_STREAM_RISLR_IJ = 14
_STREAM_RISLR_AB = 15

_MASK64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def _as_i64(v: int) -> int:
    v &= _MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _mix_int(z: int) -> int:
    """splitmix64 output function on a Python int (exact, mod 2^64)."""
    z &= _MASK64
    z = ((z ^ (z >> 30)) * _M1) & _MASK64
    z = ((z ^ (z >> 27)) * _M2) & _MASK64
    return z ^ (z >> 31)


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 lanes viewed as unsigned."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    """splitmix64 output function on int64 tensors (wrapping multiply)."""
    z = (z ^ _srl(z, 30)) * _as_i64(_M1)
    z = (z ^ _srl(z, 27)) * _as_i64(_M2)
    return z ^ _srl(z, 31)


def _stream_key(seed: int, stream: int) -> int:
    return _as_i64(_mix_int((seed * _GOLDEN + stream * 0xD1B54A32D192ED03) & _MASK64))


def counter_uniforms(seed: int, stream: int, start: int, count: int,
                     device="cpu") -> torch.Tensor:
    """Uniform doubles in (0, 1) at counters start .. start+count-1."""
    key = _stream_key(seed, stream)
    c = torch.arange(start, start + count, dtype=torch.int64, device=device)
    z = _mix((c + 1) * _as_i64(_GOLDEN) + key)
    return (_srl(z, 11).to(torch.float64) + 0.5) * (2.0 ** -53)


def counter_normals(seed: int, stream: int, start: int, count: int,
                    device="cpu") -> torch.Tensor:
    """Standard normal doubles at indices start .. start+count-1 (Box-Muller).

    Index t uses the uniforms at counters 2t and 2t+1 of the same stream.
    """
    key = _stream_key(seed, stream)
    c = torch.arange(2 * start, 2 * (start + count), dtype=torch.int64, device=device)
    z = _mix((c + 1) * _as_i64(_GOLDEN) + key)
    u = (_srl(z, 11).to(torch.float64) + 0.5) * (2.0 ** -53)
    del z, c
    u = u.view(count, 2)
    r = torch.sqrt(-2.0 * torch.log(u[:, 0]))
    return r * torch.cos((2.0 * math.pi) * u[:, 1])


def _normal_tensor(seed, stream, shape, device, chunk_elems=1 << 26, symmetric=False):
    """Draw an i.i.d. N(0,1) tensor of `shape` = (P, n, m) in P-blocks.

    With symmetric=True (n == m) the upper triangle (with diagonal) of every
    P-slice is kept and mirrored, so each slice is a symmetric matrix whose
    independent entries are i.i.d. N(0, 1).
    """
    P = shape[0]
    per = int(np.prod(shape[1:]))
    out = torch.empty(shape, dtype=torch.float64, device=device)
    pb = max(1, chunk_elems // max(per, 1))
    for p0 in range(0, P, pb):
        p1 = min(P, p0 + pb)
        g = counter_normals(seed, stream, p0 * per, (p1 - p0) * per, device)
        g = g.view((p1 - p0,) + tuple(shape[1:]))
        if symmetric:
            up = torch.triu(g)
            g = up + torch.triu(g, diagonal=1).transpose(1, 2)
        out[p0:p1] = g
        del g
    return out


@dataclasses.dataclass
class Problem:
    """One synthetic molecule.  All tensors are float64 on `device`.

    b_ia: (naux, no, nv), b_ij: (naux, no, no), b_ab: (naux, nv, nv).
    bris_*: same blocks with naux_ris rows (None when no ris tensor is built).
    The exchange part of the ris operator uses rows [0, naux_ris_k).
    """

    no: int
    nv: int
    naux: int
    eps_occ: torch.Tensor
    eps_vir: torch.Tensor
    b_ia: torch.Tensor
    b_ij: torch.Tensor
    b_ab: torch.Tensor
    a_x: float = 0.25
    naux_ris: int = 0
    naux_ris_k: int = 0
    t_cut: float = TCUT_HA_DEFAULT
    bris_ia: Optional[torch.Tensor] = None
    bris_ij: Optional[torch.Tensor] = None
    bris_ab: Optional[torch.Tensor] = None
    seed: int = 0
    # range-separated hybrid: exchange integrals a_x (pq|rs) + b_x (pq|rs)^LR,
    # the long-range part factored through its own tensor C (naux_lr rows)
    # and, in the ris model, through naux_ris_k rows of a minimal C
    b_x: float = 0.0
    naux_lr: int = 0
    blr_ia: Optional[torch.Tensor] = None
    blr_ij: Optional[torch.Tensor] = None
    blr_ab: Optional[torch.Tensor] = None
    brislr_ia: Optional[torch.Tensor] = None
    brislr_ij: Optional[torch.Tensor] = None
    brislr_ab: Optional[torch.Tensor] = None

    @property
    def n(self) -> int:
        return self.no * self.nv

    def to(self, device) -> "Problem":
        kw = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            kw[f.name] = v.to(device) if isinstance(v, torch.Tensor) else v
        return Problem(**kw)

    def numpy(self) -> dict:
        """Plain dict of numpy float64 arrays and scalars (for the oracle)."""
        d = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            d[f.name] = v.detach().cpu().numpy() if isinstance(v, torch.Tensor) else v
        return d

    def active_ranges(self):
        """(i0, nv_act): occupied i >= i0 and virtual a < nv_act are active.

        Sec. 3.1: exchange ERIs with a virtual above eps_HOMO + t_cut or an
        occupied below eps_LUMO - t_cut are dropped (energies sorted).
        """
        eo = self.eps_occ.detach().cpu().numpy()
        ev = self.eps_vir.detach().cpu().numpy()
        homo, lumo = eo[-1], ev[0]
        nv_act = int(np.sum(ev <= homo + self.t_cut))
        i0 = int(np.sum(eo < lumo - self.t_cut))
        return i0, nv_act


def _svd_rotation(blocks, naux, rows, dev):
    """Leading `rows` left singular directions of [blocks] (Naux x ...),
    descending, with a deterministic sign (largest entry positive)."""
    gram = torch.zeros((naux, naux), dtype=torch.float64, device=dev)
    for blk in blocks:
        m = blk.reshape(naux, -1)
        gram += m @ m.T
    _, vecs = torch.linalg.eigh(gram.cpu())
    rot = torch.flip(vecs[:, naux - rows:], dims=[1]).to(dev)
    idx = torch.argmax(rot.abs(), dim=0)
    sgn = torch.sign(rot[idx, torch.arange(rows, device=dev)])
    sgn[sgn == 0] = 1.0
    return rot * sgn


def make_problem(no: int, nv: int, naux: int, naux_ris: int = 0,
                 naux_ris_k: Optional[int] = None, a_x: float = 0.25,
                 seed: int = 0, noise: float = 0.05, device="cpu",
                 ris_source: str = "svd", t_cut: float = TCUT_HA_DEFAULT,
                 coupling: float = 0.5, b_x: float = 0.0, naux_lr: int = 0) -> Problem:
    """Build a synthetic problem.

    ris_source: "svd" (leading components of the shared SVD, then noise),
    "full" (ris tensor = the full tensor, times noise if noise > 0), or
    "none" (no ris tensor).
    coupling: target value of ||B_ia||_2^2 in Ha.
    b_x, naux_lr: range-separated hybrid.  With naux_lr > 0 a second tensor
    C (long-range integrals, its own streams, same distributions and scale
    rule as B) enters the exchange with weight b_x; the ris model gets the
    leading naux_ris_k SVD directions of C (times 1 + noise Z).
    """
    dev = torch.device(device)
    eps_occ, _ = torch.sort(-1.0 + 0.7 * counter_uniforms(seed, _STREAM_EPS_OCC, 0, no, dev))
    eps_vir, _ = torch.sort(0.05 + 1.95 * counter_uniforms(seed, _STREAM_EPS_VIR, 0, nv, dev))

    b_ia = _normal_tensor(seed, _STREAM_B_IA, (naux, no, nv), dev)
    g2 = b_ia.reshape(naux, no * nv)
    # the (Naux x Naux) Gram matrices are formed on the device and
    # diagonalised on the host, so that the result does not depend on the
    # device's eigensolver
    smax2 = float(torch.linalg.eigvalsh((g2 @ g2.T).cpu())[-1])
    scale = math.sqrt(coupling / smax2) if smax2 > 0 else 0.0
    b_ia.mul_(scale)
    b_ij = _normal_tensor(seed, _STREAM_B_IJ, (naux, no, no), dev, symmetric=True).mul_(scale)
    b_ab = _normal_tensor(seed, _STREAM_B_AB, (naux, nv, nv), dev, symmetric=True).mul_(scale)

    prob = Problem(no=no, nv=nv, naux=naux, eps_occ=eps_occ, eps_vir=eps_vir,
                   b_ia=b_ia, b_ij=b_ij, b_ab=b_ab, a_x=a_x, t_cut=t_cut, seed=seed)
    if naux_lr > 0:
        c_ia = _normal_tensor(seed, _STREAM_LR_IA, (naux_lr, no, nv), dev)
        c2 = c_ia.reshape(naux_lr, no * nv)
        cmax2 = float(torch.linalg.eigvalsh((c2 @ c2.T).cpu())[-1])
        cs = math.sqrt(coupling / cmax2) if cmax2 > 0 else 0.0
        c_ia.mul_(cs)
        prob.b_x = float(b_x)
        prob.naux_lr = naux_lr
        prob.blr_ia = c_ia
        prob.blr_ij = _normal_tensor(seed, _STREAM_LR_IJ, (naux_lr, no, no), dev, symmetric=True).mul_(cs)
        prob.blr_ab = _normal_tensor(seed, _STREAM_LR_AB, (naux_lr, nv, nv), dev, symmetric=True).mul_(cs)
    if ris_source == "none":
        return prob
    if ris_source == "full":
        naux_ris = naux
        rot = None
    elif ris_source == "svd":
        if not (0 < naux_ris <= naux):
            raise ValueError("naux_ris must be in (0, naux]")
        gram = torch.zeros((naux, naux), dtype=torch.float64, device=dev)
        for blk in (b_ia, b_ij, b_ab):
            m = blk.reshape(naux, -1)
            gram += m @ m.T
        _, vecs = torch.linalg.eigh(gram.cpu())
        rot = torch.flip(vecs[:, naux - naux_ris:], dims=[1]).to(dev)  # descending
        # deterministic sign: the largest-magnitude entry of each column > 0
        idx = torch.argmax(rot.abs(), dim=0)
        sgn = torch.sign(rot[idx, torch.arange(naux_ris, device=dev)])
        sgn[sgn == 0] = 1.0
        rot = rot * sgn
        del gram, vecs
    else:
        raise ValueError(ris_source)

    def rotate(blk):
        if rot is None:
            return blk.clone()
        return (rot.T @ blk.reshape(naux, -1)).reshape((naux_ris,) + tuple(blk.shape[1:]))

    bris_ia = rotate(b_ia)
    bris_ij = rotate(b_ij)
    bris_ab = rotate(b_ab)
    if noise > 0:
        bris_ia.mul_(1.0 + noise * _normal_tensor(seed, _STREAM_RIS_IA, tuple(bris_ia.shape), dev))
        bris_ij.mul_(1.0 + noise * _normal_tensor(seed, _STREAM_RIS_IJ, tuple(bris_ij.shape), dev,
                                                  symmetric=True))
        bris_ab.mul_(1.0 + noise * _normal_tensor(seed, _STREAM_RIS_AB, tuple(bris_ab.shape), dev,
                                                  symmetric=True))
    if naux_ris_k is None:
        naux_ris_k = max(1, int(round(naux_ris / 9.0)))
    prob.naux_ris = naux_ris
    prob.naux_ris_k = int(min(naux_ris_k, naux_ris))
    prob.bris_ia, prob.bris_ij, prob.bris_ab = bris_ia, bris_ij, bris_ab
    if naux_lr > 0:
        rows = min(prob.naux_ris_k, naux_lr)
        if ris_source == "full":
            rl = None
            rows = naux_lr
        else:
            rl = _svd_rotation((prob.blr_ia, prob.blr_ij, prob.blr_ab), naux_lr, rows, dev)

        def rotate_lr(blk):
            if rl is None:
                return blk.clone()
            return (rl.T @ blk.reshape(naux_lr, -1)).reshape((rows,) + tuple(blk.shape[1:]))

        c_ia, c_ij, c_ab = rotate_lr(prob.blr_ia), rotate_lr(prob.blr_ij), rotate_lr(prob.blr_ab)
        if noise > 0:
            c_ia.mul_(1.0 + noise * _normal_tensor(seed, _STREAM_RISLR_IA, tuple(c_ia.shape), dev))
            c_ij.mul_(1.0 + noise * _normal_tensor(seed, _STREAM_RISLR_IJ, tuple(c_ij.shape), dev, symmetric=True))
            c_ab.mul_(1.0 + noise * _normal_tensor(seed, _STREAM_RISLR_AB, tuple(c_ab.shape), dev, symmetric=True))
        prob.brislr_ia, prob.brislr_ij, prob.brislr_ab = c_ia, c_ij, c_ab
    return prob


def make_dipoles(prob: Problem, nrhs: int = 3, seed: Optional[int] = None) -> torch.Tensor:
    """Dipole-like right-hand sides, shape (nrhs, no*nv), float64.

    P_{ia,u} = g_{ia,u} / (eps_a - eps_i) with g ~ N(0, 1).
    """
    seed = prob.seed if seed is None else seed
    dev = prob.eps_occ.device
    g = counter_normals(seed, _STREAM_DIPOLE, 0, nrhs * prob.n, dev).view(nrhs, prob.no, prob.nv)
    de = prob.eps_vir[None, None, :] - prob.eps_occ[None, :, None]
    return (g / de).reshape(nrhs, prob.n)


def make_block(seed: int, stream: int, nvec: int, n: int, device="cpu") -> torch.Tensor:
    """A block of nvec random N(0,1) vectors of length n, shape (nvec, n)."""
    return counter_normals(seed, 1000 + stream, 0, nvec * n, device).view(nvec, n)


_CONFIGS = {
    # name: (no, nv, naux, naux_ris, seed)
    "c0": (20, 80, 400, 90, 0),
    "c1": (100, 400, 2000, 450, 100),
    "c2": (200, 800, 4000, 900, 200),
}


def config_sizes(name: str):
    """(no, nv, naux, naux_ris, seed) of a named fixed-size workload."""
    return _CONFIGS[name]


def molecule_sizes(no: int):
    """Sizes of a molecule in the batched and served workloads.

    nv = 4 no, Naux = 20 no, Naux_ris = round(4.5 no), exchange rows
    round(0.5 no).
    """
    return dict(no=no, nv=4 * no, naux=20 * no, naux_ris=int(round(4.5 * no)),
                naux_ris_k=max(1, int(round(0.5 * no))))


def batch_member(m: int) -> dict:
    """Molecule m of the batched workload (64 molecules of uneven size).

    no = round(exp(U[ln 20, ln 200])) with the sizes of molecule_sizes, and
    k drawn uniformly from {5, 10, 20}; seed 300 + m.
    """
    u = counter_uniforms(300 + m, 7, 0, 2)
    no = int(round(math.exp(math.log(20.0) + float(u[0]) * (math.log(200.0) - math.log(20.0)))))
    k = (5, 10, 20)[min(2, int(float(u[1]) * 3.0))]
    d = molecule_sizes(no)
    d.update(k=k, seed=300 + m)
    return d


def serve_trace(n: int, seed: int = 400, no_min: int = 20, no_max: int = 300) -> list:
    """A served request stream: n requests in arrival order.

    Request r (seed 400000 + r): no log-uniform in [no_min, no_max] with the
    sizes of molecule_sizes; 70% eigen-solves (TDA or RPA with probability
    1/2 each, k uniform in 5..20), 30% polarizabilities (3 right-hand sides,
    3 frequencies uniform in [0, 0.3] Ha, sorted).  `gap` is an Exp(1)
    inter-arrival draw, to be divided by the arrival rate.
    """
    out = []
    for r in range(n):
        u = counter_uniforms(seed * 1000 + r, 9, 0, 8)
        no = int(round(math.exp(math.log(no_min) + float(u[0]) * (math.log(no_max) - math.log(no_min)))))
        d = molecule_sizes(no)
        d["seed"] = seed * 1000 + r
        d["gap"] = -math.log(float(u[1]))
        if float(u[2]) < 0.7:
            d["kind"] = "eigen"
            d["mode"] = "tda" if float(u[3]) < 0.5 else "rpa"
            d["k"] = 5 + min(15, int(float(u[4]) * 16.0))
        else:
            d["kind"] = "polarizability"
            d["omegas"] = sorted(0.3 * float(x) for x in u[5:8])
        out.append(d)
    return out


def related_problem(p: Problem, step: float = 0.01, seed: int = 1) -> Problem:
    """A neighbour of problem p, as after a small geometry step: every
    three-index tensor multiplied elementwise by (1 + step Z) (Z ~ N(0, 1),
    mirrored for the ij and ab blocks) and the orbital energies moved by
    0.1 step U[-1, 1] (kept sorted)."""
    dev = p.b_ia.device
    base = 7_000_000 + seed

    def bump(t, stream, symmetric):
        if t is None:
            return None
        return t * (1.0 + step * _normal_tensor(base, stream, tuple(t.shape), dev, symmetric=symmetric))

    eo, _ = torch.sort(p.eps_occ + 0.1 * step * (2.0 * counter_uniforms(base, 1, 0, p.no, dev) - 1.0))
    ev, _ = torch.sort(p.eps_vir + 0.1 * step * (2.0 * counter_uniforms(base, 2, 0, p.nv, dev) - 1.0))
    kw = {f.name: getattr(p, f.name) for f in dataclasses.fields(p)}
    kw.update(eps_occ=eo, eps_vir=ev, b_ia=bump(p.b_ia, 3, False), b_ij=bump(p.b_ij, 4, True),
              b_ab=bump(p.b_ab, 5, True), bris_ia=bump(p.bris_ia, 6, False), bris_ij=bump(p.bris_ij, 7, True),
              bris_ab=bump(p.bris_ab, 8, True))
    return Problem(**kw)
