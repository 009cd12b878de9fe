"""Thin Python front end of librid.so (argument marshalling only).

PyTorch provides device memory (through the allocator callbacks) and the HIP
stream; every step of every solve runs in the library's kernels.
"""

from __future__ import annotations

import ctypes
import weakref
from typing import Optional, Sequence

import numpy as np
import torch

from . import _binding as B

_PRECOND = {"diag": B.RID_PRECOND_DIAG, "ris": B.RID_PRECOND_RIS}
_PRECISION = {"fp64": B.RID_PRECISION_FP64, "mixed": B.RID_PRECISION_MIXED}
_MODE = {"tda": B.RID_TDA, "rpa": B.RID_RPA}
_OPS = {"A": B.RID_OP_A, "APB_AMB": B.RID_OP_APB_AMB, "T": B.RID_OP_T, "TPM": B.RID_OP_TPM}
_DTYPES = {"f64": B.RID_F64, "f32": B.RID_F32, "bf16": B.RID_BF16}


class RidError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (status %d): %s" % (B.lib.rid_status_string(status).decode(), status, message))
        self.status = status


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _need_dev(t: torch.Tensor, shape, name, dtypes=(torch.float64,)):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype not in dtypes:
        raise TypeError("%s must be a CUDA tensor of dtype %s" % (name, " or ".join(str(d) for d in dtypes)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))


class Context:
    """A device, a stream and a PyTorch-backed device allocator."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        self.device = device
        self.stream = stream or torch.cuda.current_stream(device)
        self._children = weakref.WeakSet()  # problems and servers, closed before the context
        blocks = {}
        self._blocks = blocks
        dev = torch.device("cuda", device)

        # the callbacks hold the block table, not the context, so that no
        # reference cycle decides the order of finalisation
        def _alloc(user, nbytes):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
            except Exception as e:  # out of memory: the library reports RID_ERR_NO_MEMORY
                blocks["last_failure"] = "%d bytes: %s" % (int(nbytes), str(e).splitlines()[0][:300])
                return None
            blocks[t.data_ptr()] = t
            return t.data_ptr()

        def _free(user, p):
            if p:
                blocks.pop(int(p), None)

        self._alloc_ref = (B.ALLOC_FN(_alloc), B.FREE_FN(_free))
        alloc = B.rid_allocator(None, self._alloc_ref[0], self._alloc_ref[1])
        h = ctypes.c_void_p()
        s = B.lib.rid_context_create(device, ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(alloc), ctypes.byref(h))
        if s != B.RID_OK:
            raise RidError(s, B.lib.rid_last_error(None).decode())
        self.handle = h

    def profile(self, on: bool = True):
        """Enable or disable per-kernel-family launch timing."""
        self.check(B.lib.rid_profile_enable(self.handle, 1 if on else 0))

    def tune_save(self, path: str) -> int:
        """Write the context's tuning decisions to a file; returns their count."""
        n = ctypes.c_int32()
        self.check(B.lib.rid_tune_save(self.handle, path.encode(), ctypes.byref(n)))
        return n.value

    def tune_load(self, path: str) -> int:
        """Add a tuning file's decisions to the context; returns their count."""
        n = ctypes.c_int32()
        self.check(B.lib.rid_tune_load(self.handle, path.encode(), ctypes.byref(n)))
        return n.value

    def profile_only(self, family: Optional[str] = None):
        """Record only one kernel family's launches (None: all families)."""
        self.check(B.lib.rid_profile_only(self.handle, family.encode() if family else None))

    def profile_read(self) -> dict:
        """Per-family totals since the last read: {name: dict(launches, ms, flops, bytes)}."""
        cap = 64
        arr = (B.rid_kernel_stat * cap)()
        n = ctypes.c_int32()
        self.check(B.lib.rid_profile_read(self.handle, arr, cap, ctypes.byref(n)))
        out = {}
        for i in range(min(n.value, cap)):
            s = arr[i]
            out[s.name.decode()] = dict(launches=int(s.launches), ms=s.total_ms, flops=s.flops, bytes=s.bytes)
        return out

    def last_error(self) -> str:
        """The library's last error text, and the allocator's last failure."""
        msg = B.lib.rid_last_error(self.handle).decode() if getattr(self, "handle", None) else ""
        if "last_failure" in self._blocks:
            msg += " (allocator: %s)" % self._blocks["last_failure"]
        return msg

    def check(self, s: int, ok=(B.RID_OK,)):
        if s not in ok:
            raise RidError(s, B.lib.rid_last_error(self.handle).decode())
        return s

    def close(self):
        if getattr(self, "handle", None):
            for ch in list(self._children):
                ch.close()
            B.lib.rid_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_opts(precond: str = "ris", precision: str = "fp64", guess: Optional[torch.Tensor] = None,
                 **kw) -> B.rid_solve_opts:
    """Solve options.  guess: optional (n, N) float64 device tensor of start
    vectors (warm start); the caller keeps it alive until the solve ends."""
    o = B.rid_solve_opts()
    B.lib.rid_solve_opts_default(ctypes.byref(o))
    o.precond = _PRECOND[precond]
    o.precision = _PRECISION[precision]
    if guess is not None:
        _need_dev(guess, None, "guess")
        o.guess_dev = guess.data_ptr()
        o.n_guess = guess.shape[0]
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Problem:
    """One molecule: orbital energies and borrowed device tensors.

    The three-index tensors are float64, or float32 (then only mixed-precision
    solves run, and the library keeps no FP32 copy of them).
    """

    def __init__(self, ctx: Context, eps_occ, eps_vir, b_ia, b_ij, b_ab, a_x: float,
                 bris_ia=None, bris_ij=None, bris_ab=None, naux_ris_k: int = 0, t_cut: float = 0.0,
                 b_x: float = 0.0, blr=None, brislr=None):
        """blr / brislr: optional (ia, ij, ab) long-range tensors of a
        range-separated hybrid (weight b_x), full and ris model."""
        self.ctx = ctx
        self.eps_occ = np.ascontiguousarray(np.asarray(eps_occ, dtype=np.float64))
        self.eps_vir = np.ascontiguousarray(np.asarray(eps_vir, dtype=np.float64))
        no, nv = len(self.eps_occ), len(self.eps_vir)
        naux = b_ia.shape[0]
        fp = (torch.float64, torch.float32)
        _need_dev(b_ia, (naux, no, nv), "b_ia", fp)
        _need_dev(b_ij, (naux, no, no), "b_ij", (b_ia.dtype,))
        _need_dev(b_ab, (naux, nv, nv), "b_ab", (b_ia.dtype,))
        nris = 0
        if bris_ia is not None:
            nris = bris_ia.shape[0]
            _need_dev(bris_ia, (nris, no, nv), "bris_ia", fp)
            _need_dev(bris_ij, (nris, no, no), "bris_ij", (bris_ia.dtype,))
            _need_dev(bris_ab, (nris, nv, nv), "bris_ab", (bris_ia.dtype,))
        nlr = nrislr = 0
        if blr is not None:
            nlr = blr[0].shape[0]
            for t, shp, nm in zip(blr, ((nlr, no, nv), (nlr, no, no), (nlr, nv, nv)), ("ia", "ij", "ab")):
                _need_dev(t, shp, "blr_" + nm, (b_ia.dtype,))
        if brislr is not None:
            nrislr = brislr[0].shape[0]
            for t, shp, nm in zip(brislr, ((nrislr, no, nv), (nrislr, no, no), (nrislr, nv, nv)), ("ia", "ij", "ab")):
                _need_dev(t, shp, "brislr_" + nm, (bris_ia.dtype,))
        self.no, self.nv, self.naux, self.naux_ris = no, nv, naux, nris
        self.n = no * nv
        self._keep = (b_ia, b_ij, b_ab, bris_ia, bris_ij, bris_ab, blr, brislr)
        d = B.rid_problem_desc()
        d.no, d.nv, d.naux, d.naux_ris, d.naux_ris_k = no, nv, naux, nris, naux_ris_k
        d.a_x = a_x
        d.t_cut_ha = t_cut if np.isfinite(t_cut) else 0.0
        d.eps_occ_host = _dptr(self.eps_occ)
        d.eps_vir_host = _dptr(self.eps_vir)
        d.b_ia_dev, d.b_ij_dev, d.b_ab_dev = b_ia.data_ptr(), b_ij.data_ptr(), b_ab.data_ptr()
        d.b_dtype = B.RID_F64 if b_ia.dtype == torch.float64 else B.RID_F32
        d.bris_dtype = B.RID_F64
        if nris:
            d.bris_ia_dev, d.bris_ij_dev, d.bris_ab_dev = bris_ia.data_ptr(), bris_ij.data_ptr(), bris_ab.data_ptr()
            d.bris_dtype = B.RID_F64 if bris_ia.dtype == torch.float64 else B.RID_F32
        d.b_x = b_x
        d.naux_lr = nlr
        if nlr:
            d.blr_ia_dev, d.blr_ij_dev, d.blr_ab_dev = (t.data_ptr() for t in blr)
        d.naux_ris_lr = nrislr
        if nrislr:
            d.brislr_ia_dev, d.brislr_ij_dev, d.brislr_ab_dev = (t.data_ptr() for t in brislr)
        h = ctypes.c_void_p()
        ctx.check(B.lib.rid_problem_create(ctx.handle, ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        ctx._children.add(self)

    @classmethod
    def from_synth(cls, ctx: Context, p) -> "Problem":
        """From a synth.Problem whose tensors live on the context's device."""
        lr = (p.blr_ia, p.blr_ij, p.blr_ab) if getattr(p, "naux_lr", 0) else None
        rislr = (p.brislr_ia, p.brislr_ij, p.brislr_ab) if getattr(p, "brislr_ia", None) is not None else None
        return cls(ctx, p.eps_occ.cpu().numpy(), p.eps_vir.cpu().numpy(), p.b_ia, p.b_ij, p.b_ab, p.a_x,
                   p.bris_ia, p.bris_ij, p.bris_ab, p.naux_ris_k, p.t_cut, getattr(p, "b_x", 0.0), lr, rislr)

    def window(self):
        i0, na = ctypes.c_int32(), ctypes.c_int32()
        self.ctx.check(B.lib.rid_problem_window(self.handle, ctypes.byref(i0), ctypes.byref(na)))
        return i0.value, na.value

    def footprint(self) -> int:
        b = ctypes.c_uint64()
        self.ctx.check(B.lib.rid_problem_footprint(self.handle, ctypes.byref(b)))
        return int(b.value)

    def apply(self, op: str, x: torch.Tensor, dtype: str = "f64"):
        """op(x) for x (nvec, N) float64 on the device; returns y or (y, y2)."""
        _need_dev(x, None, "x")
        nvec = x.shape[0]
        if x.shape[1] != self.n:
            raise ValueError("x must have N = no*nv columns")
        y = torch.empty_like(x)
        pair = op in ("APB_AMB", "TPM")
        y2 = torch.empty_like(x) if pair else None
        self.ctx.check(B.lib.rid_apply_operator(self.handle, _OPS[op], _DTYPES[dtype], nvec, _ptr(x), _ptr(y),
                                                _ptr(y2)))
        return (y, y2) if pair else y

    def eigen(self, k: int, mode: str = "tda", precond: str = "ris", precision: str = "fp64",
              vectors: bool = True, **kw):
        """k lowest roots.  Returns dict(omega, resid, x, y, stats, status)."""
        o = default_opts(precond, precision, **kw)
        om = np.zeros(k)
        rs = np.zeros(k)
        x = torch.empty((k, self.n), dtype=torch.float64, device=self.b_device) if vectors else None
        y = torch.empty((k, self.n), dtype=torch.float64, device=self.b_device) if (vectors and mode == "rpa") else None
        st = B.rid_stats()
        s = self.ctx.check(B.lib.rid_eigen_solve(self.handle, ctypes.byref(o), k, _MODE[mode], _dptr(om), _ptr(x),
                                                 _ptr(y), _dptr(rs), ctypes.byref(st)),
                           ok=(B.RID_OK, B.RID_WARN_NOT_CONVERGED))
        return dict(omega=om, resid=rs, x=x, y=y, stats=st.as_dict(), status=s)

    def polarizability(self, p: torch.Tensor, omegas: Sequence[float], precond: str = "ris",
                       precision: str = "fp64", vectors: bool = False, **kw):
        """alpha[f, u, v] for right-hand sides p (nrhs, N).  Returns dict."""
        _need_dev(p, None, "p")
        nrhs = p.shape[0]
        om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
        nf = len(om)
        o = default_opts(precond, precision, **kw)
        alpha = np.zeros((nf, nrhs, nrhs))
        rs = np.zeros((nf, nrhs))
        u = torch.empty((nf, nrhs, self.n), dtype=torch.float64, device=self.b_device) if vectors else None
        st = B.rid_stats()
        s = self.ctx.check(B.lib.rid_response_solve(self.handle, ctypes.byref(o), nrhs, _ptr(p), nf, _dptr(om),
                                                    _dptr(alpha), _ptr(u), _dptr(rs), ctypes.byref(st)),
                           ok=(B.RID_OK, B.RID_WARN_NOT_CONVERGED))
        return dict(alpha=alpha, resid=rs, u=u, stats=st.as_dict(), status=s)

    @property
    def b_device(self):
        return self._keep[0].device

    def close(self):
        if getattr(self, "handle", None):
            if getattr(self.ctx, "handle", None):
                B.lib.rid_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _aux_desc(mol, mo: torch.Tensor, minimal: bool, theta: float, lmax: int):
    """rid_aux_basis_desc of a molecule (synth.Molecule fields) and the host
    arrays it points to (kept alive by the caller)."""
    d = B.rid_aux_basis_desc()
    keep = []

    def host(a, dtype, ptr):
        a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
        keep.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ptr))

    d.natom = len(mol.radius)
    d.coords_host = host(mol.coords, np.float64, ctypes.c_double)
    d.radius_host = host(mol.radius, np.float64, ctypes.c_double)
    d.ao_count_host = host(mol.ao_count, np.int32, ctypes.c_int32)
    d.ao_exp_host = host(mol.ao_exp, np.float64, ctypes.c_double)
    d.nao = len(mol.ao_exp)
    d.mo_dev = mo.data_ptr()
    d.no, d.nv = mol.no, mol.nv
    d.kappa = mol.kappa
    if minimal:
        d.nshell = 0
        d.theta = theta
        d.lmax = lmax
    else:
        d.nshell = len(mol.shell_exp)
        d.shell_atom_host = host(mol.shell_atom, np.int32, ctypes.c_int32)
        d.shell_l_host = host(mol.shell_l, np.int32, ctypes.c_int32)
        d.shell_exp_host = host(mol.shell_exp, np.float64, ctypes.c_double)
    return d, keep


def aux_tensor(ctx: Context, mol, minimal: bool = True, theta: float = 0.6, lmax: int = 2):
    """The RI tensor of a molecule's auxiliary basis, built on the device:
    the minimal basis of the ris model (exponents theta / R_A^2, shells up
    to lmax) or, with minimal=False, the molecule's full shell list.
    Returns (b_ia, b_ij, b_ab, naux_s) as float64 device tensors."""
    dev = torch.device("cuda", ctx.device)
    mo = torch.as_tensor(np.ascontiguousarray(mol.mo), dtype=torch.float64, device=dev)
    d, keep = _aux_desc(mol, mo, minimal, theta, lmax)
    naux, ns = ctypes.c_int32(), ctypes.c_int32()
    s = B.lib.rid_aux_basis_size(ctypes.byref(d), ctypes.byref(naux), ctypes.byref(ns))
    if s != B.RID_OK:
        raise RidError(s, B.lib.rid_last_error(None).decode())
    n = naux.value
    bia = torch.empty((n, mol.no, mol.nv), dtype=torch.float64, device=dev)
    bij = torch.empty((n, mol.no, mol.no), dtype=torch.float64, device=dev)
    bab = torch.empty((n, mol.nv, mol.nv), dtype=torch.float64, device=dev)
    ctx.check(B.lib.rid_aux_tensor_build(ctx.handle, ctypes.byref(d), _ptr(bia), _ptr(bij), _ptr(bab)))
    del keep
    return bia, bij, bab, ns.value


def molecule_problem(ctx: Context, mol, theta: float = 0.6, lmax: int = 2, a_x: float = 0.25,
                     t_cut: float = float("inf")):
    """A response problem built from a molecule on the device: A from the
    molecule's full auxiliary basis, the ris model from the minimal one
    (Coulomb: every function; exchange: the s functions)."""
    fia, fij, fab, _ = aux_tensor(ctx, mol, minimal=False)
    ria, rij, rab, ns = aux_tensor(ctx, mol, minimal=True, theta=theta, lmax=lmax)
    return Problem(ctx, mol.eps_occ, mol.eps_vir, fia, fij, fab, a_x, ria, rij, rab, ns, t_cut)


def make_request(kind: str, opts: B.rid_solve_opts, k: int = 0, mode: str = "tda",
                 p: Optional[torch.Tensor] = None, omegas: Optional[np.ndarray] = None,
                 x_out: Optional[torch.Tensor] = None, y_out: Optional[torch.Tensor] = None):
    """A batch/server request.  Eigen requests may name device tensors
    x_out (k, N) and y_out (k, N, full TDDFT) that receive X and Y."""
    r = B.rid_request()
    r.opts = opts
    keep = []
    if kind == "eigen":
        r.kind, r.k, r.mode = 0, k, _MODE[mode]
        if x_out is not None:
            _need_dev(x_out, (k, x_out.shape[1]), "x_out")
            r.x_dev = x_out.data_ptr()
            keep.append(x_out)
        if y_out is not None:
            _need_dev(y_out, (k, y_out.shape[1]), "y_out")
            r.y_dev = y_out.data_ptr()
            keep.append(y_out)
    else:
        r.kind = 1
        om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
        keep.append(om)
        r.nrhs, r.nfreq = p.shape[0], len(om)
        r.p_dev = p.data_ptr()
        r.omega_host = _dptr(om)
        keep.append(p)
    return r, keep


def request_footprint(prob: "Problem", req: B.rid_request) -> int:
    """Estimated device bytes of a request (what the server admits by)."""
    b = ctypes.c_uint64()
    prob.ctx.check(B.lib.rid_request_footprint(prob.handle, ctypes.byref(req), ctypes.byref(b)))
    return int(b.value)


def make_result(req: B.rid_request):
    res = B.rid_result()
    keep = {}
    if req.kind == 0:
        keep["omega"] = np.zeros(req.k)
        keep["resid"] = np.zeros(req.k)
    else:
        keep["alpha"] = np.zeros((req.nfreq, req.nrhs, req.nrhs))
        keep["resid"] = np.zeros((req.nfreq, req.nrhs))
        res.alpha_host = _dptr(keep["alpha"])
    if "omega" in keep:
        res.omega_host = _dptr(keep["omega"])
    res.resid_host = _dptr(keep["resid"])
    return res, keep


def batch_solve(ctx: Context, problems: Sequence[Problem], requests: Sequence[B.rid_request]):
    n = len(problems)
    hp = (ctypes.c_void_p * n)(*[p.handle.value for p in problems])
    rq = (B.rid_request * n)(*requests)
    results, keeps = [], []
    for r in requests:
        res, keep = make_result(r)
        results.append(res)
        keeps.append(keep)
    rs = (B.rid_result * n)(*results)
    # the arrays above copied the structs: point the copies at the kept buffers
    for i in range(n):
        k = keeps[i]
        if "omega" in k:
            rs[i].omega_host = _dptr(k["omega"])
        if "alpha" in k:
            rs[i].alpha_host = _dptr(k["alpha"])
        rs[i].resid_host = _dptr(k["resid"])
    # the library admits solves by the device memory it sees free: hand back
    # blocks that PyTorch caches but does not use
    torch.cuda.synchronize(ctx.device)
    torch.cuda.empty_cache()
    s = B.lib.rid_batch_solve(ctx.handle, n, ctypes.cast(hp, ctypes.POINTER(ctypes.c_void_p)), rq, rs)
    out = []
    for i in range(n):
        d = dict(keeps[i])
        d["status"] = rs[i].status
        d["stats"] = rs[i].stats.as_dict()
        d["t_start_ms"] = rs[i].t_admit_ms
        d["t_done_ms"] = rs[i].t_done_ms
        out.append(d)
    return s, out


class Server:
    """Continuous-batching request server."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int):
        self.ctx = ctx
        o = B.rid_server_opts(hbm_budget_bytes, max_slots)
        h = ctypes.c_void_p()
        ctx.check(B.lib.rid_server_create(ctx.handle, ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self._live = {}
        ctx._children.add(self)

    def submit(self, prob: Problem, req: B.rid_request, keep=()) -> int:
        res, bufs = make_result(req)
        box = {"req": req, "res": res, "bufs": bufs, "keep": keep, "prob": prob}
        t = ctypes.c_uint64()
        self.ctx.check(B.lib.rid_server_submit(self.handle, prob.handle, ctypes.byref(box["req"]),
                                               ctypes.byref(box["res"]), ctypes.byref(t)))
        self._live[t.value] = box
        return t.value

    def poll(self, ticket: int) -> bool:
        s = B.lib.rid_server_poll(self.handle, ticket)
        if s == B.RID_OK:
            return True
        if s == B.RID_ERR_PENDING:
            return False
        raise RidError(s, "poll failed")

    def wait(self, ticket: int, timeout_ms: int = -1) -> dict:
        s = B.lib.rid_server_wait(self.handle, ticket, timeout_ms)
        if s != B.RID_OK:
            raise RidError(s, "wait failed")
        box = self._live[ticket]
        res = box["res"]
        d = dict(box["bufs"])
        d.update(status=res.status, stats=res.stats.as_dict(), t_arrival_ms=res.t_arrival_ms,
                 t_admit_ms=res.t_admit_ms, t_done_ms=res.t_done_ms)
        return d

    def cancel(self, ticket: int):
        self.ctx.check(B.lib.rid_server_cancel(self.handle, ticket))

    def close(self):
        if getattr(self, "handle", None):
            if getattr(self.ctx, "handle", None):
                B.lib.rid_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
