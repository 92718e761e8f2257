"""Thin Python binding of libmobius.so (argument marshalling only).

Every operation runs in the HIP library; torch is used for device memory and
the current stream.  Canonical fields are complex128 CUDA tensors:
  links   [4][Lt][Lz][Ly][Lx][3][3]
  spinor  [Ls][Lt][Lz][Ly][Lx][4][3]   (multi-RHS: leading [nrhs])
Packed half-lattice fields are opaque uint8 tensors of
``field_bytes(prec) * nrhs`` bytes.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmobius.so")

F64, F32, F16 = 0, 1, 2
PREC = {"f64": F64, "f32": F32, "f16": F16}
(OP_HOP, OP_M5, OP_SCHUR, OP_FULL, OP_SCHUR_RIGHT, OP_HOP_LEFT, OP_SCHUR_LEFT,
 OP_SCHUR_COMPLEMENT) = range(8)
OK, NOT_CONVERGED = 0, 1

EXPORTS = ("mobius_create", "mobius_destroy", "mobius_field_bytes", "mobius_pack",
           "mobius_unpack", "mobius_dslash", "mobius_dslash_dag", "mobius_m5inv",
           "mobius_cg_solve", "mobius_batch_solve", "mobius_propagator4d", "mobius_force", "mobius_force_lie",
           "mobius_tune", "mobius_set_tuning", "mobius_last_error", "mobius_dslash_noalloc",
           "mobius_bulk5d", "mobius_cg_solve_dag", "mobius_force_wall", "mobius_tune_brick")


class MobiusError(RuntimeError):
    pass


class _Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("Ls", ctypes.c_int32), ("M5", ctypes.c_double),
                ("mf", ctypes.c_double), ("b5", ctypes.c_double), ("c5", ctypes.c_double),
                ("mu", ctypes.c_double), ("b5s", ctypes.POINTER(ctypes.c_double)),
                ("c5s", ctypes.POINTER(ctypes.c_double)), ("brick", ctypes.c_int32 * 3)]


class _BrickTrial(ctypes.Structure):
    _fields_ = [("brick", ctypes.c_int32 * 3), ("hop_us", ctypes.c_double)]


def _make_params(dims, Ls, M5, mf, b5, c5, mu=0.0, b5s=None, c5s=None, brick=None):
    """mobius_params for a lattice; returns it with the arrays it points to
    (kept alive by the caller for as long as the struct is used)."""
    p = _Params((ctypes.c_int32 * 4)(*[int(d) for d in dims]), int(Ls), M5, mf, b5, c5, mu)
    keep = []
    for name, v in (("b5s", b5s), ("c5s", c5s)):
        if v is not None:
            if len(v) != int(Ls):
                raise MobiusError(f"{name} must hold Ls = {int(Ls)} values")
            a = (ctypes.c_double * int(Ls))(*[float(x) for x in v])
            keep.append(a)
            setattr(p, name, ctypes.cast(a, ctypes.POINTER(ctypes.c_double)))
    if brick is not None:
        if len(brick) != 3:
            raise MobiusError("brick must hold (Bx, By, Bz)")
        p.brick = (ctypes.c_int32 * 3)(*[int(b) for b in brick])
    return p, keep


class _SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int32),
                ("inner_prec", ctypes.c_int32), ("reliable_delta", ctypes.c_double),
                ("nrhs", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("err_tol", ctypes.c_double), ("form", ctypes.c_int32)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("prefetch", ctypes.c_int32),
                ("stage_links", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("nt_links", ctypes.c_int32), ("mfma", ctypes.c_int32), ("hop_us", ctypes.c_double)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("dirac_apps", ctypes.c_int32),
                ("reliable_updates", ctypes.c_int32), ("status", ctypes.c_int32),
                ("true_resid", ctypes.c_double), ("schur_resid", ctypes.c_double),
                ("seconds", ctypes.c_double), ("algo_bytes", ctypes.c_double),
                ("flops", ctypes.c_double), ("kappa", ctypes.c_double),
                ("err_bound", ctypes.c_double)]


@dataclass
class SolveInfo:
    iters: int
    dirac_apps: int
    reliable_updates: int
    status: int
    true_resid: float
    schur_resid: float
    seconds: float
    algo_bytes: float
    flops: float
    kappa: float
    err_bound: float


_lib = None


def lib():
    """Load libmobius.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MobiusError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1206_5214_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.mobius_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Params), vp, vp]
        L.mobius_destroy.argtypes = [vp]
        L.mobius_field_bytes.argtypes = [vp, i32]
        L.mobius_field_bytes.restype = i64
        L.mobius_pack.argtypes = [vp, i32, vp, vp, vp, i32, vp]
        L.mobius_unpack.argtypes = [vp, i32, vp, vp, vp, i32, vp]
        L.mobius_dslash.argtypes = [vp, i32, i32, i32, vp, vp, i32, vp]
        L.mobius_dslash_dag.argtypes = [vp, i32, i32, i32, vp, vp, i32, vp]
        L.mobius_m5inv.argtypes = [vp, i32, i32, vp, vp, i32, vp]
        L.mobius_dslash_noalloc.argtypes = [vp, i32, i32, i32, i32, vp, vp, i32, vp]
        L.mobius_cg_solve.argtypes = [vp, vp, vp, ctypes.POINTER(_SolveOpts),
                                      ctypes.POINTER(_SolveInfo), vp]
        L.mobius_batch_solve.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), ctypes.POINTER(_SolveOpts),
                                         ctypes.POINTER(_SolveInfo), vp]
        L.mobius_propagator4d.argtypes = [vp, vp, vp, ctypes.POINTER(_SolveOpts),
                                          ctypes.POINTER(_SolveInfo), vp]
        L.mobius_bulk5d.argtypes = [vp, vp, vp, ctypes.POINTER(_SolveOpts),
                                    ctypes.POINTER(_SolveInfo), vp]
        L.mobius_cg_solve_dag.argtypes = [vp, vp, vp, ctypes.POINTER(_SolveOpts),
                                          ctypes.POINTER(_SolveInfo), vp]
        L.mobius_force_wall.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(_SolveOpts), ctypes.POINTER(_SolveInfo), vp]
        L.mobius_force.argtypes = [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(_SolveOpts), ctypes.POINTER(_SolveInfo), vp]
        L.mobius_force_lie.argtypes = [vp, vp, vp, vp, vp]
        L.mobius_tune_brick.argtypes = [ctypes.POINTER(_Params), vp, i32, i32, ctypes.POINTER(_BrickTrial),
                                        i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(ctypes.c_double), vp]
        L.mobius_tune.argtypes = [vp, i32, i32, ctypes.POINTER(_TuneResult), vp]
        L.mobius_set_tuning.argtypes = [vp, ctypes.POINTER(_TuneResult)]
        L.mobius_last_error.restype = ctypes.c_char_p
        for f in EXPORTS:
            if f not in ("mobius_field_bytes", "mobius_last_error"):
                getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        msg = lib().mobius_last_error().decode()
        raise MobiusError(f"libmobius error {rc}: {msg}")
    return rc


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _require_cuda(t, dtype=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise MobiusError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise MobiusError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise MobiusError(f"{name} must have dtype {dtype}, got {t.dtype}")


class Operator:
    """A red/black Moebius operator on one lattice (owns the packed links)."""

    def __init__(self, dims, Ls, M5, mf, b5, c5, links, mu=0.0, b5s=None, c5s=None, brick=None):
        """b5s, c5s: optional per-slice coefficients (Ls values each) of the
        general operator; they replace b5, c5.  brick: (Bx, By, Bz) of the
        site order (None: the library's choice; see tune_brick)."""
        import torch
        _require_cuda(links, torch.complex128, "links")
        Lx, Ly, Lz, Lt = dims
        if tuple(links.shape) != (4, Lt, Lz, Ly, Lx, 3, 3):
            raise MobiusError(f"links have shape {tuple(links.shape)}")
        self.dims = tuple(int(d) for d in dims)
        self.Ls = int(Ls)
        self.params = dict(M5=M5, mf=mf, b5=b5, c5=c5, mu=mu, b5s=b5s, c5s=c5s)
        self.brick = None if brick is None else tuple(int(b) for b in brick)
        p, keep = _make_params(self.dims, self.Ls, M5, mf, b5, c5, mu, b5s, c5s, brick)
        h = ctypes.c_void_p()
        _check(lib().mobius_create(ctypes.byref(h), ctypes.byref(p), _ptr(links), _stream()))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().mobius_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- fields ----------------------------------------------------------
    @property
    def V(self):
        Lx, Ly, Lz, Lt = self.dims
        return Lx * Ly * Lz * Lt

    def canon_shape(self, nrhs=None):
        Lx, Ly, Lz, Lt = self.dims
        s = (self.Ls, Lt, Lz, Ly, Lx, 4, 3)
        return s if nrhs is None else (nrhs,) + s

    def link_shape(self):
        Lx, Ly, Lz, Lt = self.dims
        return (4, Lt, Lz, Ly, Lx, 3, 3)

    def field_bytes(self, prec):
        return int(lib().mobius_field_bytes(self._h, prec))

    def new_field(self, prec, nrhs=1):
        import torch
        return torch.zeros(self.field_bytes(prec) * nrhs, dtype=torch.uint8, device="cuda")

    def _check_canon(self, t, nrhs, name):
        import torch
        _require_cuda(t, torch.complex128, name)
        want = 1
        for d in self.canon_shape():
            want *= d
        if t.numel() != want * nrhs:
            raise MobiusError(f"{name} has {t.numel()} elements, expected {want * nrhs}")

    def _check_packed(self, t, prec, nrhs, name):
        import torch
        _require_cuda(t, torch.uint8, name)
        need = self.field_bytes(prec)
        if need < 0:
            raise MobiusError(f"unknown precision {prec}")
        if t.numel() < need * nrhs:
            raise MobiusError(f"{name} holds {t.numel()} bytes, needs {need * nrhs}")

    def pack(self, canon, prec, nrhs=1):
        self._check_canon(canon, nrhs, "canonical field")
        even, odd = self.new_field(prec, nrhs), self.new_field(prec, nrhs)
        _check(lib().mobius_pack(self._h, prec, _ptr(canon), _ptr(even), _ptr(odd), nrhs,
                                 _stream()))
        return even, odd

    def pack_full(self, canon, prec, nrhs=1):
        """Pack a canonical field into one buffer holding its nrhs even halves
        followed by its nrhs odd halves (the operand form of OP_FULL)."""
        self._check_canon(canon, nrhs, "canonical field")
        fb = self.field_bytes(prec) * nrhs
        buf = self.new_field(prec, 2 * nrhs)
        _check(lib().mobius_pack(self._h, prec, _ptr(canon), _ptr(buf), _ptr(buf[fb:]), nrhs,
                                 _stream()))
        return buf

    def unpack_full(self, buf, prec, nrhs=1):
        """Inverse of pack_full."""
        fb = self.field_bytes(prec) * nrhs
        self._check_packed(buf, prec, 2 * nrhs, "full field")
        return self.unpack(buf[:fb], buf[fb:2 * fb], prec, nrhs)

    def unpack(self, even, odd, prec, nrhs=1):
        import torch
        self._check_packed(even, prec, nrhs, "even half")
        self._check_packed(odd, prec, nrhs, "odd half")
        out = torch.empty(self.canon_shape(nrhs if nrhs > 1 else None), dtype=torch.complex128,
                          device="cuda")
        _check(lib().mobius_unpack(self._h, prec, _ptr(even), _ptr(odd), _ptr(out), nrhs,
                                   _stream()))
        return out

    # -- operators -------------------------------------------------------
    def dslash(self, x, out_parity, prec, op=OP_HOP, dag=False, out=None, nrhs=1):
        """Red/black block of D_DW (or D_DW^+) on packed fields; see mobius.h.
        For op=OP_FULL, x and out hold both halves (see pack_full)."""
        nf = 2 * nrhs if op == OP_FULL else nrhs
        if out is None:
            out = self.new_field(max(prec, 0) if prec in (F64, F32, F16) else F64, nf)
        self._check_packed(x, prec, nf, "input")
        self._check_packed(out, prec, nf, "output")
        f = lib().mobius_dslash_dag if dag else lib().mobius_dslash
        _check(f(self._h, prec, op, out_parity, _ptr(x), _ptr(out), nrhs, _stream()))
        return out

    def dslash_noalloc(self, x, out, out_parity, prec, op=OP_HOP, dag=False, nrhs=1):
        """mobius_dslash_noalloc: the operator blocks of dslash into a caller's
        output, with no allocation in the library (SCHUR uses its fixed
        per-GPU workspace; see mobius.h)."""
        nf = 2 * nrhs if op == OP_FULL else nrhs
        self._check_packed(x, prec, nf, "input")
        self._check_packed(out, prec, nf, "output")
        _check(lib().mobius_dslash_noalloc(self._h, prec, op, out_parity, int(dag), _ptr(x),
                                           _ptr(out), nrhs, _stream()))
        return out

    def m5inv(self, x, prec, dag=False, out=None, nrhs=1):
        if out is None:
            out = self.new_field(prec, nrhs)
        self._check_packed(x, prec, nrhs, "input")
        self._check_packed(out, prec, nrhs, "output")
        _check(lib().mobius_m5inv(self._h, prec, int(dag), _ptr(x), _ptr(out), nrhs, _stream()))
        return out

    def solve(self, src, tol=1e-10, maxiter=10000, inner_prec=F64, reliable_delta=0.0,
              check_every=0, err_tol=0.0, form=0, dagger=False):
        """Solve D_DW psi = src (canonical complex128, optional leading nrhs), or
        D_DW^+ psi = src with dagger.  reliable_delta <= 0 selects the library's
        default for inner_prec; err_tol > 0 also iterates until kappa * Schur
        residual <= err_tol; form 0/1 = left/right-preconditioned Schur system,
        2 = the Schur system of the left form D^ = D-^-1 D_DW D- (constant b5, c5),
        3 = the Schur complement S = I - D_oe I^-1 D_eo itself."""
        import torch
        nrhs = 1 if src.dim() == 7 else int(src.shape[0])
        self._check_canon(src, nrhs, "source")
        sol = torch.empty_like(src)
        opts = _SolveOpts(tol, maxiter, inner_prec, reliable_delta, nrhs, check_every, err_tol, form)
        infos = (_SolveInfo * nrhs)()
        f = lib().mobius_cg_solve_dag if dagger else lib().mobius_cg_solve
        rc = _check(f(self._h, _ptr(src), _ptr(sol), ctypes.byref(opts), infos, _stream()))
        return sol, [_info(i) for i in infos], rc

    def propagator4d(self, src4, tol=1e-10, maxiter=10000, inner_prec=F64, reliable_delta=0.0,
                     check_every=0, err_tol=0.0):
        """q = D_ov(m)^-1 b through the 5d solve D_DW(m) psi = D_DW(1) P b (see
        mobius_propagator4d); src4 canonical complex128 [t][z][y][x][4][3], with
        an optional leading nrhs."""
        import torch
        Lx, Ly, Lz, Lt = self.dims
        shape4 = (Lt, Lz, Ly, Lx, 4, 3)
        nrhs = 1 if src4.dim() == 6 else int(src4.shape[0])
        _require_cuda(src4, torch.complex128, "source")
        if tuple(src4.shape[-6:]) != shape4 or src4.numel() != nrhs * Lt * Lz * Ly * Lx * 12:
            raise MobiusError(f"source has shape {tuple(src4.shape)}, expected [nrhs,] {shape4}")
        sol = torch.empty_like(src4)
        opts = _SolveOpts(tol, maxiter, inner_prec, reliable_delta, nrhs, check_every, err_tol)
        infos = (_SolveInfo * nrhs)()
        rc = _check(lib().mobius_propagator4d(self._h, _ptr(src4), _ptr(sol), ctypes.byref(opts),
                                              infos, _stream()))
        return sol, [_info(i) for i in infos], rc

    def bulk5d(self, psi4, tol=1e-10, maxiter=10000, inner_prec=F64, reliable_delta=0.0,
               check_every=0, err_tol=0.0):
        """Psi = P^+ D_DW(m)^-1 D_DW(1) P B from the overlap solution psi =
        D_ov(m)^-1 b with one Pauli-Villars solve (see mobius_bulk5d); psi4
        canonical complex128 [t][z][y][x][4][3] with an optional leading nrhs.
        Returns (Psi canonical 5d, [SolveInfo of the Pauli-Villars solve], rc)."""
        import torch
        Lx, Ly, Lz, Lt = self.dims
        shape4 = (Lt, Lz, Ly, Lx, 4, 3)
        nrhs = 1 if psi4.dim() == 6 else int(psi4.shape[0])
        _require_cuda(psi4, torch.complex128, "psi4")
        if tuple(psi4.shape[-6:]) != shape4 or psi4.numel() != nrhs * Lt * Lz * Ly * Lx * 12:
            raise MobiusError(f"psi4 has shape {tuple(psi4.shape)}, expected [nrhs,] {shape4}")
        Psi = torch.empty(self.canon_shape(nrhs if nrhs > 1 else None), dtype=torch.complex128,
                          device=psi4.device)
        opts = _SolveOpts(tol, maxiter, inner_prec, reliable_delta, nrhs, check_every, err_tol)
        infos = (_SolveInfo * nrhs)()
        rc = _check(lib().mobius_bulk5d(self._h, _ptr(psi4), _ptr(Psi), ctypes.byref(opts), infos,
                                        _stream()))
        return Psi, [_info(i) for i in infos], rc

    def force_wall(self, phi4, tol=1e-12, maxiter=20000, inner_prec=F64, reliable_delta=0.0,
                   check_every=0, link_grad=True):
        """S = phi^+ (D_ov^+ D_ov)^-1 phi for a 4d pseudofermion on the wall and
        its link gradient by the two inversions of the 4d HMC (see
        mobius_force_wall).  Returns (S, grad_links or None, SolveInfo, rc)."""
        import torch
        Lx, Ly, Lz, Lt = self.dims
        _require_cuda(phi4, torch.complex128, "phi4")
        if tuple(phi4.shape) != (Lt, Lz, Ly, Lx, 4, 3):
            raise MobiusError(f"phi4 has shape {tuple(phi4.shape)}")
        grad = (torch.empty(self.link_shape(), dtype=torch.complex128, device=phi4.device)
                if link_grad else None)
        action = ctypes.c_double(0.0)
        opts = _SolveOpts(tol, maxiter, inner_prec, reliable_delta, 1, check_every)
        info = _SolveInfo()
        gl = _ptr(grad) if grad is not None else ctypes.c_void_p(None)
        rc = _check(lib().mobius_force_wall(self._h, _ptr(phi4), gl, ctypes.byref(action),
                                            ctypes.byref(opts), ctypes.byref(info), _stream()))
        return action.value, grad, _info(info), rc

    def force_lie(self, links, grad):
        """F = TA(U G^+) per link (see mobius_force_lie): the su(3) form of a
        link gradient G, with dS/deps = Re tr(F X) for U -> e^{eps X} U."""
        import torch
        _require_cuda(links, torch.complex128, "links")
        _require_cuda(grad, torch.complex128, "gradient")
        if tuple(links.shape) != self.link_shape() or tuple(grad.shape) != self.link_shape():
            raise MobiusError(f"links and gradient must have shape {self.link_shape()}")
        out = torch.empty_like(links)
        _check(lib().mobius_force_lie(self._h, _ptr(links), _ptr(grad), _ptr(out), _stream()))
        return out

    def tune(self, prec, reps=10):
        """Autotune the hop launch parameters of this operator for one storage
        precision; returns the chosen parameters and the measured hop time."""
        r = _TuneResult()
        _check(lib().mobius_tune(self._h, prec, reps, ctypes.byref(r), _stream()))
        return {"prec": r.prec, "prefetch": r.prefetch, "stage_links": r.stage_links,
                "xcd_remap": r.xcd_remap, "nt_links": r.nt_links, "mfma": r.mfma, "hop_us": r.hop_us}

    def set_tuning(self, prec, prefetch, stage_links, xcd_remap, nt_links, mfma=0):
        """Set the hop launch parameters for one precision explicitly."""
        r = _TuneResult(prec, prefetch, stage_links, xcd_remap, nt_links, mfma, 0.0)
        _check(lib().mobius_set_tuning(self._h, ctypes.byref(r)))

    def force(self, phi, tol=1e-12, maxiter=20000, inner_prec=F64, reliable_delta=0.0,
              check_every=0, link_grad=True):
        """S = phi_o^+ (D_pre^+ D_pre)^-1 phi_o (phi canonical complex128, its odd
        sites used) with dS/dU (canonical links layout; None when link_grad is
        false, which skips the link-derivative pass) and dS/dphi = 2 X.
        Returns (S, grad_links, grad_phi, SolveInfo, rc)."""
        import torch
        self._check_canon(phi, 1, "phi")
        grad_links = (torch.empty(self.link_shape(), dtype=torch.complex128, device=phi.device)
                      if link_grad else None)
        grad_phi = torch.empty_like(phi)
        action = ctypes.c_double(0.0)
        opts = _SolveOpts(tol, maxiter, inner_prec, reliable_delta, 1, check_every)
        info = _SolveInfo()
        gl = _ptr(grad_links) if grad_links is not None else ctypes.c_void_p(None)
        rc = _check(lib().mobius_force(self._h, _ptr(phi), gl, _ptr(grad_phi),
                                       ctypes.byref(action), ctypes.byref(opts), ctypes.byref(info),
                                       _stream()))
        return action.value, grad_links, grad_phi, _info(info), rc


def _info(i):
    return SolveInfo(i.iters, i.dirac_apps, i.reliable_updates, i.status, i.true_resid,
                     i.schur_resid, i.seconds, i.algo_bytes, i.flops, i.kappa, i.err_bound)


def tune_brick(dims, Ls, M5, mf, b5, c5, links, prec=F16, reps=10, mu=0.0, b5s=None, c5s=None):
    """Time the tuned hop for candidate site-order bricks (mobius_tune_brick) and
    return (brick, hop_us, trials): the brick to pass to Operator, its hop time
    and every candidate as ((Bx, By, Bz), hop_us) in the order timed."""
    import torch
    _require_cuda(links, torch.complex128, "links")
    p, keep = _make_params(dims, Ls, M5, mf, b5, c5, mu, b5s, c5s)
    trials = (_BrickTrial * 12)()
    n = ctypes.c_int32()
    brick = (ctypes.c_int32 * 3)()
    us = ctypes.c_double()
    _check(lib().mobius_tune_brick(ctypes.byref(p), _ptr(links), int(prec), int(reps), trials, 12,
                                   ctypes.byref(n), brick, ctypes.byref(us), _stream()))
    return (tuple(brick), us.value,
            [(tuple(trials[i].brick), trials[i].hop_us) for i in range(n.value)])


def batch_solve(ops, srcs, tol=1e-10, maxiter=10000, inner_prec=F64, reliable_delta=0.0,
                check_every=0, err_tol=0.0):
    """Solve D_DW psi_j = src_j for several lattices at once (one Operator per
    lattice, the same number of right-hand sides each).  Returns the list of
    solutions, a list (per lattice) of lists of SolveInfo, and the return code."""
    import torch
    if len(ops) != len(srcs) or not ops:
        raise MobiusError("batch_solve needs one source per operator")
    if len({id(o) for o in ops}) != len(ops):
        raise MobiusError("batch_solve needs distinct operators")
    nrhs = 1 if srcs[0].dim() == 7 else int(srcs[0].shape[0])
    sols = []
    for op, src in zip(ops, srcs):
        op._check_canon(src, nrhs, "source")
        sols.append(torch.empty_like(src))
    n = len(ops)
    vp = ctypes.c_void_p
    hs = (vp * n)(*[o._h for o in ops])
    ss = (vp * n)(*[s.data_ptr() for s in srcs])
    xs = (vp * n)(*[s.data_ptr() for s in sols])
    opts = _SolveOpts(tol, maxiter, inner_prec, reliable_delta, nrhs, check_every, err_tol)
    infos = (_SolveInfo * (n * nrhs))()
    rc = _check(lib().mobius_batch_solve(n, hs, ss, xs, ctypes.byref(opts), infos, _stream()))
    out = [[_info(infos[j * nrhs + r]) for r in range(nrhs)] for j in range(n)]
    return sols, out, rc
