"""Plain FP64 CPU oracle for the Moebius domain-wall operator and its red/black CG.

TEST INFRASTRUCTURE ONLY: the product package never imports this module.  Only
the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.  It shares no code with the HIP path.

The arithmetic lives in ``mobius_oracle.c`` (plain C, FP64, natural layout);
this module only loads it with ctypes and marshals numpy arrays.  See
``mobius_oracle.h`` for the layouts and sign conventions.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mobius_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("Ls", ctypes.c_int32), ("M5", ctypes.c_double),
                ("mf", ctypes.c_double), ("b5", ctypes.c_double), ("c5", ctypes.c_double),
                ("mu", ctypes.c_double), ("b5s", ctypes.POINTER(ctypes.c_double)),
                ("c5s", ctypes.POINTER(ctypes.c_double))]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_resid", ctypes.c_double), ("true_resid", ctypes.c_double)]


def _bind(path):
    L = ctypes.CDLL(path)
    P = ctypes.POINTER(_Params)
    vp = ctypes.c_void_p
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_set_num_threads.argtypes = [ctypes.c_int]
    L.orc_set_num_threads.restype = None
    L.orc_wilson.argtypes = [P, vp, vp, vp, ctypes.c_int]
    L.orc_dw.argtypes = [P, vp, vp, vp, ctypes.c_int]
    L.orc_dw_sites.argtypes = [P, vp, vp, ctypes.c_int, ctypes.c_int64, vp, vp, ctypes.c_int]
    L.orc_hop.argtypes = [P, vp, ctypes.c_int, vp, vp, ctypes.c_int]
    L.orc_m5.argtypes = [P, vp, vp, vp, ctypes.c_int]
    L.orc_m5inv.argtypes = [P, vp, vp, ctypes.c_int]
    L.orc_schur.argtypes = [P, vp, vp, vp, ctypes.c_int]
    L.orc_cgls.argtypes = [P, vp, ctypes.c_int, vp, vp, ctypes.c_double, ctypes.c_int32,
                           ctypes.POINTER(_Info)]
    L.orc_solve.argtypes = [P, vp, vp, vp, ctypes.c_double, ctypes.c_int32,
                            ctypes.POINTER(_Info)]
    L.orc_cgne.argtypes = [P, vp, vp, vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_Info)]
    L.orc_force.argtypes = [P, vp, vp, vp, ctypes.c_int64, vp, vp, ctypes.c_double,
                            ctypes.c_int32, ctypes.POINTER(_Info)]
    L.orc_force.restype = ctypes.c_double
    L.orc_dw_left.argtypes = [P, vp, vp, vp, ctypes.c_int]
    L.orc_dw_left.restype = None
    L.orc_schur_right.argtypes = [P, vp, vp, vp, ctypes.c_int]
    L.orc_schur_right.restype = None
    L.orc_solve_form.argtypes = [P, vp, vp, vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int,
                                 ctypes.POINTER(_Info)]
    L.orc_solve_form.restype = None
    L.orc_force_wall.argtypes = [P, vp, vp, ctypes.c_int64, vp, vp, ctypes.c_double, ctypes.c_int32,
                                 ctypes.POINTER(_Info)]
    L.orc_force_wall.restype = ctypes.c_double
    for f in ("orc_wilson", "orc_dw", "orc_dw_sites", "orc_hop", "orc_m5", "orc_m5inv",
              "orc_schur", "orc_cgls", "orc_solve", "orc_cgne"):
        getattr(L, f).restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _bind(_LIB_PATH)
    return _lib


@contextlib.contextmanager
def using(path):
    """Temporarily route every oracle call through another build of the same
    source (used by the tests that plant a mistake in a copy of the oracle)."""
    global _lib
    saved = _lib
    _lib = _bind(path)
    try:
        yield
    finally:
        _lib = saved


@dataclass(frozen=True)
class Params:
    """Operator parameters: dims (Lx,Ly,Lz,Lt), Ls, M5 (> 0), mf, b5, c5, the
    chemical potential mu (time-like hops carry e^{+-mu}), and optional
    per-slice coefficients b5s, c5s (Ls values each, s = 1..Ls; they replace
    b5, c5: the general operator of Sec. 2.1)."""
    dims: tuple
    Ls: int
    M5: float
    mf: float
    b5: float
    c5: float
    mu: float = 0.0
    b5s: tuple = None
    c5s: tuple = None

    def c(self) -> _Params:
        P = _Params((ctypes.c_int32 * 4)(*self.dims), self.Ls, self.M5, self.mf, self.b5, self.c5,
                    self.mu)
        if self.b5s is not None or self.c5s is not None:
            b = self.b5s if self.b5s is not None else (self.b5,) * self.Ls
            c = self.c5s if self.c5s is not None else (self.c5,) * self.Ls
            assert len(b) == self.Ls and len(c) == self.Ls
            P._keep = ((ctypes.c_double * self.Ls)(*b), (ctypes.c_double * self.Ls)(*c))
            P.b5s = ctypes.cast(P._keep[0], ctypes.POINTER(ctypes.c_double))
            P.c5s = ctypes.cast(P._keep[1], ctypes.POINTER(ctypes.c_double))
        return P

    def b5_at(self, s):
        """b5 of slice s (0-based)."""
        return self.b5s[s] if self.b5s is not None else self.b5

    def c5_at(self, s):
        """c5 of slice s (0-based)."""
        return self.c5s[s] if self.c5s is not None else self.c5

    @property
    def V(self) -> int:
        return int(np.prod(self.dims))

    def shape5(self):
        Lx, Ly, Lz, Lt = self.dims
        return (self.Ls, Lt, Lz, Ly, Lx, 4, 3)

    def shape4(self):
        Lx, Ly, Lz, Lt = self.dims
        return (Lt, Lz, Ly, Lx, 4, 3)

    def link_shape(self):
        Lx, Ly, Lz, Lt = self.dims
        return (4, Lt, Lz, Ly, Lx, 3, 3)


@dataclass
class Info:
    iters: int
    converged: bool
    rel_resid: float
    true_resid: float


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Number of OpenMP threads of later oracle calls in this process."""
    lib().orc_set_num_threads(int(n))


def wilson(p: Params, U, psi4, dag=False):
    U, psi4 = _c128(U), _c128(psi4)
    out = np.empty_like(psi4)
    lib().orc_wilson(ctypes.byref(p.c()), _ptr(U), _ptr(psi4), _ptr(out), int(dag))
    return out


def dw(p: Params, U, psi, dag=False):
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().orc_dw(ctypes.byref(p.c()), _ptr(U), _ptr(psi), _ptr(out), int(dag))
    return out


def dw_sites(p: Params, U, psi, sites, in_parity=-1, dag=False):
    """D_DW psi (or D_DW^+ psi) at the listed canonical 4d site indices -> [n][Ls][4][3]."""
    U, psi = _c128(U), _c128(psi)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), p.Ls, 4, 3), np.complex128)
    lib().orc_dw_sites(ctypes.byref(p.c()), _ptr(U), _ptr(psi), int(in_parity), len(sites),
                       _ptr(sites), _ptr(out), int(dag))
    return out


def hop(p: Params, U, psi, out_parity, dag=False):
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().orc_hop(ctypes.byref(p.c()), _ptr(U), int(out_parity), _ptr(psi), _ptr(out), int(dag))
    return out


def m5(p: Params, U, psi, dag=False):
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().orc_m5(ctypes.byref(p.c()), _ptr(U), _ptr(psi), _ptr(out), int(dag))
    return out


def m5inv(p: Params, psi, dag=False):
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().orc_m5inv(ctypes.byref(p.c()), _ptr(psi), _ptr(out), int(dag))
    return out


def schur(p: Params, U, psi, dag=False):
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().orc_schur(ctypes.byref(p.c()), _ptr(U), _ptr(psi), _ptr(out), int(dag))
    return out


def cgls(p: Params, U, b, tol=1e-12, maxiter=10000, which="schur"):
    U, b = _c128(U), _c128(b)
    x = np.empty_like(b)
    info = _Info()
    lib().orc_cgls(ctypes.byref(p.c()), _ptr(U), 0 if which == "schur" else 1, _ptr(b), _ptr(x),
                   float(tol), int(maxiter), ctypes.byref(info))
    return x, Info(info.iters, bool(info.converged), info.rel_resid, info.true_resid)


def solve(p: Params, U, eta, tol=1e-12, maxiter=10000):
    """Red/black solve of D_DW psi = eta; returns (psi, Info) with the true residual."""
    U, eta = _c128(U), _c128(eta)
    psi = np.empty_like(eta)
    info = _Info()
    lib().orc_solve(ctypes.byref(p.c()), _ptr(U), _ptr(eta), _ptr(psi), float(tol), int(maxiter),
                    ctypes.byref(info))
    return psi, Info(info.iters, bool(info.converged), info.rel_resid, info.true_resid)


def dw_left(p: Params, U, psi, dag=False):
    """The left form D^ = D-^-1 D_DW D- (Sec. 2.1) or its adjoint."""
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().orc_dw_left(ctypes.byref(p.c()), _ptr(U), _ptr(psi), _ptr(out), int(dag))
    return out


def hop_left(p: Params, U, psi, out_parity, dag=False):
    """Off-diagonal block of the left form (parity 1-out_parity -> out_parity):
    D^ restricted to the input parity, the output parity kept."""
    out = dw_left(p, U, restrict(p, psi, 1 - out_parity), dag=dag)
    return restrict(p, out, out_parity)


def schur_left(p: Params, U, psi, dag=False):
    """Left-preconditioned Schur operator of the left form on the odd parity,
    1 - I^-1 D^_oe I^-1 D^_eo (its diagonal blocks are I), or its adjoint
    1 - D^_eo^+ I^-+ D^_oe^+ I^-+."""
    x = restrict(p, psi, 1)
    if not dag:
        t = m5inv(p, hop_left(p, U, x, 0))
        t = m5inv(p, hop_left(p, U, t, 1))
    else:
        t = hop_left(p, U, m5inv(p, x, dag=True), 0, dag=True)
        t = hop_left(p, U, m5inv(p, t, dag=True), 1, dag=True)
    return restrict(p, x - t, 1)


def schur_complement(p: Params, U, psi, dag=False):
    """The Schur complement of the even block on the odd parity (Sec. 3),
    S = I - D_oe I^-1 D_eo, or its adjoint I^+ - D_eo^+ I^-+ D_oe^+, from the
    blocks as the definition states them (no diagonal block taken out)."""
    x = restrict(p, psi, 1)
    t = hop(p, U, m5inv(p, hop(p, U, x, 0, dag=dag), dag=dag), 1, dag=dag)
    return restrict(p, m5(p, U, x, dag=dag) - t, 1)


def schur_right(p: Params, U, psi, dag=False):
    """D_R = 1 - D_oe I^-1 D_eo I^-1 (or its adjoint) on an odd-parity field."""
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().orc_schur_right(ctypes.byref(p.c()), _ptr(U), _ptr(psi), _ptr(out), int(dag))
    return out


def solve_form(p: Params, U, eta, form, tol=1e-12, maxiter=10000):
    """Red/black solve in form 0 (left), 1 (right) or 2 (the adjoint system
    D_DW^+ psi = eta); returns (psi, Info)."""
    U, eta = _c128(U), _c128(eta)
    psi = np.empty_like(eta)
    info = _Info()
    lib().orc_solve_form(ctypes.byref(p.c()), _ptr(U), _ptr(eta), _ptr(psi), float(tol), int(maxiter),
                         int(form), ctypes.byref(info))
    return psi, Info(info.iters, bool(info.converged), info.rel_resid, info.true_resid)


def force_wall(p: Params, U, phi4, links=None, tol=1e-13, maxiter=20000):
    """S = phi^+ [P^+ D(m)^-1 D(1) D(1)^+ D(m)^-+ P]_11 phi (phi 4d, on the wall;
    Sec. 2.4) and its link gradient (as force()).  Returns (S, grad, Info)."""
    U, phi4 = _c128(U), _c128(phi4)
    info = _Info()
    if links is None:
        grad = np.empty(p.link_shape(), np.complex128)
        lk, nl = None, 0
    else:
        ids = np.ascontiguousarray([mu * p.V + i for mu, i in links], dtype=np.int64)
        grad = np.empty((len(ids), 3, 3), np.complex128)
        lk, nl = _ptr(ids), len(ids)
    S = lib().orc_force_wall(ctypes.byref(p.c()), _ptr(U), _ptr(phi4), nl, lk, _ptr(grad), float(tol),
                             int(maxiter), ctypes.byref(info))
    return float(S), grad, Info(info.iters, bool(info.converged), info.rel_resid, info.true_resid)


def propagator4d(p: Params, U, b4, tol=1e-12, maxiter=20000):
    """q = [P^+ D_DW(m)^-1 D_DW(1) P b]_1, the overlap propagator D_ov(m)^-1 b
    obtained from the 5d solve (Sec. 2.2).  The chiral shift P puts b on the
    walls (P- b on slice 1, P+ b on slice Ls; P+ = spins 0, 1 in the chiral
    basis), D_DW(1) is the Pauli-Villars operator (mf = 1, same links and
    M5, b5, c5), and q = (P^+ psi)_1 = P- psi_1 + P+ psi_Ls.  b4: [t][z][y][x][4][3]
    (leading nrhs allowed).  Returns (q, [Info of each 5d solve])."""
    b4 = _c128(b4)
    single = b4.ndim == 6
    bs = b4[None] if single else b4
    pv = Params(p.dims, p.Ls, p.M5, 1.0, p.b5, p.c5, p.mu, p.b5s, p.c5s)
    qs, infos = [], []
    for b in bs:
        wall = np.zeros(p.shape5(), complex)
        wall[0, ..., 2:, :] = b[..., 2:, :]
        wall[p.Ls - 1, ..., :2, :] = b[..., :2, :]
        psi, info = solve(p, U, dw(pv, U, wall), tol=tol, maxiter=maxiter)
        q = np.empty_like(b)
        q[..., 2:, :] = psi[0, ..., 2:, :]
        q[..., :2, :] = psi[p.Ls - 1, ..., :2, :]
        qs.append(q)
        infos.append(info)
    return (qs[0] if single else np.stack(qs)), infos


def bulk5d(p: Params, U, psi4, tol=1e-12, maxiter=20000):
    """Overlap to bulk domain-wall reconstruction (Sec. 2.3): from the overlap
    solution psi = D_ov(m)^-1 b, the 5d field Psi = P^+ D_DW(m)^-1 D_DW(1) P B
    (B = b on slice 1 only) with a Pauli-Villars solve instead of a D_DW(m)
    solve:  psi~ = psi on slice 1,  Omega = P^+ D_DW(1)^-1 D_DW(m) P psi~,
    Psi_1 = psi and Psi_s = -Omega_s for s = 2..Ls.  (Omega_1 = D_ov(m) psi = b.)
    psi4: [t][z][y][x][4][3] (leading nrhs allowed).  Returns (Psi, Omega,
    [Info of each Pauli-Villars solve])."""
    psi4 = _c128(psi4)
    single = psi4.ndim == 6
    ps = psi4[None] if single else psi4
    pv = Params(p.dims, p.Ls, p.M5, 1.0, p.b5, p.c5, p.mu, p.b5s, p.c5s)
    Ps, Os, infos = [], [], []
    for psi in ps:
        wall = np.zeros(p.shape5(), complex)      # P psi~: P- psi on slice 1, P+ psi on slice Ls
        wall[0, ..., 2:, :] = psi[..., 2:, :]
        wall[p.Ls - 1, ..., :2, :] = psi[..., :2, :]
        y, info = solve(pv, U, dw(p, U, wall), tol=tol, maxiter=maxiter)
        omega = np.empty_like(y)                  # (P^+ y)_s = P- y_s + P+ y_{s-1}
        omega[..., 2:, :] = y[..., 2:, :]
        omega[..., :2, :] = np.roll(y, 1, axis=0)[..., :2, :]
        Psi = -omega
        Psi[0] = psi
        Ps.append(Psi)
        Os.append(omega)
        infos.append(info)
    if single:
        return Ps[0], Os[0], infos
    return np.stack(Ps), np.stack(Os), infos


def cgne(p: Params, U, phi, tol=1e-12, maxiter=10000):
    """X = (D_pre^+ D_pre)^{-1} phi for phi on the odd parity (plain CG)."""
    U, phi = _c128(U), _c128(phi)
    x = np.empty_like(phi)
    info = _Info()
    lib().orc_cgne(ctypes.byref(p.c()), _ptr(U), _ptr(phi), _ptr(x), float(tol), int(maxiter),
                   ctypes.byref(info))
    return x, Info(info.iters, bool(info.converged), info.rel_resid, info.true_resid)


def force(p: Params, U, phi, links=None, tol=1e-13, maxiter=20000):
    """S = phi^+ (D_pre^+ D_pre)^{-1} phi (phi on the odd parity) and its link
    gradient dS/dRe U + i dS/dIm U.  links: None for every link (gradient in the
    canonical link layout [4][Lt][Lz][Ly][Lx][3][3]) or a sequence of (mu,
    canonical 4d index) pairs (gradient [n][3][3]).  Returns (S, X, grad, Info)."""
    U, phi = _c128(U), _c128(phi)
    x = np.empty_like(phi)
    info = _Info()
    if links is None:
        grad = np.empty(p.link_shape(), np.complex128)
        lk, nl = None, 0
    else:
        ids = np.ascontiguousarray([mu * p.V + i for mu, i in links], dtype=np.int64)
        grad = np.empty((len(ids), 3, 3), np.complex128)
        lk, nl = _ptr(ids), len(ids)
    S = lib().orc_force(ctypes.byref(p.c()), _ptr(U), _ptr(phi), _ptr(x), nl, lk, _ptr(grad),
                        float(tol), int(maxiter), ctypes.byref(info))
    return float(S), x, grad, Info(info.iters, bool(info.converged), info.rel_resid,
                                   info.true_resid)


def force_lie(U, G):
    """F = TA(U G^+) per link, TA(M) = (M - M^+)/2 - tr(M - M^+)/6: the su(3)
    form of the link gradient G (dS/dRe U + i dS/dIm U), with dS/deps =
    Re tr(F X) for U -> e^{eps X} U.  U, G: [..., 3, 3]."""
    M = _c128(U) @ np.conj(np.swapaxes(_c128(G), -1, -2))
    A = 0.5 * (M - np.conj(np.swapaxes(M, -1, -2)))
    tr = np.trace(A, axis1=-2, axis2=-1) / 3.0
    return A - tr[..., None, None] * np.eye(3)


def parity_mask(p: Params):
    """Boolean [Lt][Lz][Ly][Lx] mask of odd sites ((x+y+z+t) mod 2 == 1)."""
    Lx, Ly, Lz, Lt = p.dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    return ((x + y + z + t) % 2) == 1


def restrict(p: Params, psi, parity):
    """Copy of a 5d field with the sites of the other parity set to zero."""
    m = parity_mask(p) if parity == 1 else ~parity_mask(p)
    out = np.array(psi, copy=True)
    out[:, ~m] = 0
    return out
