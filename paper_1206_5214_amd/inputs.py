"""Seeded synthetic inputs: SU(3) gauge links and sources.

This module holds no arithmetic of the method itself (no Dirac operator, no
solver).  It only draws the synthetic fields that both the HIP path and the
CPU checker consume, in the canonical layouts:

  links   complex128 [4][Lt][Lz][Ly][Lx][3][3]   (mu = x, y, z, t; row a, column b)
  spinor  complex128 [Ls][Lt][Lz][Ly][Lx][4][3]  (s, then 4d site, then spin, colour)

Recipe for the links (the paper's own runs used quenched Wilson-gauge
ensembles that are not available; these stand in for them):
  rng = numpy.random.default_rng(seed); for all 4*V links at once, in C order
  of [mu][t][z][y][x]: draw A with real parts then imaginary parts ~ N(0,1);
  H = (A + A^+)/2 minus its trace/3 (Hermitian, traceless);
  U = V diag(exp(i eps lambda)) V^+ from the eigen-decomposition of H;
  re-unitarise: Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1),
  so det U = 1 to rounding.
Gaussian sources continue the same generator: real parts then imaginary
parts ~ N(0,1), canonical order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: lattice, Moebius parameters, link recipe, seed."""
    name: str
    dims: tuple          # (Lx, Ly, Lz, Lt)
    Ls: int
    M5: float
    mf: float
    b5: float
    c5: float
    eps: float           # link spread in exp(i eps H)
    seed: int
    tol: float = 1e-10
    notes: str = ""

    @property
    def V(self) -> int:
        return int(np.prod(self.dims))

    @property
    def N5(self) -> int:
        """half-lattice 5d sites"""
        return self.V // 2 * self.Ls


# The five synthetic workloads the build is measured and checked on.
WORKLOADS = {
    "shamir_4x4x4x4_ls8": Workload("shamir_4x4x4x4_ls8", (4, 4, 4, 4), 8, 1.8, 0.01, 1.0, 0.0,
                                   0.3, 0, notes="Shamir limit (c5 = 0), FP64"),
    "mobius_16x16x16x32_ls16": Workload("mobius_16x16x16x32_ls16", (16, 16, 16, 32), 16, 1.8, 0.01,
                                        1.5, 0.5, 0.5, 0,
                                        notes="Moebius alpha = 2; FP64 vs FP32/FP16 inner"),
    "mobius_24x24x24x64_ls12": Workload("mobius_24x24x24x64_ls12", (24, 24, 24, 64), 12, 1.8, 0.005,
                                        1.75, 0.75, 0.6, 0,
                                        notes="headline lattice: mixed precision vs FP64"),
    "batch_8_12_16_ls8": Workload("batch_8_12_16_ls8", (16, 16, 16, 16), 8, 1.8, 0.01, 1.5, 0.5,
                                  0.5, 3, notes="largest lattice of the uneven batch"),
    "force_8x8x8x16_ls8": Workload("force_8x8x8x16_ls8", (8, 8, 8, 16), 8, 1.8, 0.01, 1.5, 0.5,
                                   0.5, 4, notes="fermion-force finite-difference check"),
    "force_24x24x24x64_ls12": Workload("force_24x24x24x64_ls12", (24, 24, 24, 64), 12, 1.8, 0.005,
                                       1.5, 0.5, 0.6, 5, notes="fermion force, timed"),
}

# Uneven batch solved in lockstep: 8^4, 12^4, 16^4 at Ls = 8 (seeds 1-3), Moebius
# b5 = 1.5, c5 = 0.5 with the 16^3 x 32 link spread.
UNEVEN_BATCH = tuple(
    Workload(f"batch_{L}x{L}x{L}x{L}_ls8", (L, L, L, L), 8, 1.8, 0.01, 1.5, 0.5, 0.5, seed,
             notes="uneven batch member")
    for L, seed in ((8, 1), (12, 2), (16, 3)))

# Multi-RHS: the 12 spin-colour point sources of wall_point_sources on the
# 16^3 x 32, Ls = 16 Moebius lattice.
MULTI_RHS = WORKLOADS["mobius_16x16x16x32_ls16"]


def _reunitarize(U: np.ndarray) -> np.ndarray:
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def random_links(dims, eps: float, rng: np.random.Generator, chunk: int = 1 << 20) -> np.ndarray:
    """SU(3) links exp(i eps H), H Gaussian Hermitian traceless, re-unitarised."""
    Lx, Ly, Lz, Lt = dims
    n = 4 * Lx * Ly * Lz * Lt
    re = rng.standard_normal((n, 3, 3))
    im = rng.standard_normal((n, 3, 3))
    out = np.empty((n, 3, 3), np.complex128)
    eye = np.eye(3)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        A = re[a:b] + 1j * im[a:b]
        H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
        tr = np.trace(H, axis1=-2, axis2=-1).real
        H = H - (tr / 3.0)[:, None, None] * eye
        w, v = np.linalg.eigh(H)
        ph = np.exp(1j * eps * w)
        U = (v * ph[:, None, :]) @ np.conj(np.swapaxes(v, -1, -2))
        out[a:b] = _reunitarize(U)
    return out.reshape(4, Lt, Lz, Ly, Lx, 3, 3)


def unit_links(dims) -> np.ndarray:
    Lx, Ly, Lz, Lt = dims
    U = np.zeros((4, Lt, Lz, Ly, Lx, 3, 3), np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def gaussian_spinor(dims, Ls: int, rng: np.random.Generator, nrhs: int | None = None) -> np.ndarray:
    Lx, Ly, Lz, Lt = dims
    shape = (Ls, Lt, Lz, Ly, Lx, 4, 3)
    if nrhs is not None:
        shape = (nrhs,) + shape
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


def wall_point_sources(dims, Ls: int) -> np.ndarray:
    """12 point sources at the origin, one per (spin, colour) index a = 3*spin + colour,
    placed on the walls as the 4d quark field q = P- Psi_1 + P+ Psi_Ls is read off
    (Sec. 2.2): the P- spins (2, 3) at s = 1 and the P+ spins (0, 1) at s = Ls.
    Pure placement: [12][Ls][Lt][Lz][Ly][Lx][4][3]."""
    Lx, Ly, Lz, Lt = dims
    src = np.zeros((12, Ls, Lt, Lz, Ly, Lx, 4, 3), np.complex128)
    for a in range(12):
        spin, col = divmod(a, 3)
        s = Ls - 1 if spin < 2 else 0
        src[a, s, 0, 0, 0, 0, spin, col] = 1.0
    return src


def workload_fields(w: Workload, with_source: bool = True, nrhs: int | None = None):
    """(links, source) for a workload, from one generator seeded with w.seed."""
    rng = np.random.default_rng(w.seed)
    U = random_links(w.dims, w.eps, rng)
    if not with_source:
        return U, None
    return U, gaussian_spinor(w.dims, w.Ls, rng, nrhs)
