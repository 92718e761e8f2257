"""Free-field (unit-link) closed forms used to pin the oracle.

These are momentum-space formulas derived from the paper's definitions; they
share nothing with the oracle's matrix-free code.  Index order of a 5d symbol:
row/column = 4*s + spin (colour is trivial at unit links).
"""
from __future__ import annotations

import numpy as np

SIGMA = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]),
         np.array([[1, 0], [0, -1]], complex)]


def gammas():
    """Chiral basis: g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0, 1], [1, 0]]."""
    Z, I2 = np.zeros((2, 2)), np.eye(2)
    g = [np.block([[Z, -1j * s], [1j * s, Z]]) for s in SIGMA]
    g.append(np.block([[Z, I2], [I2, Z]]).astype(complex))
    return g


G = gammas()
G5 = G[0] @ G[1] @ G[2] @ G[3]
PP = 0.5 * (np.eye(4) + G5)
PM = 0.5 * (np.eye(4) - G5)


def momenta(dims, rng, n):
    """n random lattice momenta p_mu = 2 pi k_mu / L_mu."""
    out = []
    for _ in range(n):
        out.append(np.array([2 * np.pi * rng.integers(0, L) / L for L in dims]))
    return out


def plane_wave(dims, p):
    """e^{i p.x} on the [t][z][y][x] grid."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    return np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))


def wilson_symbol(p, M5, dag=False):
    """D_W(p) at unit links: the forward hop gives -1/2 (1-g) e^{ip}, the backward
    -1/2 (1+g) e^{-ip}, so D_W(p) = (4 - M5 - sum cos p) + i sum g sin p."""
    s = 1j * sum(G[mu] * np.sin(p[mu]) for mu in range(4))
    return (4 - M5 - np.sum(np.cos(p))) * np.eye(4) + (-s if dag else s)


def mobius_kernel(Dw, b5, c5):
    """(b5 + c5) D_W / (2 + (b5 - c5) D_W)  (Sec. 2)."""
    return np.linalg.solve(2 * np.eye(4) + (b5 - c5) * Dw, (b5 + c5) * Dw)


def polar_sign(H, Ls):
    """eps_Ls(H) = ((1+H)^Ls - (1-H)^Ls) / ((1+H)^Ls + (1-H)^Ls)  (Sec. 2)."""
    n = H.shape[0]
    A = np.linalg.matrix_power(np.eye(n) + H, Ls)
    B = np.linalg.matrix_power(np.eye(n) - H, Ls)
    return np.linalg.solve((A + B).T, (A - B).T).T


def overlap_symbol(p, M5, b5, c5, Ls, m):
    """D_ov(m) = (1+m)/2 + (1-m)/2 g5 eps_Ls(g5 D_Moebius)  (App. A form)."""
    H = G5 @ mobius_kernel(wilson_symbol(p, M5), b5, c5)
    return 0.5 * (1 + m) * np.eye(4) + 0.5 * (1 - m) * G5 @ polar_sign(H, Ls)


def perm_matrix(Ls):
    """P_{ss'} = delta_{ss'} P- + delta_{s',(s+1) mod Ls} P+  (Sec. 2.2)."""
    P = np.zeros((4 * Ls, 4 * Ls), complex)
    for s in range(Ls):
        P[4 * s:4 * s + 4, 4 * s:4 * s + 4] += PM
        sp = (s + 1) % Ls
        P[4 * s:4 * s + 4, 4 * sp:4 * sp + 4] += PP
    return P


def reflection(Ls):
    """R_{ss'} = delta_{Ls+1-s, s'} on the 4Ls index."""
    R = np.zeros((4 * Ls, 4 * Ls))
    for s in range(Ls):
        R[4 * s:4 * s + 4, 4 * (Ls - 1 - s):4 * (Ls - 1 - s) + 4] = np.eye(4)
    return R


def overlap_symbol_sdep(p, M5, b5s, c5s, m):
    """D_ov(m) of the general operator with per-slice coefficients (Sec. 2.2):
    (1+m)/2 + (1-m)/2 g5 (X - 1)(X + 1)^-1 with X = T_1^-1 T_2^-1 ... T_Ls^-1,
    T_s = (1 - H_s)/(1 + H_s), H_s = g5 (b5(s)+c5(s)) D_W (2 + (b5(s)-c5(s)) D_W)^-1."""
    Dw = wilson_symbol(p, M5)
    I4 = np.eye(4)
    X = I4.astype(complex)
    for b, c in zip(b5s, c5s):
        H = G5 @ np.linalg.solve(2 * I4 + (b - c) * Dw, (b + c) * Dw)
        X = X @ np.linalg.solve(I4 - H, I4 + H)
    return 0.5 * (1 + m) * I4 + 0.5 * (1 - m) * G5 @ (X - I4) @ np.linalg.inv(X + I4)
