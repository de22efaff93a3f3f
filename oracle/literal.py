"""The paper's printed matrices, assembled by Kronecker products (oracle).

Used on tiny grids only, as an independent check of the stencil operators in
``grid`` and as the dense system for the pins of the Poisson solve, the
projection and the fixed point.

Printed in Sec. 2: S_n,per, S_p, D_n,per, D_p; S_F = S_p^T (x) I_n,
D_F = -D_p^T (x) I_n; S_M = I_p (x) S_n^T (Neumann) or I_p (x) S_n,per^T
(periodic); D_M = I_p (x) (-D_n^T) (Neumann) or I_p (x) D_n,per^T (periodic);
f_b^+ = (f0, 0, f1)/2 and f_b^- = p (f0, 0, -f1).  Printed in Sec. 3: the
Laplacians Delta_n,per and Delta_p.

Reading: the Neumann S_n and D_n are used but not printed; they are taken to
have the banded form of S_p and D_p with p replaced by n (rows = interior
faces, columns = cells).  The garbled bands of D_n,per and S_n,per are read as
the circulants D_n,per = n (shift - I), S_n,per = (I + shift)/2, with the
corner entries shown in the print.
"""
from __future__ import annotations

import numpy as np
from scipy import sparse as sp

from .grid import Grid, NEUMANN, PERIODIC


def S_per(n: int) -> np.ndarray:
    """S_n,per: entries 1/2 at (j, j) and (j, j-1 mod n)."""
    S = np.zeros((n, n))
    for j in range(n):
        S[j, j] += 0.5
        S[j, (j - 1) % n] += 0.5
    return S


def D_per(n: int, s: float) -> np.ndarray:
    """D_n,per: s * (-1 at (j, j), +1 at (j, j-1 mod n))."""
    D = np.zeros((n, n))
    for j in range(n):
        D[j, j] -= s
        D[j, (j - 1) % n] += s
    return D


def S_band(n: int) -> np.ndarray:
    """S_p (and the Neumann S_n): (n-1) x n, 1/2 at (r, r) and (r, r+1)."""
    S = np.zeros((n - 1, n))
    for r in range(n - 1):
        S[r, r] = 0.5
        S[r, r + 1] = 0.5
    return S


def D_band(n: int, s: float) -> np.ndarray:
    """D_p (and the Neumann D_n): (n-1) x n, s * (-1 at (r, r), +1 at (r, r+1))."""
    D = np.zeros((n - 1, n))
    for r in range(n - 1):
        D[r, r] = -s
        D[r, r + 1] = s
    return D


def Lap_per(n: int) -> np.ndarray:
    """Delta_n,per as printed: 2 on the diagonal, -1 on the cyclic off-diagonals."""
    L = 2.0 * np.eye(n)
    for j in range(n):
        L[j, (j + 1) % n] -= 1.0
        L[j, (j - 1) % n] -= 1.0
    if n == 2:   # both neighbours coincide
        L = np.array([[2.0, -2.0], [-2.0, 2.0]])
    return L


def Lap_neu(p: int) -> np.ndarray:
    """Delta_p as printed: tridiagonal (-1, 2, -1) with corners 1."""
    L = 2.0 * np.eye(p) - np.eye(p, k=1) - np.eye(p, k=-1)
    L[0, 0] = 1.0
    L[-1, -1] = 1.0
    if p == 1:
        L = np.zeros((1, 1))
    return L


def _axis_mats(g: Grid, a: int):
    """(S_a^T, D_M-factor) acting from faces of axis a to its cells."""
    n = g.size(a)
    s = g.scale(a)
    if g.axis_bc(a) == PERIODIC:
        return S_per(n).T, D_per(n, s).T
    if n == 1:
        return np.zeros((1, 0)), np.zeros((1, 0))
    return S_band(n).T, -D_band(n, s).T


def _spatial_kron(g: Grid, a: int, M) -> sp.csr_matrix:
    """I (x) ... (x) M (x) ... (x) I over the (C, Y, X) ordering, M on axis a."""
    out = None
    for ax in (2, 1, 0):                 # slowest (colour) to fastest (x)
        F = sp.csr_matrix(M) if ax == a else sp.identity(g.size(ax), format="csr")
        out = F if out is None else sp.kron(out, F, format="csr")
    return out


def operators(g: Grid):
    """Sparse (S_M blocks, S_F, D_M blocks, D_F) of the discrete model."""
    IP = sp.identity(g.P, format="csr")
    SM, DM = [], []
    for a in range(3):
        S_t, D_t = _axis_mats(g, a)
        SM.append(sp.kron(IP, _spatial_kron(g, a, S_t), format="csr"))
        DM.append(sp.kron(IP, _spatial_kron(g, a, D_t), format="csr"))
    n_sp = g.X * g.Y * g.C
    I_sp = sp.identity(n_sp, format="csr")
    SF = sp.kron(sp.csr_matrix(S_band(g.P).T), I_sp, format="csr")
    DF = sp.kron(sp.csr_matrix(-D_band(g.P, g.st).T), I_sp, format="csr")
    return SM, SF, DM, DF


def K_sparse(g: Grid) -> sp.csr_matrix:
    """K = blockdiag(S_M,x, S_M,y, S_M,c, S_F): primal -> (u_x, u_y, u_c, v)."""
    SM, SF, _, _ = operators(g)
    return sp.block_diag(SM + [SF], format="csr")


def A_sparse(g: Grid) -> sp.csr_matrix:
    """A = (D_M | D_F), acting on (m_x, m_y, m_c, f)."""
    _, _, DM, DF = operators(g)
    return sp.hstack(DM + [DF], format="csr")


def K_matrix(g: Grid) -> np.ndarray:
    return K_sparse(g).toarray()


def A_matrix(g: Grid) -> np.ndarray:
    return A_sparse(g).toarray()


def fb_vectors(g: Grid, f0: np.ndarray, f1: np.ndarray):
    """(f_b^+, f_b^-) as flat vectors over the centred grid."""
    n_sp = g.X * g.Y * g.C
    zeros = np.zeros(n_sp * (g.P - 2))
    plus = 0.5 * np.concatenate([np.ravel(f0), zeros, np.ravel(f1)])
    minus = g.st * np.concatenate([np.ravel(f0), zeros, -np.ravel(f1)])
    return plus, minus


def c_vector(g: Grid, f0, f1) -> np.ndarray:
    """c = (0, f_b^+): the affine part of (u, v) = K x + c."""
    n = g.n_centre
    plus, _ = fb_vectors(g, f0, f1)
    return np.concatenate([np.zeros(3 * n), plus])
