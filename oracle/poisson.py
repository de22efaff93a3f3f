"""Pseudo-inverse of A A^T by fast transforms (oracle).

Sec. 3, Step 1: the projection onto C_d needs (A A^T)^+ = Q diag(1/lambda) Q^T
with 1/lambda replaced by 0 where lambda = 0.  A A^T is a sum of one
Laplacian per axis: n^2 Delta_n,per (periodic axis), n^2 Delta_n (Neumann
axis) and p^2 Delta_p (time).  Delta_n,per is diagonalised by the Fourier
matrix with eigenvalues 4 sin^2(j pi / n), Delta_p by the orthonormal DCT-II
matrix C_p with eigenvalues 4 sin^2(j pi / (2p)).  Remark 2 extends this to 4D
with Neumann x, y, time and periodic colour.

Here the DCT-II is scipy's orthonormal ``dct(type=2, norm='ortho')`` (equal to
C_p as printed) and the Fourier transform is numpy's FFT.
"""
from __future__ import annotations

import numpy as np
from scipy import fft as sfft

from .grid import Grid, PERIODIC, _NP_AXIS


def axis_eigs(n: int, bc: int, s: float) -> np.ndarray:
    """Eigenvalues of s^2 Delta along one axis: 4 s^2 sin^2(j pi / n) periodic,
    4 s^2 sin^2(j pi / (2 n)) Neumann."""
    j = np.arange(n, dtype=np.float64)
    if bc == PERIODIC:
        return 4.0 * s * s * np.sin(np.pi * j / n) ** 2
    return 4.0 * s * s * np.sin(np.pi * j / (2.0 * n)) ** 2


def eigenvalues(g: Grid) -> np.ndarray:
    """lambda(j_t, j_c, j_y, j_x) of A A^T, shape (P, C, Y, X)."""
    lam = np.zeros(g.centre_shape)
    lam += axis_eigs(g.P, 0, g.st)[:, None, None, None]
    for a in range(3):
        e = axis_eigs(g.size(a), g.axis_bc(a), g.scale(a))
        shp = [1, 1, 1, 1]
        shp[_NP_AXIS[a]] = g.size(a)
        lam = lam + e.reshape(shp)
    return lam


def solve(g: Grid, r: np.ndarray) -> np.ndarray:
    """phi = (A A^T)^+ r for r of shape (P, C, Y, X)."""
    neu_axes = [0] + [_NP_AXIS[a] for a in range(3) if g.axis_bc(a) != PERIODIC]
    per_axes = [_NP_AXIS[a] for a in range(3) if g.axis_bc(a) == PERIODIC]
    z = np.asarray(r, dtype=np.float64)
    for ax in neu_axes:
        z = sfft.dct(z, type=2, norm="ortho", axis=ax)
    zc = z.astype(np.complex128)
    for ax in per_axes:
        zc = np.fft.fft(zc, axis=ax)
    lam = eigenvalues(g)
    inv = np.zeros_like(lam)
    nz = lam > 0.0
    inv[nz] = 1.0 / lam[nz]
    zc = zc * inv
    for ax in per_axes:
        zc = np.fft.ifft(zc, axis=ax)
    z = zc.real
    for ax in neu_axes:
        z = sfft.idct(z, type=2, norm="ortho", axis=ax)
    return z
