"""Staggered-grid discretisation of the dynamic transport model (oracle).

Follows Sec. 2 of the paper ("Discretization (Spatial 1D)", the discrete model
with S_M, S_F, D_M, D_F and the boundary vectors f_b^+, f_b^-) and its 4D
extension of Remark 2 (Neumann x, y and time; periodic colour).

Conventions (natural, unpadded arrays, float64, last axis fastest):

* centred nodes (cell centres x half-times): shape (P, C, Y, X);
* density f: interior times k = 1..P-1, shape (P-1, C, Y, X); the fixed end
  densities f0 = f(., 0) and f1 = f(., 1) have shape (C, Y, X);
* momentum component m_a along spatial axis a (0 = x, 1 = y, 2 = colour) lives
  on the faces of that axis at half-times.  Face j sits between cells j-1 and
  j.  Neumann (kappa = 1): unknown faces j = 1..n-1, faces 0 and n are zero.
  Periodic (kappa = 0): faces j = 0..n-1, face 0 lies between cells n-1 and 0.

The difference operators carry the factor n_a / extent_a (the paper uses the
unit domain, i.e. the factor n, and p for time).  Flattening a C-ordered
(P, C, Y, X) array gives the paper's column-wise vec ordering with space
fastest inside each time slice, so I_p (x) S acts inside each slice.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

NEUMANN = 0
PERIODIC = 1

# numpy axis of each spatial axis in a (P, C, Y, X) array
_NP_AXIS = {0: 3, 1: 2, 2: 1}


@dataclass(frozen=True)
class Grid:
    """Sizes and boundary conditions of one transport problem.

    X, Y, C: spatial sizes (x, y, colour); P: number of time steps.
    bc: per spatial axis, NEUMANN or PERIODIC.  An axis of size 1 is treated
    as absent (Neumann: it carries no unknown face).
    extent: per spatial axis, the physical length of the axis (default 1).
    """

    X: int
    Y: int
    C: int
    P: int
    bc: tuple = (NEUMANN, NEUMANN, PERIODIC)
    extent: tuple = (1.0, 1.0, 1.0)

    def size(self, a: int) -> int:
        return (self.X, self.Y, self.C)[a]

    def axis_bc(self, a: int) -> int:
        return NEUMANN if self.size(a) == 1 else self.bc[a]

    def scale(self, a: int) -> float:
        """Factor of the spatial forward difference: n / extent."""
        return self.size(a) / float(self.extent[a])

    @property
    def st(self) -> float:
        """Factor of the time difference: p (time interval [0, 1])."""
        return float(self.P)

    def nfaces(self, a: int) -> int:
        n = self.size(a)
        return n - 1 if self.axis_bc(a) == NEUMANN else n

    @property
    def centre_shape(self):
        return (self.P, self.C, self.Y, self.X)

    @property
    def f_shape(self):
        return (self.P - 1, self.C, self.Y, self.X)

    def m_shape(self, a: int):
        s = list(self.centre_shape)
        s[_NP_AXIS[a]] = self.nfaces(a)
        return tuple(s)

    @property
    def n_centre(self) -> int:
        return self.P * self.C * self.Y * self.X

    def cell_volume(self) -> float:
        """Quadrature weight of one centred node: prod_a h_a times h_t."""
        v = 1.0 / self.P
        for a in range(3):
            v *= float(self.extent[a]) / self.size(a)
        return v


# ---- spatial operators along one axis (Sec. 2, S_M and D_M) ----------------

def _sl(ax: int, start, stop):
    idx = [slice(None)] * 4
    idx[ax] = slice(start, stop)
    return tuple(idx)


def _with_walls(m: np.ndarray, ax: int) -> np.ndarray:
    """Neumann faces 0..n: the unknown faces 1..n-1 with zero walls added."""
    shp = list(m.shape)
    shp[ax] = 1
    z = np.zeros(shp)
    return np.concatenate([z, m, z], axis=ax)


def face_avg(g: Grid, m: np.ndarray, a: int) -> np.ndarray:
    """S_M on axis a: face -> cell mean, u[i] = (m[i] + m[i+1]) / 2."""
    ax = _NP_AXIS[a]
    if g.axis_bc(a) == PERIODIC:
        return 0.5 * (m + np.roll(m, -1, axis=ax))
    mp = _with_walls(m, ax)
    return 0.5 * (mp[_sl(ax, 0, -1)] + mp[_sl(ax, 1, None)])


def face_div(g: Grid, m: np.ndarray, a: int) -> np.ndarray:
    """D_M on axis a: forward difference from faces to cells,
    s (m[i+1] - m[i]) with s = n / extent."""
    ax = _NP_AXIS[a]
    s = g.scale(a)
    if g.axis_bc(a) == PERIODIC:
        return s * (np.roll(m, -1, axis=ax) - m)
    mp = _with_walls(m, ax)
    return s * (mp[_sl(ax, 1, None)] - mp[_sl(ax, 0, -1)])


def face_avg_adj(g: Grid, w: np.ndarray, a: int) -> np.ndarray:
    """S_M^T on axis a: cell -> face, face j gets (w[j-1] + w[j]) / 2."""
    ax = _NP_AXIS[a]
    if g.axis_bc(a) == PERIODIC:
        return 0.5 * (np.roll(w, 1, axis=ax) + w)
    return 0.5 * (w[_sl(ax, 0, -1)] + w[_sl(ax, 1, None)])


def face_div_adj(g: Grid, phi: np.ndarray, a: int) -> np.ndarray:
    """D_M^T on axis a: face j gets s (phi[j-1] - phi[j])."""
    ax = _NP_AXIS[a]
    s = g.scale(a)
    if g.axis_bc(a) == PERIODIC:
        return s * (np.roll(phi, 1, axis=ax) - phi)
    return s * (phi[_sl(ax, 0, -1)] - phi[_sl(ax, 1, None)])


# ---- time operators (Sec. 2, S_F, D_F, f_b^+, f_b^-) ----------------------

def _with_ends(f, f0, f1):
    return np.concatenate([f0[None], f, f1[None]], axis=0)   # (P+1, C, Y, X)


def time_avg(g: Grid, f, f0, f1) -> np.ndarray:
    """S_F f + f_b^+: v[k'] = (F[k'] + F[k'+1]) / 2 with F[0] = f0, F[P] = f1."""
    F = _with_ends(f, f0, f1)
    return 0.5 * (F[:-1] + F[1:])


def time_div(g: Grid, f, f0, f1) -> np.ndarray:
    """D_F f - f_b^-: p (F[k'+1] - F[k']) with F[0] = f0, F[P] = f1."""
    F = _with_ends(f, f0, f1)
    return g.st * (F[1:] - F[:-1])


def time_avg_adj(g: Grid, w) -> np.ndarray:
    """S_F^T: interior time k = 1..P-1 gets (w[k-1] + w[k]) / 2."""
    return 0.5 * (w[:-1] + w[1:])


def time_div_adj(g: Grid, phi) -> np.ndarray:
    """D_F^T: interior time k gets p (phi[k-1] - phi[k])."""
    return g.st * (phi[:-1] - phi[1:])


def fb_plus(g: Grid, f0, f1) -> np.ndarray:
    """f_b^+ = (f0, 0, ..., 0, f1) / 2 on the centred grid."""
    out = np.zeros(g.centre_shape)
    out[0] += 0.5 * f0
    out[-1] += 0.5 * f1
    return out


def fb_minus(g: Grid, f0, f1) -> np.ndarray:
    """f_b^- = p (f0, 0, ..., 0, -f1) on the centred grid."""
    out = np.zeros(g.centre_shape)
    out[0] += g.st * f0
    out[-1] -= g.st * f1
    return out


# ---- assembled operators on x = (m_x, m_y, m_c, f) ------------------------

def K_apply(g: Grid, x, f0, f1):
    """(u, v) = K x + c = (S_M m, S_F f + f_b^+); u has three components."""
    mx, my, mc, f = x
    return (face_avg(g, mx, 0), face_avg(g, my, 1), face_avg(g, mc, 2),
            time_avg(g, f, f0, f1))


def K_lin(g: Grid, x):
    """K x without the affine boundary term."""
    z0 = np.zeros(g.centre_shape[1:])
    return K_apply(g, x, z0, z0)


def KT_apply(g: Grid, w):
    """K^T w = (S_M^T w_m, S_F^T w_f)."""
    wx, wy, wc, wf = w
    return (face_avg_adj(g, wx, 0), face_avg_adj(g, wy, 1),
            face_avg_adj(g, wc, 2), time_avg_adj(g, wf))


def A_residual(g: Grid, x, f0, f1) -> np.ndarray:
    """A x - f_b^- = D_M m + D_F f - f_b^- (the discrete continuity residual)."""
    mx, my, mc, f = x
    return (face_div(g, mx, 0) + face_div(g, my, 1) + face_div(g, mc, 2)
            + time_div(g, f, f0, f1))


def A_lin(g: Grid, x) -> np.ndarray:
    z0 = np.zeros(g.centre_shape[1:])
    return A_residual(g, x, z0, z0)


def AT_apply(g: Grid, phi):
    """A^T phi = (D_M^T phi, D_F^T phi)."""
    return (face_div_adj(g, phi, 0), face_div_adj(g, phi, 1),
            face_div_adj(g, phi, 2), time_div_adj(g, phi))


def zeros_primal(g: Grid):
    return (np.zeros(g.m_shape(0)), np.zeros(g.m_shape(1)),
            np.zeros(g.m_shape(2)), np.zeros(g.f_shape))


def zeros_dual(g: Grid):
    return tuple(np.zeros(g.centre_shape) for _ in range(4))


def flat(parts) -> np.ndarray:
    return np.concatenate([np.ravel(p) for p in parts])


def unflat_primal(g: Grid, vec: np.ndarray):
    shapes = [g.m_shape(0), g.m_shape(1), g.m_shape(2), g.f_shape]
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(vec[o:o + n].reshape(s))
        o += n
    return tuple(out)
