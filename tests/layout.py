"""Conversion between the library's padded buffers and the oracle's natural
arrays (test glue only; neither side imports it)."""
import numpy as np

from oracle import grid as G


def to_natural(g: G.Grid, F, Mx, My, Mc):
    """Padded single-problem arrays -> (m_x, m_y, m_c, f) of the oracle."""
    F, Mx, My, Mc = (np.asarray(a, dtype=np.float64) for a in (F, Mx, My, Mc))
    f = F[1:g.P]
    mx = Mx if g.axis_bc(0) == G.PERIODIC else Mx[..., 1:]
    my = My if g.axis_bc(1) == G.PERIODIC else My[..., 1:, :]
    mc = Mc if g.axis_bc(2) == G.PERIODIC else Mc[:, 1:]
    return mx, my, mc, f


def to_padded(g: G.Grid, x, f0, f1):
    """Oracle primal -> padded (F, Mx, My, Mc) float32 arrays."""
    mx, my, mc, f = x
    P, C, Y, X = g.centre_shape
    F = np.concatenate([f0[None], f, f1[None]]).astype(np.float32)
    Mx = np.zeros((P, C, Y, X), np.float32)
    My = np.zeros((P, C, Y, X), np.float32)
    Mc = np.zeros((P, C, Y, X), np.float32)
    if g.axis_bc(0) == G.PERIODIC:
        Mx[:] = mx
    else:
        Mx[..., 1:] = mx
    if g.axis_bc(1) == G.PERIODIC:
        My[:] = my
    else:
        My[..., 1:, :] = my
    if g.axis_bc(2) == G.PERIODIC:
        Mc[:] = mc
    else:
        Mc[:, 1:] = mc
    return F, Mx, My, Mc


def rel(a, b) -> float:
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
