"""Closed-form quadratic transport in 1D through quantile functions (oracle pin).

For the quadratic cost of Sec. 1, the optimal transport between two
densities on an interval is the monotone rearrangement: with quantile
functions Q0 = F0^{-1}, Q1 = F1^{-1} of the cumulative distributions, the
minimal energy of the dynamic problem is (1/2) int_0^1 |Q0(s) - Q1(s)|^2 ds
(times the mass) and the geodesic (displacement interpolation, Sec. 1) at
time t has quantile function (1 - t) Q0 + t Q1.

A histogram on n cells of [0, 1] is read as a piecewise-constant density, so
its CDF is piecewise linear and its quantile function is piecewise linear
with jumps across empty cells.  Both quantities are computed exactly here.
"""
from __future__ import annotations

import numpy as np


def _pieces(h: np.ndarray):
    """Linear pieces of Q: cell i with mass maps s in (s_lo, s_hi) onto
    x in (i/n, (i+1)/n)."""
    h = np.asarray(h, dtype=np.float64)
    n = h.size
    cum = np.concatenate([[0.0], np.cumsum(h / n)])
    cum /= cum[-1]
    pos = h > 0
    x_lo = (np.arange(n) / n)[pos]
    return cum[:-1][pos], cum[1:][pos], x_lo, x_lo + 1.0 / n


def _eval(pc, s, side: str):
    """Q at s, as the limit from the right ('right') or the left ('left')."""
    s_lo, s_hi, x_lo, x_hi = pc
    s = np.asarray(s, dtype=np.float64)
    i = np.searchsorted(s_hi, s, side="right" if side == "right" else "left")
    i = np.clip(i, 0, s_hi.size - 1)
    return x_lo[i] + (s - s_lo[i]) / (s_hi[i] - s_lo[i]) * (x_hi[i] - x_lo[i])


def quantile(h: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Right-continuous quantile function of the histogram h at s."""
    return _eval(_pieces(h), s, "right")


def _breaks(p0, p1):
    return np.unique(np.concatenate([p0[0], p0[1], p1[0], p1[1]]))


def w2_half_sq(h0: np.ndarray, h1: np.ndarray) -> float:
    """(1/2) int_0^1 |Q0 - Q1|^2 ds for two histograms on [0, 1], exact."""
    p0, p1 = _pieces(h0), _pieces(h1)
    S = _breaks(p0, p1)
    dl = _eval(p0, S[:-1], "right") - _eval(p1, S[:-1], "right")
    dr = _eval(p0, S[1:], "left") - _eval(p1, S[1:], "left")
    ds = np.diff(S)
    return 0.5 * float(np.sum(ds * (dl * dl + dl * dr + dr * dr) / 3.0))


def interpolant_cells(h0: np.ndarray, h1: np.ndarray, t: float) -> np.ndarray:
    """Cell averages (mean-one scaling) of the displacement interpolation at
    time t, from its quantile function (1 - t) Q0 + t Q1."""
    p0, p1 = _pieces(h0), _pieces(h1)
    S = _breaks(p0, p1)
    ql = (1 - t) * _eval(p0, S[:-1], "right") + t * _eval(p1, S[:-1], "right")
    qr = (1 - t) * _eval(p0, S[1:], "left") + t * _eval(p1, S[1:], "left")
    ds = np.diff(S)
    n = np.asarray(h0).size
    edges = np.arange(n + 1) / n
    # F_t(x) = |{s : Q_t(s) <= x}|, summed over the linear pieces
    x = edges[:, None]
    span = np.where(qr > ql, qr - ql, 1.0)
    frac = np.where(qr > ql, np.clip((x - ql) / span, 0.0, 1.0),
                    (x >= ql).astype(np.float64))
    cdf = np.sum(ds * frac, axis=1)
    return np.diff(cdf) * n
