"""Pointwise proximal map of the kinetic energy J (oracle).

Sec. 3, Step 2: at each centred node, with a_m (a vector with one entry per
spatial axis) and a_f,

    (u, v) = argmin |u|^2 / (2 v) + sigma/2 |u - a_m|^2 + sigma/2 (v - a_f)^2

over the domain of J (Sec. 2: J = |m|^2 / (2 f) for f > 0, J(0, 0) = 0,
+inf otherwise).  Zeroing the gradient gives u = sigma v a_m / (1 + sigma v)
and the cubic 2 (1 + sigma v)^2 (v - a_f) - sigma |a_m|^2 = 0, solved here by
Newton steps (the paper's suggestion).

Reading of the branch (the paper states only the cubic): a positive root
exists iff 2 a_f + sigma |a_m|^2 > 0; it is then unique.  Otherwise the
minimiser is (0, 0), the only point of dom J with v <= 0.  Newton starts at
v0 = max(a_f, 0) + sigma |a_m|^2 / 2, right of the root where the cubic is
increasing and convex, so the iterates decrease monotonically to the root.
"""
from __future__ import annotations

import numpy as np


def J(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Perspective energy per node; u has the spatial axes on axis 0."""
    u2 = np.sum(np.asarray(u) ** 2, axis=0)
    v = np.asarray(v, dtype=np.float64)
    out = np.full(v.shape, np.inf)
    pos = v > 0
    out[pos] = u2[pos] / (2.0 * v[pos])
    out[(v == 0) & (u2 == 0)] = 0.0
    return out


def cubic(v, a2, af, sigma):
    """f(v) = 2 (1 + sigma v)^2 (v - a_f) - sigma |a_m|^2."""
    return 2.0 * (1.0 + sigma * v) ** 2 * (v - af) - sigma * a2


def solve_v(a2: np.ndarray, af: np.ndarray, sigma: float,
            rtol: float = 1e-15, max_iter: int = 200) -> np.ndarray:
    """Positive root of the cubic where it exists, else 0."""
    a2 = np.asarray(a2, dtype=np.float64)
    af = np.asarray(af, dtype=np.float64)
    shape = np.broadcast(a2, af).shape
    a2 = np.broadcast_to(a2, shape).ravel()
    af = np.broadcast_to(af, shape).ravel()
    active = 2.0 * af + sigma * a2 > 0.0
    v = np.where(active, np.maximum(af, 0.0) + 0.5 * sigma * a2, 0.0)
    todo = np.flatnonzero(active)
    for _ in range(max_iter):
        if todo.size == 0:
            break
        vt, at, ft = v[todo], a2[todo], af[todo]
        w = 1.0 + sigma * vt
        g = 2.0 * w * w * (vt - ft) - sigma * at
        dg = 4.0 * sigma * w * (vt - ft) + 2.0 * w * w
        vn = vt - g / dg
        vn = np.where(vn > 0.0, vn, 0.5 * vt)   # guard: stay in v > 0
        v[todo] = vn
        todo = todo[np.abs(vn - vt) > rtol * vn]
    v = v.reshape(shape)
    return v


def solve_v_closed(a2: np.ndarray, af: np.ndarray, sigma: float) -> np.ndarray:
    """Positive root of the cubic in closed form (Cardano), else 0.

    With w = 1 + sigma v the cubic 2 (1 + sigma v)^2 (v - a_f) = sigma |a_m|^2
    becomes w^3 - beta w^2 - gamma = 0, beta = 1 + sigma a_f,
    gamma = sigma^2 |a_m|^2 / 2 >= 0.  It has exactly one positive root, and
    that root exceeds 1 (v > 0) iff the value at w = 1,
    -sigma (a_f + sigma |a_m|^2 / 2), is negative: the branch condition of
    solve_v.  Two forms avoid cancellation:
      beta > 0: w = beta / 3 + t with the depressed cubic t^3 + p t + q = 0,
        p = -beta^2 / 3, q = -2 beta^3 / 27 - gamma; its discriminant
        (q/2)^2 + (p/3)^3 = gamma^2 / 4 + gamma beta^3 / 27 >= 0, so
        t = A + beta^2 / (9 A), A = cbrt(-q/2 + sqrt(disc)) > 0 (all terms
        positive);
      beta <= 0 (then gamma > 1 where the root is active): s = 1 / w solves
        the depressed cubic s^3 + (beta / gamma) s - 1 / gamma = 0, whose
        roots sum to 0 and multiply to 1 / gamma > 0, so exactly one is
        positive.  With P = -beta / (3 gamma) >= 0 and H = 1 / (2 gamma):
        disc = H^2 - P^3 >= 0 gives s = A + P / A, A = cbrt(H + sqrt(disc));
        disc < 0 gives s = 2 sqrt(P) cos(acos(H / P^{3/2}) / 3), the argument
        in (0, 1] where the largest root is well conditioned."""
    a2 = np.asarray(a2, dtype=np.float64)
    af = np.asarray(af, dtype=np.float64)
    a2, af = np.broadcast_arrays(a2, af)
    active = 2.0 * af + sigma * a2 > 0.0
    beta = 1.0 + sigma * af
    gamma = 0.5 * sigma * sigma * a2
    w = np.ones(beta.shape)
    pos = active & (beta > 0.0)
    if np.any(pos):
        b, g = beta[pos], gamma[pos]
        A = np.cbrt(b ** 3 / 27.0 + 0.5 * g + np.sqrt(0.25 * g * g + g * b ** 3 / 27.0))
        w[pos] = b / 3.0 + A + b * b / (9.0 * A)
    neg = active & (beta <= 0.0)
    if np.any(neg):
        b, g = beta[neg], gamma[neg]
        P = -b / (3.0 * g)
        H = 0.5 / g
        disc = H * H - P ** 3
        sv = np.empty(b.shape)
        one = disc >= 0.0
        A = np.cbrt(H[one] + np.sqrt(disc[one]))
        sv[one] = A + P[one] / A
        thr = ~one
        sv[thr] = 2.0 * np.sqrt(P[thr]) * np.cos(np.arccos(np.minimum(H[thr] / P[thr] ** 1.5, 1.0)) / 3.0)
        w[neg] = 1.0 / sv
    return np.where(active, np.maximum((w - 1.0) / sigma, 0.0), 0.0)


def prox(am: np.ndarray, af: np.ndarray, sigma: float):
    """(u, v) = prox of J / sigma at (a_m, a_f); a_m has the axes on axis 0."""
    am = np.asarray(am, dtype=np.float64)
    a2 = np.sum(am ** 2, axis=0)
    v = solve_v(a2, af, sigma)
    u = sigma * v / (1.0 + sigma * v) * am
    return u, v
