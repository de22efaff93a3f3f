"""Direct convex minimisation of the discrete model on tiny grids (oracle pin).

The discrete model of Sec. 2 is: minimise sum J(K x + c) subject to
A x = f_b^-.  On grids small enough for dense algebra this is solved here
without Algorithm 1: the affine constraint set is parametrised as
x = x_p + Z w (Z an orthonormal basis of the null space of A, from the
printed matrices in ``literal``), and the smooth convex objective (v > 0 on
the path) is minimised in w by damped Newton steps with a backtracking line
search that keeps v > 0.  The result is the minimiser that Algorithm 1
converges to, computed by an unrelated route.
"""
from __future__ import annotations

import numpy as np
from scipy import linalg
from scipy import sparse as sp

from . import literal
from .grid import Grid


def _objective_parts(K, c, x, n):
    z = K @ x + c
    u = z[: 3 * n].reshape(3, n)
    v = z[3 * n:]
    return u, v


def minimise(g: Grid, f0, f1, tol: float = 1e-13, max_iter: int = 200):
    """Return (x, cost) with x the flat primal (m_x, m_y, m_c, f)."""
    f0 = np.asarray(f0, dtype=np.float64)
    f1 = np.asarray(f1, dtype=np.float64)
    n = g.n_centre
    K = literal.K_sparse(g)
    A = literal.A_sparse(g).toarray()
    c = literal.c_vector(g, f0, f1)
    _, fbm = literal.fb_vectors(g, f0, f1)
    Z = linalg.null_space(A)

    # feasible start with v > 0: linear interpolation of the density in time,
    # momentum from the least-squares solution of the remaining constraint
    n_sp = g.X * g.Y * g.C
    n_m = A.shape[1] - (g.P - 1) * n_sp
    t = np.arange(1, g.P) / g.P
    f_lin = ((1 - t)[:, None] * f0.ravel()[None] + t[:, None] * f1.ravel()[None]).ravel()
    A_m, A_f = A[:, :n_m], A[:, n_m:]
    m0 = np.linalg.lstsq(A_m, fbm - A_f @ f_lin, rcond=None)[0]
    x0 = np.concatenate([m0, f_lin])
    KZ = K @ Z

    def obj(x):
        u, v = _objective_parts(K, c, x, n)
        if np.any(v <= 0):
            return np.inf
        return float(np.sum(np.sum(u * u, axis=0) / (2 * v)))

    x = x0
    for _ in range(max_iter):
        u, v = _objective_parts(K, c, x, n)
        # gradient and Hessian of J w.r.t. (u, v), per node
        gu = u / v                                   # (3, n)
        gv = -np.sum(u * u, axis=0) / (2 * v * v)
        grad_z = np.concatenate([gu.ravel(), gv])
        gw = KZ.T @ grad_z
        if np.linalg.norm(gw) <= tol * max(1.0, obj(x)):
            break
        # Hessian blocks: d2/du2 = I / v, d2/dudv = -u / v^2, d2/dv2 = |u|^2 / v^3
        idx = np.arange(n)
        rows, cols, vals = [], [], []
        for i in range(3):
            rows += [i * n + idx, i * n + idx, 3 * n + idx]
            cols += [i * n + idx, 3 * n + idx, i * n + idx]
            vals += [1.0 / v, -u[i] / v ** 2, -u[i] / v ** 2]
        rows.append(3 * n + idx)
        cols.append(3 * n + idx)
        vals.append(np.sum(u * u, axis=0) / v ** 3)
        H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(4 * n, 4 * n))
        Hw = KZ.T @ (H @ KZ)
        step = -np.linalg.lstsq(Hw + 1e-14 * np.eye(Hw.shape[0]), gw, rcond=None)[0]
        dx = Z @ step
        f_cur = obj(x)
        # largest step that keeps v > 0, then Armijo backtracking
        dv = (K @ dx)[3 * n:]
        neg = dv < 0
        alpha = 1.0
        if neg.any():
            alpha = min(1.0, 0.95 * float(np.min(-v[neg] / dv[neg])))
        while alpha > 1e-12:
            xn = x + alpha * dx
            fn = obj(xn)
            if np.isfinite(fn) and fn <= f_cur + 1e-4 * alpha * float(gw @ step):
                break
            alpha *= 0.5
        if alpha <= 1e-12:
            break
        x = x + alpha * dx
    cost = g.cell_volume() * obj(x)
    return x, cost
