"""Algorithm 1 of the paper (PDHG for the discrete model), FP64 oracle.

The algorithm is Chambolle-Pock in the form of Algorithm 8 of [BSS14], as the
paper states in Sec. 3.  Initialisation: m = 0, f = 0, b = b_bar = 0, theta = 1
and tau sigma < 1.  One iteration r -> r + 1:

1. a = x^r - tau sigma K^T b_bar^r, with x = (m, f) and K^T = (S_M^T, S_F^T);
   x^{r+1} = Pi_{C_d}(a) = a - A^T (A A^T)^+ (A a - f_b^-)  (Step 1);
2. z^{r+1} = prox of J / sigma at K x^{r+1} + c + b^r, with c = (0, f_b^+)
   (Step 2, pointwise);
3. b^{r+1} = b^r + K x^{r+1} + c - z^{r+1};
4. b_bar^{r+1} = b^{r+1} + theta (b^{r+1} - b^r).

Reported quantities (the paper defines none; it runs a fixed iteration count):

* cost   = cell volume * sum J(z), an approximation of the transport energy;
* r_prim = ||K x + c - z|| / ||z||  (equals ||b^{r+1} - b^r|| / ||z||);
* r_dual = ||x^{r+1} - x^r|| / ||x^{r+1}||;
* r_div  = ||A x - f_b^-|| / ||f_b^-||  (the constraint of Step 1);
* e_mass = max_k |sum f(., k/p) - M0| / M0 over the interior time slices.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import grid as G
from . import poisson, prox


@dataclass
class State:
    x: tuple                      # (m_x, m_y, m_c, f) natural arrays
    b: tuple                      # dual, four centred arrays
    bbar: tuple
    it: int = 0
    z: tuple = None               # last prox output (u_x, u_y, u_c, v)
    hist: list = field(default_factory=list)


def init_cold(g: G.Grid) -> State:
    return State(x=G.zeros_primal(g), b=G.zeros_dual(g), bbar=G.zeros_dual(g))


def project(g: G.Grid, a, f0, f1):
    """Pi_{C_d}(a) = a - A^T (A A^T)^+ (A a - f_b^-) (Sec. 3, Step 1)."""
    r = G.A_residual(g, a, f0, f1)
    phi = poisson.solve(g, r)
    corr = G.AT_apply(g, phi)
    return tuple(ai - ci for ai, ci in zip(a, corr))


def _norm(parts) -> float:
    return float(np.sqrt(sum(np.sum(np.asarray(p) ** 2) for p in parts)))


def step(g: G.Grid, st: State, f0, f1, tau: float, sigma: float,
         theta: float = 1.0, record: bool = False) -> State:
    """One iteration of Algorithm 1."""
    # Step 1: a = x - tau sigma K^T b_bar, then project onto C_d
    ktb = G.KT_apply(g, st.bbar)
    a = tuple(xi - tau * sigma * ki for xi, ki in zip(st.x, ktb))
    x_new = project(g, a, f0, f1)
    # Step 2: pointwise prox at K x + c + b
    kx = G.K_apply(g, x_new, f0, f1)
    am = np.stack([kx[i] + st.b[i] for i in range(3)])
    af = kx[3] + st.b[3]
    u, v = prox.prox(am, af, sigma)
    z = (u[0], u[1], u[2], v)
    # Steps 3-4: dual ascent and extrapolation
    b_new = tuple(st.b[i] + kx[i] - z[i] for i in range(4))
    bbar = tuple(b_new[i] + theta * (b_new[i] - st.b[i]) for i in range(4))
    out = State(x=x_new, b=b_new, bbar=bbar, it=st.it + 1, z=z, hist=st.hist)
    if record:
        out.hist.append(residuals(g, out, f0, f1, x_prev=st.x))
    return out


def residuals(g: G.Grid, st: State, f0, f1, x_prev=None) -> dict:
    """cost, r_prim, r_dual, r_div and e_mass of the state after an iteration."""
    kx = G.K_apply(g, st.x, f0, f1)
    z = st.z
    out = {"it": st.it}
    if z is not None:
        u = np.stack(z[:3])
        out["cost"] = g.cell_volume() * float(np.sum(prox.J(u, z[3])))
        out["r_prim"] = _norm([kx[i] - z[i] for i in range(4)]) / max(_norm(z), 1e-300)
    if x_prev is not None:
        out["r_dual"] = _norm([a - b for a, b in zip(st.x, x_prev)]) / max(_norm(st.x), 1e-300)
    out["r_div"] = _norm([G.A_residual(g, st.x, f0, f1)]) / _norm([G.fb_minus(g, f0, f1)])
    M0 = float(np.sum(f0))
    f = st.x[3]
    if f.shape[0] > 0:
        sl = np.sum(f, axis=(1, 2, 3))
        out["e_mass"] = float(np.max(np.abs(sl - M0)) / M0)
    else:
        out["e_mass"] = 0.0
    return out


def state_residuals(g: G.Grid, x, b, f0, f1, sigma: float) -> dict:
    """Residuals of a state (x, b) without iterating: z = prox of J / sigma at
    K x + c + b (Sec. 3, Step 2, as in the next iteration's prox but with the
    current x), then r_prim = ||K x + c - z|| / ||z|| and cost = cell volume *
    sum J(z); at a fixed point of Algorithm 1 z = K x + c, so r_prim = 0 and
    the cost is the objective at x.  Also r_div and e_mass of x."""
    f0 = np.asarray(f0, dtype=np.float64)
    f1 = np.asarray(f1, dtype=np.float64)
    kx = G.K_apply(g, x, f0, f1)
    am = np.stack([kx[i] + b[i] for i in range(3)])
    af = kx[3] + b[3]
    u, v = prox.prox(am, af, sigma)
    z = (u[0], u[1], u[2], v)
    out = {
        "cost": g.cell_volume() * float(np.sum(prox.J(u, v))),
        "r_prim": _norm([kx[i] - z[i] for i in range(4)]) / max(_norm(z), 1e-300),
        "r_div": _norm([G.A_residual(g, x, f0, f1)]) / _norm([G.fb_minus(g, f0, f1)]),
    }
    M0 = float(np.sum(f0))
    f = x[3]
    out["e_mass"] = float(np.max(np.abs(np.sum(f, axis=(1, 2, 3)) - M0)) / M0) if f.shape[0] else 0.0
    return out


def solve(g: G.Grid, f0, f1, tau: float, sigma: float, iters: int,
          theta: float = 1.0, state: State = None, record_every: int = 0) -> State:
    """Run Algorithm 1 for a fixed number of iterations from a cold start
    (or from ``state``).  f0, f1: arrays of shape (C, Y, X), upcast to FP64."""
    f0 = np.asarray(f0, dtype=np.float64)
    f1 = np.asarray(f1, dtype=np.float64)
    st = init_cold(g) if state is None else state
    for i in range(iters):
        rec = record_every > 0 and ((i + 1) % record_every == 0 or i + 1 == iters)
        st = step(g, st, f0, f1, tau, sigma, theta, record=rec)
    return st


def transport_cost(g: G.Grid, x, f0, f1) -> float:
    """cell volume * sum J(K x + c): the objective of the discrete model."""
    kx = G.K_apply(g, x, np.asarray(f0, float), np.asarray(f1, float))
    return g.cell_volume() * float(np.sum(prox.J(np.stack(kx[:3]), kx[3])))
