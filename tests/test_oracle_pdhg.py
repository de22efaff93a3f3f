"""Pins of the oracle's Algorithm 1: its fixed point against a direct convex
minimiser, the projection of Step 1, conservation laws, symmetries and the
closed-form 1D transport."""
import numpy as np
import pytest

from oracle import direct
from oracle import grid as G
from oracle import literal as L
from oracle import pdhg, transport1d
from synth import inputs

TAU, SIGMA = 10.0, 0.099


def _pair(shape, seed, lo=0.2):
    rng = np.random.default_rng(seed)
    a = rng.uniform(lo, 1.0, shape)
    b = rng.uniform(lo, 1.0, shape)
    return a / a.mean(), b / b.mean()


@pytest.mark.parametrize("shape", [
    (4, 3, 3, 4, (G.NEUMANN, G.NEUMANN, G.PERIODIC)),
    (5, 1, 1, 4, (G.NEUMANN, G.NEUMANN, G.NEUMANN)),
    (5, 1, 1, 3, (G.PERIODIC, G.NEUMANN, G.NEUMANN)),
])
def test_fixed_point_equals_direct_minimiser(shape):
    X, Y, C, P, bc = shape
    g = G.Grid(X, Y, C, P, bc)
    f0, f1 = _pair((C, Y, X), 5)
    xd, cost_d = direct.minimise(g, f0, f1)
    st = pdhg.solve(g, f0, f1, TAU, SIGMA, 3000, record_every=3000)
    h = st.hist[-1]
    assert h["r_prim"] < 1e-12 and h["r_dual"] < 1e-12
    assert h["cost"] == pytest.approx(cost_d, rel=1e-11)
    np.testing.assert_allclose(G.flat(st.x), xd, atol=1e-8)


def test_projection_is_kkt_solution(rng):
    """Pi_{C_d}(a) solves min |x - a|^2 s.t. A x = f_b^- (dense KKT system)."""
    g = G.Grid(3, 4, 3, 3)
    f0, f1 = _pair((3, 4, 3), 9)
    a = tuple(rng.standard_normal(s) for s in
              (g.m_shape(0), g.m_shape(1), g.m_shape(2), g.f_shape))
    p = pdhg.project(g, a, f0, f1)
    A = L.A_matrix(g)
    _, fbm = L.fb_vectors(g, f0, f1)
    n = A.shape[1]
    # A has rank rows-1 (constant mode); drop one row for the KKT solve
    Ar, br = A[1:], fbm[1:]
    KKT = np.block([[np.eye(n), Ar.T], [Ar, np.zeros((Ar.shape[0], Ar.shape[0]))]])
    sol = np.linalg.solve(KKT, np.concatenate([G.flat(a), br]))
    np.testing.assert_allclose(G.flat(p), sol[:n], atol=1e-12)
    # idempotent, and feasible
    pp = pdhg.project(g, p, f0, f1)
    np.testing.assert_allclose(G.flat(pp), G.flat(p), atol=1e-12)
    assert np.abs(G.A_residual(g, p, f0, f1)).max() < 1e-11


def test_projection_ignores_a_gradient_shift(rng):
    """The projection of Step 1 is affine with Pi(a) = Pi(a - A^T phi) for
    every potential phi (A^T phi lies in the range that the projection
    removes): the identity that lets the GPU carry the previous iteration's
    potential and solve only for the change.  Checked against the dense KKT
    solution above through pdhg.project, on a periodic-colour and a 1D
    periodic grid, with a random phi including a constant part."""
    for g in (G.Grid(3, 4, 3, 3), G.Grid(6, 1, 1, 4, (G.PERIODIC, G.NEUMANN, G.NEUMANN))):
        f0, f1 = _pair((g.C, g.Y, g.X), 11)
        a = tuple(rng.standard_normal(s) for s in
                  (g.m_shape(0), g.m_shape(1), g.m_shape(2), g.f_shape))
        phi = rng.standard_normal(g.centre_shape) + 3.0
        shift = G.AT_apply(g, phi)
        b = tuple(ai - si for ai, si in zip(a, shift))
        np.testing.assert_allclose(G.flat(pdhg.project(g, b, f0, f1)),
                                   G.flat(pdhg.project(g, a, f0, f1)), atol=1e-11)
        # and the shift is not trivial
        assert np.linalg.norm(G.flat(shift)) > 1.0


def test_cfg1_shape_invariants():
    """16 x 16 x 3 x 8 RGB workload: r_div at rounding level after every
    projection and exact mass in every time slice."""
    g = G.Grid(16, 16, 3, 8)
    f0, f1 = inputs.cfg1_pair()
    f0, f1 = f0.astype(np.float64), f1.astype(np.float64)
    f1 *= f0.sum() / f1.sum()
    st = pdhg.solve(g, f0, f1, TAU, SIGMA, 60, record_every=20)
    for h in st.hist:
        assert h["r_div"] < 1e-13
        assert h["e_mass"] < 1e-13
    assert st.hist[-1]["cost"] > 0


def test_time_reversal():
    """Swapping f0 and f1 reverses time: f[k] -> f[P-k], m -> -m reversed."""
    g = G.Grid(5, 4, 3, 4)
    f0, f1 = _pair((3, 4, 5), 21)
    a = pdhg.solve(g, f0, f1, TAU, SIGMA, 200)
    b = pdhg.solve(g, f1, f0, TAU, SIGMA, 200)
    np.testing.assert_allclose(b.x[3], a.x[3][::-1], atol=1e-12)
    for i in range(3):
        np.testing.assert_allclose(b.x[i], -a.x[i][::-1], atol=1e-12)


def test_colour_cyclic_shift_equivariance():
    """Periodic colour: cyclically permuting the channels of f0 and f1 permutes
    the solution the same way (the point of Fig. 1)."""
    g = G.Grid(4, 3, 3, 4)
    f0, f1 = _pair((3, 3, 4), 31)
    sh = lambda z: np.roll(z, 1, axis=-3)
    a = pdhg.solve(g, f0, f1, TAU, SIGMA, 150)
    b = pdhg.solve(g, sh(f0), sh(f1), TAU, SIGMA, 150)
    np.testing.assert_allclose(b.x[3], sh(a.x[3]), atol=1e-12)
    np.testing.assert_allclose(b.x[0], sh(a.x[0]), atol=1e-12)
    # colour faces shift with the cells (face c sits between c-1 and c)
    np.testing.assert_allclose(b.x[2], sh(a.x[2]), atol=1e-12)


def test_neumann_colour_is_not_shift_equivariant():
    """With Neumann colour the result depends on the channel order (Fig. 1,
    first row)."""
    bc = (G.NEUMANN, G.NEUMANN, G.NEUMANN)
    g = G.Grid(4, 3, 3, 4, bc)
    f0, f1 = _pair((3, 3, 4), 31)
    sh = lambda z: np.roll(z, 1, axis=-3)
    a = pdhg.solve(g, f0, f1, TAU, SIGMA, 150)
    b = pdhg.solve(g, sh(f0), sh(f1), TAU, SIGMA, 150)
    assert np.abs(b.x[3] - sh(a.x[3])).max() > 1e-3


def test_xy_transpose_and_reflection():
    g = G.Grid(4, 4, 3, 3)
    f0, f1 = _pair((3, 4, 4), 41)
    a = pdhg.solve(g, f0, f1, TAU, SIGMA, 120)
    t = lambda z: np.swapaxes(z, -1, -2)
    b = pdhg.solve(g, t(f0), t(f1), TAU, SIGMA, 120)
    np.testing.assert_allclose(b.x[3], t(a.x[3]), atol=1e-12)
    np.testing.assert_allclose(b.x[1], t(a.x[0]), atol=1e-12)
    # x reflection: cells reverse, interior faces reverse with a sign flip
    r = lambda z: z[..., ::-1]
    c = pdhg.solve(g, r(f0), r(f1), TAU, SIGMA, 120)
    np.testing.assert_allclose(c.x[3], r(a.x[3]), atol=1e-12)
    np.testing.assert_allclose(c.x[0], -r(a.x[0]), atol=1e-12)


def test_constant_density_is_a_fixed_point():
    g = G.Grid(4, 3, 3, 4)
    f = np.ones((3, 3, 4))
    st = pdhg.solve(g, f, f, TAU, SIGMA, 400, record_every=400)
    np.testing.assert_allclose(st.x[3], 1.0, atol=1e-10)
    for i in range(3):
        np.testing.assert_allclose(st.x[i], 0.0, atol=1e-10)
    assert st.hist[-1]["cost"] < 1e-18


def test_scaling_law():
    """Data alpha f with (alpha tau, sigma / alpha) gives alpha times the
    iterates: J is 1-homogeneous and the projection is linear."""
    g = G.Grid(4, 3, 3, 3)
    f0, f1 = _pair((3, 3, 4), 51)
    al = 3.5
    a = pdhg.solve(g, f0, f1, 2.0, 0.3, 50)
    b = pdhg.solve(g, al * f0, al * f1, al * 2.0, 0.3 / al, 50)
    np.testing.assert_allclose(G.flat(b.x), al * G.flat(a.x), rtol=1e-10, atol=1e-12)


def _gauss(n, mu, s):
    x = (np.arange(n) + 0.5) / n
    return np.exp(-0.5 * ((x - mu) / s) ** 2)


def test_transport1d_closed_form_values():
    """Uniform on [0,1] to uniform on [0,1/2]: Q0(s) = s, Q1(s) = s/2,
    (1/2) int (s/2)^2 ds = 1/24.  Shift of a uniform block by d: d^2 / 2."""
    h0 = np.ones(8)
    h1 = np.r_[2 * np.ones(4), np.zeros(4)]
    assert transport1d.w2_half_sq(h0, h1) == pytest.approx(1.0 / 24.0, rel=1e-14)
    a = np.r_[np.zeros(2), 4 * np.ones(2), np.zeros(4)]
    b = np.r_[np.zeros(5), 4 * np.ones(2), np.zeros(1)]
    assert transport1d.w2_half_sq(a, b) == pytest.approx(0.5 * (3 / 8) ** 2, rel=1e-14)
    # interpolant of a translation is the translated block
    mid = transport1d.interpolant_cells(a, b, 0.5)
    np.testing.assert_allclose(mid, np.r_[np.zeros(3), 2, 4, 2, np.zeros(2)], atol=1e-13)


def test_discrete_cost_converges_to_quadratic_transport():
    """1D Neumann: the discrete minimum approaches (1/2) W_2^2 as the grid is
    refined (P = n / 2), by a factor of at least 2.5 per doubling."""
    errs = []
    for n in (32, 64, 128):
        h0 = _gauss(n, 0.3, 0.06) + 1e-3
        h1 = 0.5 * _gauss(n, 0.6, 0.05) + _gauss(n, 0.75, 0.04) + 1e-3
        h0, h1 = h0 / h0.mean(), h1 / h1.mean()
        g = G.Grid(n, 1, 1, n // 2)
        st = pdhg.solve(g, h0[None, None], h1[None, None], TAU, SIGMA, 6000,
                        record_every=6000)
        h = st.hist[-1]
        assert h["r_prim"] < 2e-6 and h["r_dual"] < 2e-6
        w = transport1d.w2_half_sq(h0, h1)
        errs.append(abs(h["cost"] - w) / w)
    assert errs[1] < errs[0] / 2.5
    assert errs[2] < errs[1] / 2.5
    assert errs[2] < 5e-5


def test_state_residuals_at_the_fixed_point_and_without_momentum():
    """Residuals of a state without iterating (Sec. 3, Step 2 applied to the
    current x and b): at the fixed point reached by Algorithm 1 the prox
    returns K x + c itself, so r_prim vanishes and the cost is the direct
    minimiser's objective; a state without momentum (b = 0, f > 0) is a fixed
    point of the prox, J = 0 there, so r_prim and the cost are 0."""
    g = G.Grid(5, 1, 1, 4, (G.NEUMANN, G.NEUMANN, G.NEUMANN))
    f0, f1 = _pair((1, 1, 5), 5)
    _, cost_d = direct.minimise(g, f0, f1)
    st = pdhg.solve(g, f0, f1, TAU, SIGMA, 3000)
    r = pdhg.state_residuals(g, st.x, st.b, f0, f1, SIGMA)
    assert r["r_prim"] < 1e-10
    assert r["cost"] == pytest.approx(cost_d, rel=1e-10)
    assert r["r_div"] < 1e-12 and r["e_mass"] < 1e-12
    # no momentum, positive density, zero dual
    g = G.Grid(4, 3, 3, 4)
    f0, f1 = _pair((3, 3, 4), 7)
    x = G.zeros_primal(g)
    x = (x[0], x[1], x[2], np.full(g.f_shape, 0.7))
    r = pdhg.state_residuals(g, x, G.zeros_dual(g), f0, f1, SIGMA)
    assert r["r_prim"] == 0.0 and r["cost"] == 0.0
    # a state off the fixed point has a positive primal residual
    st = pdhg.solve(g, f0, f1, TAU, SIGMA, 5)
    assert pdhg.state_residuals(g, st.x, st.b, f0, f1, SIGMA)["r_prim"] > 1e-6
