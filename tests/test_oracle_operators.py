"""Pins of the oracle's staggered-grid stencils against the paper's printed
matrices (Sec. 2 and Sec. 3), on tiny grids with mixed boundary conditions."""
import numpy as np
import pytest

from oracle import grid as G
from oracle import literal as L

SHAPES = [
    # X, Y, C, P, bc(x, y, c)
    (4, 5, 3, 4, (G.NEUMANN, G.NEUMANN, G.PERIODIC)),   # RGB mixed BC, X != Y
    (3, 2, 3, 3, (G.PERIODIC, G.NEUMANN, G.PERIODIC)),  # odd periodic x
    (5, 1, 1, 4, (G.NEUMANN, G.NEUMANN, G.NEUMANN)),    # 1D Neumann
    (6, 1, 1, 3, (G.PERIODIC, G.NEUMANN, G.NEUMANN)),   # 1D periodic, even n
    (4, 3, 2, 5, (G.NEUMANN, G.PERIODIC, G.NEUMANN)),   # Neumann colour
]


def _rand_primal(g, rng):
    return tuple(rng.standard_normal(g.m_shape(a)) for a in range(3)) + (
        rng.standard_normal(g.f_shape),)


@pytest.mark.parametrize("shape", SHAPES)
def test_stencils_equal_kronecker_matrices(shape, rng):
    X, Y, C, P, bc = shape
    g = G.Grid(X, Y, C, P, bc)
    x = _rand_primal(g, rng)
    f0 = rng.uniform(0.1, 1.0, (C, Y, X))
    f1 = rng.uniform(0.1, 1.0, (C, Y, X))
    K = L.K_matrix(g)
    A = L.A_matrix(g)
    c = L.c_vector(g, f0, f1)
    _, fbm = L.fb_vectors(g, f0, f1)
    xv = G.flat(x)
    np.testing.assert_allclose(G.flat(G.K_apply(g, x, f0, f1)), K @ xv + c, atol=1e-13)
    np.testing.assert_allclose(G.A_residual(g, x, f0, f1).ravel(), A @ xv - fbm, atol=1e-12)
    w = tuple(rng.standard_normal(g.centre_shape) for _ in range(4))
    np.testing.assert_allclose(G.flat(G.KT_apply(g, w)), K.T @ G.flat(w), atol=1e-13)
    phi = rng.standard_normal(g.centre_shape)
    np.testing.assert_allclose(G.flat(G.AT_apply(g, phi)), A.T @ phi.ravel(), atol=1e-12)


@pytest.mark.parametrize("shape", SHAPES)
def test_adjoint_dot_products(shape, rng):
    X, Y, C, P, bc = shape
    g = G.Grid(X, Y, C, P, bc)
    x = _rand_primal(g, rng)
    w = tuple(rng.standard_normal(g.centre_shape) for _ in range(4))
    lhs = float(G.flat(G.K_lin(g, x)) @ G.flat(w))
    rhs = float(G.flat(x) @ G.flat(G.KT_apply(g, w)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    phi = rng.standard_normal(g.centre_shape)
    lhs = float(G.A_lin(g, x).ravel() @ phi.ravel())
    rhs = float(G.flat(x) @ G.flat(G.AT_apply(g, phi)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_boundary_vectors_as_printed():
    g = G.Grid(3, 1, 1, 4)
    f0 = np.array([[[1.0, 2.0, 3.0]]])
    f1 = np.array([[[4.0, 5.0, 6.0]]])
    plus, minus = L.fb_vectors(g, f0, f1)
    np.testing.assert_array_equal(plus, [0.5, 1, 1.5, 0, 0, 0, 0, 0, 0, 2, 2.5, 3])
    np.testing.assert_array_equal(minus, [4, 8, 12, 0, 0, 0, 0, 0, 0, -16, -20, -24])
    np.testing.assert_array_equal(G.fb_plus(g, f0, f1).ravel(), plus)
    np.testing.assert_array_equal(G.fb_minus(g, f0, f1).ravel(), minus)


@pytest.mark.parametrize("n", [3, 4, 7])
def test_laplacians_from_differences(n):
    """A A^T blocks: D_n,per^T D_n,per = n^2 Delta_n,per and
    D_p^T D_p = p^2 Delta_p (Sec. 3)."""
    D = L.D_per(n, float(n))
    np.testing.assert_allclose(D.T @ D, n * n * L.Lap_per(n), atol=1e-12)
    Dp = L.D_band(n, float(n))
    np.testing.assert_allclose(Dp.T @ Dp, n * n * L.Lap_neu(n), atol=1e-12)


def test_printed_matrix_entries():
    S = L.S_per(4)
    np.testing.assert_array_equal(S, 0.5 * np.array(
        [[1, 0, 0, 1], [1, 1, 0, 0], [0, 1, 1, 0], [0, 0, 1, 1]]))
    D = L.D_per(4, 4.0)
    np.testing.assert_array_equal(D, 4.0 * np.array(
        [[-1, 0, 0, 1], [1, -1, 0, 0], [0, 1, -1, 0], [0, 0, 1, -1]]))
    np.testing.assert_array_equal(L.S_band(3), 0.5 * np.array([[1, 1, 0], [0, 1, 1]]))
    np.testing.assert_array_equal(L.D_band(3, 3.0), 3.0 * np.array([[-1, 1, 0], [0, -1, 1]]))


@pytest.mark.parametrize("n,p,expect", [(6, 3, 3), (5, 3, 0), (4, 2, 2)])
def test_null_space_of_SM_periodic(n, p, expect):
    """Proof of Thm. 1: N(S_M) = {w (x) (1,-1,...)} for periodic even n,
    trivial otherwise."""
    g = G.Grid(n, 1, 1, p, (G.PERIODIC, G.NEUMANN, G.NEUMANN))
    SM, _, _, _ = L.operators(g)
    S = SM[0].toarray()
    nullity = S.shape[1] - np.linalg.matrix_rank(S)
    assert nullity == expect
    if expect:
        alt = np.array([(-1.0) ** j for j in range(n)])
        w = np.arange(1.0, p + 1)
        np.testing.assert_allclose(S @ np.kron(w, alt), 0.0, atol=1e-14)
