"""Pins of the oracle's pseudo-inverse of A A^T (Sec. 3 Step 1, Remark 2)."""
import numpy as np
import pytest
from scipy import fft as sfft

from oracle import grid as G
from oracle import literal as L
from oracle import poisson

SHAPES = [
    (4, 5, 3, 4, (G.NEUMANN, G.NEUMANN, G.PERIODIC)),
    (3, 4, 3, 3, (G.NEUMANN, G.NEUMANN, G.PERIODIC)),
    (5, 1, 1, 6, (G.NEUMANN, G.NEUMANN, G.NEUMANN)),
    (6, 1, 1, 4, (G.PERIODIC, G.NEUMANN, G.NEUMANN)),
    (4, 3, 3, 3, (G.NEUMANN, G.NEUMANN, G.NEUMANN)),
]


def _dct_matrix(p):
    """C_p as printed: sqrt(2/p) eps_j cos(j (2k+1) pi / (2p))."""
    j = np.arange(p)[:, None]
    k = np.arange(p)[None, :]
    C = np.sqrt(2.0 / p) * np.cos(j * (2 * k + 1) * np.pi / (2 * p))
    C[0] /= np.sqrt(2.0)
    return C


@pytest.mark.parametrize("p", [2, 3, 8, 11])
def test_dct_matrix_diagonalises_neumann_laplacian(p):
    C = _dct_matrix(p)
    np.testing.assert_allclose(C @ C.T, np.eye(p), atol=1e-13)
    q = 4.0 * np.sin(np.arange(p) * np.pi / (2 * p)) ** 2
    np.testing.assert_allclose(C.T @ np.diag(q) @ C, L.Lap_neu(p), atol=1e-13)
    # scipy's orthonormal DCT-II is the printed C_p
    np.testing.assert_allclose(sfft.dct(np.eye(p), type=2, norm="ortho", axis=0), C, atol=1e-13)


@pytest.mark.parametrize("n", [3, 6, 7])
def test_fourier_diagonalises_periodic_laplacian(n):
    F = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    q = 4.0 * np.sin(np.arange(n) * np.pi / n) ** 2
    np.testing.assert_allclose((F.conj() @ np.diag(q) @ F) / n, L.Lap_per(n), atol=1e-12)


def test_colour_laplacian_is_mean_deviation_split():
    """Delta_3,per = 3 I - J, eigenvalues {0, 3, 3}."""
    np.testing.assert_array_equal(L.Lap_per(3), 3 * np.eye(3) - np.ones((3, 3)))
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(L.Lap_per(3))), [0, 3, 3], atol=1e-14)


@pytest.mark.parametrize("shape", SHAPES)
def test_eigenvalues_match_dense_spectrum(shape):
    X, Y, C, P, bc = shape
    g = G.Grid(X, Y, C, P, bc)
    A = L.A_matrix(g)
    ev = np.sort(np.linalg.eigvalsh(A @ A.T))
    ev2 = np.sort(poisson.eigenvalues(g).ravel())
    np.testing.assert_allclose(ev, ev2, atol=1e-11 * ev.max())
    assert np.sum(ev2 == 0.0) == 1          # only the constant mode


@pytest.mark.parametrize("shape", SHAPES)
def test_solve_equals_dense_pseudo_inverse(shape, rng):
    X, Y, C, P, bc = shape
    g = G.Grid(X, Y, C, P, bc)
    A = L.A_matrix(g)
    r = rng.standard_normal(g.centre_shape)
    phi = poisson.solve(g, r)
    M = A @ A.T
    phi_dense = np.linalg.lstsq(M, r.ravel() - r.mean(), rcond=None)[0]
    phi_dense -= phi_dense.mean()
    np.testing.assert_allclose(phi.ravel(), phi_dense, atol=1e-12 * np.abs(phi_dense).max())
    assert abs(phi.mean()) < 1e-13 * np.abs(phi).max()
    np.testing.assert_allclose(M @ phi.ravel(), r.ravel() - r.mean(), atol=1e-10)


def test_solve_rgb_16x16x3x8_against_sparse_direct(rng):
    """The full RGB workload shape: compare with an iterative solve of the
    literal sparse system."""
    from scipy.sparse.linalg import cg
    g = G.Grid(16, 16, 3, 8)
    A = L.A_sparse(g)
    M = (A @ A.T).tocsr()
    r = rng.standard_normal(g.centre_shape)
    r -= r.mean()
    phi = poisson.solve(g, r)
    np.testing.assert_allclose(M @ phi.ravel(), r.ravel(), atol=1e-9 * np.abs(r).max())
    sol, info = cg(M, r.ravel(), rtol=1e-13, maxiter=5000)
    sol -= sol.mean()
    assert info == 0
    np.testing.assert_allclose(phi.ravel(), sol, atol=1e-9 * np.abs(sol).max())
