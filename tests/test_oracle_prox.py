"""Pins of the oracle's pointwise prox of J (Sec. 3, Step 2) by brute-force
minimisation of the per-node objective and by its optimality conditions."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import prox


def _objective(p, am, af, sigma):
    u, v = p[:-1], p[-1]
    if v < 0 or (v == 0 and np.any(u != 0)):
        return np.inf
    J = 0.0 if v == 0 else u @ u / (2 * v)
    return J + 0.5 * sigma * (u - am) @ (u - am) + 0.5 * sigma * (v - af) ** 2


def _brute(am, af, sigma):
    """Global minimiser by a grid search over v (u optimal in closed form for
    fixed v) followed by Nelder-Mead refinement in (u, v)."""
    a2 = am @ am
    scale = max(abs(af), np.sqrt(a2), 1.0 / sigma, 1e-6)
    vs = np.concatenate([[0.0], np.geomspace(1e-12 * scale, 1e3 * scale, 4000)])
    best, bp = np.inf, None
    for v in vs:
        u = sigma * v * am / (1 + sigma * v) if v > 0 else np.zeros_like(am)
        val = _objective(np.r_[u, v], am, af, sigma)
        if val < best:
            best, bp = val, np.r_[u, v]
    if bp[-1] > 0:
        res = minimize(lambda p: _objective(p, am, af, sigma), bp, method="Nelder-Mead",
                       options=dict(xatol=1e-14, fatol=1e-16, maxiter=40000))
        if res.fun < best:
            best, bp = res.fun, res.x
    return bp, best


CASES = np.random.default_rng(7)


@pytest.mark.parametrize("case", range(40))
def test_prox_matches_brute_force(case):
    rng = np.random.default_rng(1000 + case)
    d = int(rng.integers(1, 4))
    sigma = 10.0 ** rng.uniform(-3, 3)
    am = rng.standard_normal(d) * 10.0 ** rng.uniform(-3, 3)
    af = rng.standard_normal() * 10.0 ** rng.uniform(-3, 3)
    u, v = prox.prox(am[:, None], np.array([af]), sigma)
    ours = np.r_[u[:, 0], v[0]]
    f_ours = _objective(ours, am, af, sigma)
    bp, f_brute = _brute(am, af, sigma)
    # ours is never worse than the brute-force search
    assert f_ours <= f_brute + 1e-12 * max(1.0, abs(f_brute))
    np.testing.assert_allclose(ours, bp, rtol=1e-5, atol=1e-7 * max(1.0, np.abs(bp).max()))


def test_zero_branch_and_boundary():
    sigma = 2.0
    # 2 a_f + sigma |a_m|^2 <= 0 -> (0, 0)
    u, v = prox.prox(np.array([[0.5]]), np.array([-0.25]), sigma)
    assert v[0] == 0.0 and u[0, 0] == 0.0
    u, v = prox.prox(np.array([[0.1]]), np.array([-1.0]), sigma)
    assert v[0] == 0.0 and u[0, 0] == 0.0
    # just inside the positive branch: small positive root
    u, v = prox.prox(np.array([[0.5]]), np.array([-0.25 + 1e-9]), sigma)
    assert 0.0 < v[0] < 1e-8
    # a_m = 0, a_f > 0: prox is (0, a_f)
    u, v = prox.prox(np.zeros((3, 1)), np.array([1.7]), sigma)
    assert v[0] == pytest.approx(1.7, rel=1e-15) and np.all(u == 0)


def test_optimality_conditions(rng):
    """u / v + sigma (u - a_m) = 0 and -|u|^2 / (2 v^2) + sigma (v - a_f) = 0
    at every positive-branch node (Sec. 3, Step 2)."""
    sigma = 0.37
    am = rng.standard_normal((3, 5000)) * 3
    af = rng.standard_normal(5000) * 3
    u, v = prox.prox(am, af, sigma)
    pos = v > 0
    assert pos.sum() > 1000 and (~pos).sum() > 100
    e1 = u[:, pos] / v[pos] + sigma * (u[:, pos] - am[:, pos])
    e2 = -np.sum(u[:, pos] ** 2, axis=0) / (2 * v[pos] ** 2) + sigma * (v[pos] - af[pos])
    np.testing.assert_allclose(e1, 0.0, atol=1e-11 * np.abs(am).max())
    np.testing.assert_allclose(e2, 0.0, atol=1e-10 * (1 + np.abs(af).max()))
    cub = prox.cubic(v[pos], np.sum(am[:, pos] ** 2, axis=0), af[pos], sigma)
    np.testing.assert_allclose(cub, 0.0, atol=1e-9)
    # the zero branch is exactly where 2 a_f + sigma |a_m|^2 <= 0
    np.testing.assert_array_equal(~pos, 2 * af + sigma * np.sum(am ** 2, axis=0) <= 0)


def test_moreau_identity(rng):
    """prox_{J/sigma}(a) + (1/sigma) proj_K(sigma a) = a, where K = {(alpha,
    beta): beta + |alpha|^2 / 2 <= 0} is the domain of the conjugate of J."""
    sigma = 1.3
    am = rng.standard_normal((2, 200))
    af = rng.standard_normal(200)
    u, v = prox.prox(am, af, sigma)
    pa, pb = sigma * am - sigma * u, sigma * af - sigma * v
    # the complement lies in K (up to rounding), with equality on the positive branch
    assert np.all(pb + 0.5 * np.sum(pa ** 2, axis=0) <= 1e-10)
    pos = v > 0
    np.testing.assert_allclose((pb + 0.5 * np.sum(pa ** 2, axis=0))[pos], 0.0, atol=1e-10)


def test_closed_form_root_matches_newton():
    """The closed-form (Cardano) root agrees with the Newton root, which the
    brute-force minimisation above pins, across six decades of sigma, |a_m|
    and a_f; the comparison is in w = 1 + sigma v, the variable the closed
    form is exact in (v = (w - 1) / sigma loses digits when sigma v << 1)."""
    rng = np.random.default_rng(5)
    n = 3000
    sig = 10.0 ** rng.uniform(-3, 3, n)
    a2 = 10.0 ** rng.uniform(-4, 4, n) * rng.uniform(0, 1, n)
    af = rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 3, n)
    for i in range(n):
        vn = prox.solve_v(a2[i:i + 1], af[i:i + 1], sig[i])[0]
        vc = prox.solve_v_closed(a2[i:i + 1], af[i:i + 1], sig[i])[0]
        if vn == 0.0:
            assert vc == 0.0
        else:
            wn, wc = 1 + sig[i] * vn, 1 + sig[i] * vc
            assert abs(wc - wn) <= 1e-13 * wn, (a2[i], af[i], sig[i], vn, vc)


def test_closed_form_solves_the_cubic():
    """Residual of the cubic at the closed-form root, both forms (beta > 0
    and beta <= 0) and both discriminant signs of the second."""
    cases = [(4.0, 0.5, 1.0), (1e-6, 2.0, 3.0),          # beta > 0
             (50.0, -3.0, 1.0),                          # beta < 0, one real root
             (57.5, -1753.0, 64.0), (30.0, -11.0, 1.0)]  # beta < 0, three real roots
    for a2, af, sig in cases:
        beta, gamma = 1 + sig * af, 0.5 * sig * sig * a2
        v = prox.solve_v_closed(np.array([a2]), np.array([af]), sig)[0]
        assert v > 0
        w = 1 + sig * v
        assert abs(w ** 3 - beta * w ** 2 - gamma) <= 1e-12 * (w ** 3 + abs(beta) * w ** 2 + gamma)
