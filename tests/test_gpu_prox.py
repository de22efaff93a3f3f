"""GPU tests of the pointwise prox of J (Sec. 3, Step 2) with the Newton
root and with the closed-form (Cardano) root: node by node against the FP64
oracle through ot_dyn_prox_eval, and the whole iteration with the closed
form against the FP64 oracle."""
import numpy as np
import pytest

from oracle import grid as G
from oracle import pdhg
from oracle import prox
from synth import inputs
from tests.layout import rel

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def otdyn():
    import torch
    from paper_1501_04840_amd import otdyn as o
    assert torch.cuda.is_available()
    o.lib()
    return o


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("sigma", [0.01, 0.099, 1.0, 10.0])
def test_device_prox_against_oracle(otdyn, sigma):
    """Six decades of |a_m| and a_f.  FP32 fixes the root of
    g(v) = 2 (1 + sigma v)^2 (v - a_f) - sigma |a_m|^2 to a few ulps of the
    terms it is evaluated with, s = max(v, |a_f|, sigma |a_m|^2 / 2): where v
    is far below s no variant can do better (Newton included).  Newton and
    the closed form + Newton steps are within 2e-6 s everywhere, and where
    sigma v > 1e-3 within 3e-6 relative for 99.9% of the nodes; the closed
    form alone loses digits to v = (w - 1) / sigma (up to 100% where
    sigma v << 1), which is why the steps are taken.  Inactive nodes give
    exactly (0, 0) in every variant."""
    import torch
    _say(f"device prox sigma {sigma}")
    rng = np.random.default_rng(11)
    n = 100000
    am = (rng.standard_normal((3, n)) * 10.0 ** rng.uniform(-3, 3, n)).astype(np.float32)
    af = (rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 3, n)).astype(np.float32)
    am64, af64 = am.astype(np.float64), af.astype(np.float64)
    ur, vr = prox.prox(am64, af64, sigma)
    act = vr > 0
    big = act & (sigma * vr > 1e-3)
    assert big.sum() > 10000
    scale = np.maximum.reduce([vr, np.abs(af64), 0.5 * sigma * (am64 ** 2).sum(0)])
    amg, afg = torch.from_numpy(am).cuda(), torch.from_numpy(af).cuda()
    scaled, p999 = {}, {}
    for kind in (otdyn.OT_PROX_NEWTON, otdyn.OT_PROX_CLOSED, otdyn.OT_PROX_CLOSED_RAW):
        u = torch.full_like(amg, float("nan"))
        v = torch.full_like(afg, float("nan"))
        otdyn.ot_dyn_prox_eval(kind, amg, afg, sigma, u, v)
        torch.cuda.synchronize()
        vg = v.cpu().numpy().astype(np.float64)
        ug = u.cpu().numpy().astype(np.float64)
        assert np.all(vg[~act] == 0) and np.all(ug[:, ~act] == 0), kind
        relv = np.abs(vg - vr) / np.where(act, vr, 1.0)
        scaled[kind] = (np.abs(vg - vr) / scale)[act].max()
        p999[kind] = np.quantile(relv[big], 0.999)
        # u = sigma v a_m / (1 + sigma v): error relative to |a_m|
        du = np.abs(ug - ur).max(axis=0) / np.maximum(np.abs(am).max(axis=0), 1e-30)
        assert du.max() < 1e-6, kind
        if kind != otdyn.OT_PROX_CLOSED_RAW:
            assert scaled[kind] < 2e-6, kind
            assert p999[kind] < 3e-6, kind
            assert relv[big].max() < 2e-4, kind
    raw, closed = otdyn.OT_PROX_CLOSED_RAW, otdyn.OT_PROX_CLOSED
    assert scaled[raw] > 100 * scaled[closed] and p999[raw] > 5 * p999[closed]


def _run(o, g, f0, f1, iters, prox_kind):
    import torch
    d = o.ot_dyn_default_desc(g.X, g.Y, g.C, g.P)
    d.bc[0], d.bc[1], d.bc[2] = g.bc
    d.prox = prox_kind
    prob = o.Problem(d, "cuda")
    prob.set_boundary(torch.from_numpy(np.asarray(f0, np.float32).reshape(1, g.C, g.Y, g.X)),
                      torch.from_numpy(np.asarray(f1, np.float32).reshape(1, g.C, g.Y, g.X)))
    prob.init(o.OT_INIT_COLD)
    return prob


def test_closed_prox_cfg1_300_iterations(otdyn):
    """16 x 16 x 3 x 8, 300 iterations with the closed-form prox: f and the
    cost within 1e-5 of the FP64 oracle (which uses the Newton root)."""
    import torch
    _say("closed-form prox, cfg1 300 iterations")
    g = G.Grid(16, 16, 3, 8)
    f0, f1 = inputs.cfg1_pair()
    prob = _run(otdyn, g, f0, f1, 300, otdyn.OT_PROX_CLOSED)
    prob.step(299)
    _, rep = prob.solve(1)
    torch.cuda.synchronize()
    st = pdhg.solve(g, f0.astype(np.float64), f1.astype(np.float64), 10.0, 0.099, 300,
                    record_every=300)
    F = prob.F[0].double().cpu().numpy()
    assert rel(F[1:8], st.x[3]) < TOL
    h = st.hist[-1]
    assert abs(rep.cost - h["cost"]) <= TOL * abs(h["cost"])
    prob.close()


@pytest.mark.parametrize("shape", [(9, 1, 1, 5, (G.PERIODIC, G.NEUMANN, G.NEUMANN)),
                                   (33, 31, 3, 6, (G.NEUMANN, G.NEUMANN, G.PERIODIC))],
                         ids=["9x1x1x5", "33x31x3x6"])
def test_closed_prox_certifies_like_newton(otdyn, shape):
    """Solved to the certificate with each root: both certify, and the
    certified costs agree within 1e-5."""
    X, Y, C, P, bc = shape
    _say(f"closed vs Newton to the certificate {shape[:4]}")
    g = G.Grid(X, Y, C, P, bc)
    f0, f1 = inputs.random_pair(31 + X, X, Y, C)
    reps = []
    for kind in (otdyn.OT_PROX_NEWTON, otdyn.OT_PROX_CLOSED):
        prob = _run(otdyn, g, f0, f1, 0, kind)
        st, rep = prob.solve(40000)
        assert st == otdyn.OT_OK, (kind, rep.as_dict())
        reps.append(rep)
        prob.close()
    assert abs(reps[0].cost - reps[1].cost) <= TOL * reps[0].cost
