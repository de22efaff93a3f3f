"""GPU tests of the state-level entry points: residuals of the current state
without iterating, the extrapolated dual, the non-finite residual error and
the cold fallback of warm starts (single plans and batches)."""
import numpy as np
import pytest

from oracle import grid as G
from oracle import pdhg
from synth import inputs
from tests.layout import rel, to_natural, to_padded

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def otdyn():
    import torch
    from paper_1501_04840_amd import otdyn as o
    assert torch.cuda.is_available()
    o.lib()
    return o


def _say(msg):
    print(msg, flush=True)


def _cfg1_plan(o, **fields):
    import torch
    f0, f1 = inputs.cfg1_pair()
    d = o.ot_dyn_default_desc(16, 16, 3, 8)
    for k, v in fields.items():
        setattr(d, k, v)
    prob = o.Problem(d, "cuda")
    prob.set_boundary(torch.from_numpy(f0), torch.from_numpy(f1))
    return prob, f0, f1


def _snapshot(prob):
    return [t.clone() for t in prob.state()] + [prob.get_dual(), prob.get_dual_bar()]


def test_residuals_leave_the_state_unchanged_and_match_the_oracle(otdyn):
    """ot_dyn_residuals reduces the current state without iterating: every
    buffer bitwise unchanged, the trajectory after it the same as without
    it; r_prim and the cost of z = prox(K x + c + b) and r_div / e_mass as
    the FP64 oracle computes them on the same state."""
    import torch
    _say("residuals of the current state")
    g = G.Grid(16, 16, 3, 8)
    prob, f0, f1 = _cfg1_plan(otdyn)
    prob.init()
    _, rep0 = prob.residuals()
    assert rep0.r_dual == -1.0 and rep0.iterations == 0   # no check since init
    prob.step(40)
    torch.cuda.synchronize()
    before = _snapshot(prob)
    st, rep = prob.residuals()
    torch.cuda.synchronize()
    after = _snapshot(prob)
    for u, v in zip(before, after):
        assert torch.equal(u, v)
    assert rep.r_dual == -1.0
    x = to_natural(g, *(t[0].double().cpu().numpy() for t in prob.state()))
    b = prob.get_dual()[0].double().cpu().numpy()
    ref = pdhg.state_residuals(g, x, tuple(b[q] for q in range(4)), f0, f1, prob.desc.sigma)
    _say(f"gpu {rep.as_dict()}\noracle {ref}")
    assert abs(rep.cost - ref["cost"]) <= 1e-5 * ref["cost"]
    assert abs(rep.r_prim - ref["r_prim"]) <= 1e-3 * ref["r_prim"]
    assert abs(rep.r_div - ref["r_div"]) <= 1e-7 + 0.05 * ref["r_div"]
    assert rep.e_mass < 1e-6
    # the same trajectory as a plan that never asked for residuals
    prob.step(10)
    torch.cuda.synchronize()
    other, _, _ = _cfg1_plan(otdyn)
    other.init()
    other.step(50)
    torch.cuda.synchronize()
    for u, v in zip(_snapshot(prob), _snapshot(other)):
        assert torch.equal(u, v)
    # after a residual check r_dual is that check's
    _, srep = prob.solve(50)
    _, rrep = prob.residuals()
    assert rrep.r_dual == srep.r_dual
    prob.close()
    other.close()


def test_dual_bar_is_the_extrapolated_dual(otdyn):
    """b_bar = b + theta (b - b_old) (Step 4 with theta = 1)."""
    import torch
    _say("extrapolated dual")
    prob, _, _ = _cfg1_plan(otdyn)
    prob.init()
    prob.step(20)
    b_old = prob.get_dual()
    prob.step(1)
    b, bb = prob.get_dual(), prob.get_dual_bar()
    torch.cuda.synchronize()
    np.testing.assert_allclose(bb.cpu().numpy(), (2 * b - b_old).cpu().numpy(), rtol=0,
                               atol=1e-6 * float(b.abs().max()))
    prob.close()


def test_non_finite_dual_is_reported(otdyn):
    """A non-finite dual (set through ot_dyn_set_dual) makes the next residual
    check non-finite: ot_dyn_solve returns OT_ERR_NONFINITE.  NaN arithmetic,
    no device fault."""
    import torch
    _say("non-finite residual")
    prob, _, _ = _cfg1_plan(otdyn)
    prob.init()
    prob.step(10)
    b = prob.get_dual()
    b[0, 3, 2, 1, 5, 7] = float("nan")
    prob.set_dual(b)
    with pytest.raises(otdyn.OtDynError) as e:
        prob.solve(100)
    assert e.value.status == otdyn.OT_ERR_NONFINITE
    prob.close()


def test_warm_start_falls_back_to_cold(otdyn):
    """OT_INIT_FALLBACK: a warm start whose residual turns non-finite, and one
    that is not certified within max_iters, restart from Algorithm 1's cold
    start inside ot_dyn_solve; the report says so and counts both runs, and
    the final state is bitwise that of a plain cold solve of the same
    budget."""
    import torch
    _say("cold fallback, single plan")
    cold, _, _ = _cfg1_plan(otdyn, check_every=100)
    cold.init()
    st, crep = cold.solve(20000)
    assert st == otdyn.OT_OK and crep.fallback == 0
    n_cold = crep.iterations
    cold_end = _snapshot(cold)
    # (a) a NaN in the warm primal: non-finite at the first check
    warm, _, _ = _cfg1_plan(otdyn, check_every=100)
    warm.F[0, 3, 1, 2, 2] = float("nan")
    warm.init(otdyn.OT_INIT_PRIMAL | otdyn.OT_INIT_FALLBACK)
    st, rep = warm.solve(20000)
    assert st == otdyn.OT_OK and rep.fallback == 1 and rep.converged == 1
    assert rep.iterations == 100 + n_cold
    for u, v in zip(_snapshot(warm), cold_end):
        assert torch.equal(u, v)
    # (b) a finite warm start far from the solution, 200 iterations budget:
    # not certified, restarted cold, the cold run not certified either
    cold.init()
    cold.step(200)
    cold_200 = _snapshot(cold)
    warm.F.zero_()
    warm.Mx.fill_(5.0)
    warm.init(otdyn.OT_INIT_PRIMAL | otdyn.OT_INIT_FALLBACK)
    st, rep = warm.solve(200)
    assert st == otdyn.OT_NOT_CONVERGED and rep.fallback == 1, rep.as_dict()
    assert rep.iterations == 400
    for u, v in zip(_snapshot(warm), cold_200):
        assert torch.equal(u, v)
    # without the flag a non-certified warm start just reports it
    warm.F.zero_()
    warm.Mx.fill_(5.0)
    warm.init(otdyn.OT_INIT_PRIMAL)
    st, rep = warm.solve(200)
    assert st == otdyn.OT_NOT_CONVERGED and rep.fallback == 0 and rep.iterations == 200
    with pytest.raises(otdyn.OtDynError):
        warm.init(otdyn.OT_INIT_COLD | otdyn.OT_INIT_FALLBACK)
    warm.close()
    cold.close()


def test_batch_warm_start_falls_back_per_problem(otdyn):
    """In a batch only the warm starts that fail restart cold: problem 1
    (non-finite at the first check) and problem 2 (not certified within
    max_iters) restart, each with a budget of another max_iters and ends
    bitwise where a plain cold batch of that budget ends; problems 0 and 3
    start from their certified solutions and duals and certify at the first
    check.  Each restarted problem is alone in its shape group (a restart
    also refines the start of the other members of its group)."""
    import torch
    _say("cold fallback, batch")
    shapes = [(16, 16, 3, 8), (16, 16, 3, 8), (24, 20, 3, 8), (20, 12, 3, 8)]
    pairs = [inputs.cfg2_pair(300 + 2 * i, 301 + 2 * i, X, Y) for i, (X, Y, C, P) in enumerate(shapes)]
    base = otdyn.ot_dyn_default_desc(1, 1, 3, 2)
    base.check_every = 100

    def batch():
        b = otdyn.Batch(base, shapes)
        b.set_boundary([p[0] for p in pairs], [p[1] for p in pairs])
        return b

    full = batch()
    st, frep = full.solve(30000, chunk=100)
    assert st == otdyn.OT_OK and frep.converged == 4
    Fs, Ms = full.packed_state()
    Ds = full.packed_dual()
    short = batch()
    short.solve(200, chunk=100)
    F, M, D = Fs.clone(), Ms.clone(), Ds.clone()
    sl = 16 * 16 * 3
    F[full.off_F[1] + 3 * sl + 5] = float("nan")
    F[full.off_F[2]:full.off_F[3]] = 0.0
    M[full.off_M[2]:full.off_M[3]] = 5.0
    D[full.off_M[1] // 3 * 4:full.off_M[3] // 3 * 4] = 0.0
    warm = batch()
    warm.set_state(F, M, otdyn.OT_INIT_PRIMAL | otdyn.OT_INIT_FALLBACK)
    warm.set_dual(D)
    st, rep = warm.solve(200, chunk=100)
    r = [warm.problem(i) for i in range(4)]
    _say(f"warm {[(x.iterations, x.fallback, x.converged) for x in r]}")
    assert st == otdyn.OT_NOT_CONVERGED and rep.converged == 2 and rep.fallback == 2
    assert [x.fallback for x in r] == [0, 1, 1, 0]
    assert [x.converged for x in r] == [1, 0, 0, 1]
    assert [x.iterations for x in r] == [100, 300, 400, 100]
    for i in (1, 2):
        for u, v in zip(warm.state(i), short.state(i)):
            np.testing.assert_array_equal(u, v)
    for b in (warm, short, full):
        b.close()
