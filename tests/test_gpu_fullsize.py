"""GPU parity at the benchmarked configurations (the throughput workload
256 x 256 x 3 x 32 and the batched hue workload), in the launch sequence the
benchmarks time: the carried-potential projection past its refined start.

* One steady-state iteration at full size: after 70 iterations (past the 64
  refined ones) the GPU state (x, b, b_bar) is handed to the FP64 oracle,
  both take one more iteration of Algorithm 1, and every element of f, m_x,
  m_y, m_c and b is compared, as is the increment x^{r+1} - x^r.
* A whole trajectory at full size in the steady launch sequence: the refined
  start cut to 4 iterations (desc.carry_refine), 12 iterations compared
  element by element with the oracle's.
* Hue batches with n in {256, 360} bins and T = 32 in the carried-potential
  mode for 300 iterations, every problem compared with its own oracle run,
  with the default launch shapes and with the autotuned ones.

Tolerance: 1e-5 relative (L2) on every field, as for the other parity tests.
"""
import numpy as np
import pytest

from oracle import grid as G
from oracle import pdhg
from synth import inputs
from tests.layout import rel, to_natural

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


def _dual_natural(bt):
    """[1, 4, P, C, Y, X] device dual -> tuple of four (P, C, Y, X) FP64 arrays."""
    a = bt[0].double().cpu().numpy()
    return tuple(a[q] for q in range(4))


def test_full_size_steady_iteration_matches_oracle(otdyn):
    import torch
    X, Y, C, P = 256, 256, 3, 32
    _say(f"full-size steady iteration {X}x{Y}x{C}x{P}")
    g = G.Grid(X, Y, C, P)
    f0, f1 = inputs.cfg3_pair()
    d = otdyn.ot_dyn_default_desc(X, Y, C, P)
    assert d.refine == otdyn.OT_REFINE_CARRY and d.carry_refine == 64
    prob = otdyn.Problem(d, "cuda")
    prob.set_boundary(torch.from_numpy(f0), torch.from_numpy(f1))
    prob.init()
    prob.step(70)
    torch.cuda.synchronize()
    x0 = to_natural(g, *(t[0].double().cpu().numpy() for t in prob.state()))
    b0 = _dual_natural(prob.get_dual())
    bb0 = _dual_natural(prob.get_dual_bar())
    # one more iteration: the steady launch sequence (no refinement solve)
    otdyn.ot_dyn_profile(prob.plan, (1 << otdyn.OT_PHASE_COUNT) - 1)
    prob.step(1)
    phases = otdyn.ot_dyn_profile_read(prob.plan)
    otdyn.ot_dyn_profile(prob.plan, 0)
    assert phases["refine"][1] == 0 and phases["update"][1] == 1, phases
    x1 = to_natural(g, *(t[0].double().cpu().numpy() for t in prob.state()))
    b1 = _dual_natural(prob.get_dual())
    prob.close()
    st = pdhg.State(x=x0, b=b0, bbar=bb0)
    ref = pdhg.step(g, st, f0.astype(np.float64), f1.astype(np.float64), d.tau, d.sigma)
    errs = {n: rel(x1[a], ref.x[a]) for a, n in enumerate(("m_x", "m_y", "m_c", "f"))}
    errs.update({f"b{q}": rel(b1[q], ref.b[q]) for q in range(4)})
    inc = {n: rel(x1[a] - x0[a], ref.x[a] - x0[a]) for a, n in enumerate(("m_x", "m_y", "m_c", "f"))}
    _say(f"fields {errs}\nincrements {inc}")
    for k, v in errs.items():
        assert v < TOL, (k, v)
    for k, v in inc.items():
        assert v < 1e-3, (k, v)


def test_full_size_trajectory_in_the_steady_launch_sequence(otdyn):
    import torch
    X, Y, C, P, iters = 256, 256, 3, 32, 12
    _say(f"full-size trajectory {X}x{Y}x{C}x{P}, {iters} iterations, refined start 4")
    g = G.Grid(X, Y, C, P)
    f0, f1 = inputs.cfg3_pair()
    d = otdyn.ot_dyn_default_desc(X, Y, C, P)
    d.carry_refine = 4
    prob = otdyn.Problem(d, "cuda")
    prob.set_boundary(torch.from_numpy(f0), torch.from_numpy(f1))
    prob.init()
    prob.step(4)
    otdyn.ot_dyn_profile(prob.plan, (1 << otdyn.OT_PHASE_COUNT) - 1)
    prob.step(iters - 4)
    phases = otdyn.ot_dyn_profile_read(prob.plan)
    otdyn.ot_dyn_profile(prob.plan, 0)
    assert phases["refine"][1] == 0 and phases["update"][1] == iters - 4, phases
    gx = to_natural(g, *(t[0].double().cpu().numpy() for t in prob.state()))
    prob.close()
    st = pdhg.solve(g, f0.astype(np.float64), f1.astype(np.float64), d.tau, d.sigma, iters)
    errs = {n: rel(gx[a], st.x[a]) for a, n in enumerate(("m_x", "m_y", "m_c", "f"))}
    _say(f"fields {errs}")
    for k, v in errs.items():
        assert v < TOL, (k, v)


def _hue_batch_problems():
    """n in {256, 360} bins at T = 32 (the sizes that reach the dense one-block
    solve near its LDS limit and the fast one), plus smaller groups."""
    shapes = [(256, 32), (360, 32), (256, 32), (360, 32), (180, 32), (360, 16), (128, 32),
              (64, 16)]
    return [(n, T, inputs.von_mises_hist(7000 + 2 * i, n), inputs.von_mises_hist(7001 + 2 * i, n))
            for i, (n, T) in enumerate(shapes)]


@pytest.mark.parametrize("tuned", [False, True], ids=["default", "autotuned"])
def test_hue_batch_carried_potential_300_iterations(otdyn, tuned):
    probs = _hue_batch_problems()
    _say(f"hue batch carry mode, 300 iterations, autotuned {tuned}")
    base = otdyn.ot_dyn_default_desc(1, 1, 1, 2)
    base.bc[0] = otdyn.OT_BC_PERIODIC
    assert base.refine == otdyn.OT_REFINE_CARRY
    base.tau, base.sigma = 3.0, 0.33          # the hue benchmark's step sizes
    base.adapt = 0                            # the oracle's fixed-step iteration
    dims = [(n, 1, 1, T) for n, T, _, _ in probs]
    bt = otdyn.Batch(base, dims)
    bt.set_boundary([p[2].reshape(1, 1, -1) for p in probs], [p[3].reshape(1, 1, -1) for p in probs])
    if tuned:
        bt.autotune(5)
    iters = 300
    status, rep = bt.solve(iters, chunk=100)
    assert rep.iterations == iters
    for i, (n, T, h0, h1) in enumerate(probs):
        r = bt.problem(i)
        assert r.total_iterations == iters and r.converged == 0
        g = G.Grid(n, 1, 1, T, (G.PERIODIC, G.NEUMANN, G.NEUMANN))
        st = pdhg.solve(g, h0.reshape(1, 1, -1), h1.reshape(1, 1, -1), base.tau, base.sigma,
                        iters, record_every=iters)
        gx = to_natural(g, *bt.state(i))
        ef, em = rel(gx[3], st.x[3]), rel(gx[0], st.x[0])
        _say(f"problem {i} n={n} T={T} tuning {otdyn.ot_dyn_batch_tuning(bt.bt, i)}: "
             f"f {ef:.2e} m {em:.2e}")
        assert ef < TOL and em < TOL, (i, n, T, ef, em)
        assert abs(r.cost - st.hist[-1]["cost"]) <= TOL * st.hist[-1]["cost"]
    bt.close()
