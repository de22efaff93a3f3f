"""GPU checks of the warm-start network (include/ot_net.h) against the FP64
oracle of oracle/nn.py, and of the solver glue and warm-started batch solve.

BF16 tolerance: the network keeps weights, activations and activation
gradients in BF16 (8 significant bits, unit roundoff 2^-9 = 2e-3) and
accumulates in FP32.  Inputs and weights are rounded to BF16 before both
sides see them, so the remaining differences are the roundings of the
intermediate tensors: about 2e-3 relative per tensor, compounding over the
layers to the per-layer bounds used below.
"""
import numpy as np
import pytest

from oracle import nn
from synth import inputs

pytestmark = pytest.mark.gpu


def _bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _cos(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.fixture(scope="module")
def N():
    import torch
    from paper_1501_04840_amd import otnet
    assert torch.cuda.is_available()
    otnet.lib()
    return otnet


def _setup(N, H, W, cin, cout, base, levels, nb, seed):
    import torch
    d = N.ot_net_default_desc(H, W, cin, cout, nb)
    d.base, d.levels = base, levels
    specs = nn.layer_specs(cin, cout, base, levels)
    flat = nn.he_init(specs, seed)
    rng = np.random.default_rng(seed + 1)
    flat = flat + 0.02 * rng.standard_normal(flat.size)
    # weights to BF16 (the device rounds them so), biases stay FP32
    params = nn.unflatten(specs, flat)
    flat_r = np.concatenate([np.concatenate([_bf16(W).ravel(), np.float32(b).astype(np.float64)])
                             for W, b in (params[s[0]] for s in specs)])
    x = _bf16(rng.uniform(0.0, 2.0, size=(nb, H, W, cin)))
    t = rng.standard_normal((nb, H, W, cout))
    net = N.Net(d, "cuda:0")
    net.set_params(torch.from_numpy(flat_r.astype(np.float32)))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to("cuda:0")
    return d, specs, flat_r, x, t, net, dev


CASES = [
    # H, W, in, out, base, levels, batch
    (8, 8, 6, 21, 8, 1, 2),
    (16, 16, 6, 21, 8, 3, 2),
    (16, 24, 5, 13, 16, 4, 3),
]


@pytest.mark.parametrize("case", CASES)
def test_forward_matches_oracle(N, case):
    H, W, cin, cout, base, levels, nb = case
    d, specs, flat, x, t, net, dev = _setup(N, H, W, cin, cout, base, levels, nb, 11)
    y = net.forward(dev(x)).cpu().numpy()
    ref = nn.forward(specs, nn.unflatten(specs, flat), x, levels)
    assert y.shape == ref.shape
    assert _rel(y, ref) < 2e-2, _rel(y, ref)
    net.close()


@pytest.mark.parametrize("case", CASES)
def test_gradient_matches_oracle(N, case):
    H, W, cin, cout, base, levels, nb = case
    d, specs, flat, x, t, net, dev = _setup(N, H, W, cin, cout, base, levels, nb, 12)
    rng = np.random.default_rng(3)
    cw = rng.uniform(0.5, 2.0, cout) / cout
    groups = [(c, c + 1, cw[c] ) for c in range(cout)]
    loss, g = net.grad(dev(x), dev(t), dev(cw))
    L_ref, grads = nn.backward(specs, nn.unflatten(specs, flat), x, t, groups, levels)
    assert abs(loss - L_ref) <= 2e-2 * abs(L_ref), (loss, L_ref)
    g = g.cpu().numpy().astype(np.float64)
    gref = nn.flatten_grads(specs, grads)
    assert _cos(g, gref) > 0.999
    o = 0
    for name, k, ci, co in specs:
        n = k * k * ci * co + co
        gw, rw = g[o:o + n - co], gref[o:o + n - co]
        gb, rb = g[o + n - co:o + n], gref[o + n - co:o + n]
        # deep levels of the small cases see few pixels, where a ReLU that
        # flips under rounding moves the sum most
        assert _rel(gw, rw) < 0.12 and _cos(gw, rw) > 0.995, (name, "W", _rel(gw, rw))
        assert _rel(gb, rb) < 0.12 and _cos(gb, rb) > 0.995, (name, "b", _rel(gb, rb))
        o += n
    net.close()


def test_full_size_network_forward_and_gradient(N):
    # the warm-start network itself: 64 x 64, 6 -> 189 channels, 4 levels
    d, specs, flat, x, t, net, dev = _setup(N, 64, 64, 6, 189, 32, 4, 1, 13)
    y = net.forward(dev(x)).cpu().numpy()
    ref = nn.forward(specs, nn.unflatten(specs, flat), x, 4)
    assert _rel(y, ref) < 3e-2, _rel(y, ref)
    cw = np.full(189, 1.0 / 189)
    loss, g = net.grad(dev(x), dev(t), dev(cw))
    L_ref, grads = nn.backward(specs, nn.unflatten(specs, flat), x, t, [(0, 189, 1.0)], 4)
    assert abs(loss - L_ref) <= 2e-2 * L_ref
    assert _cos(g.cpu().numpy(), nn.flatten_grads(specs, grads)) > 0.998
    net.close()


def test_adam_step_and_param_roundtrip(N):
    import torch
    d, specs, flat, x, t, net, dev = _setup(N, 16, 16, 6, 21, 8, 3, 2, 14)
    np.testing.assert_array_equal(net.get_params().cpu().numpy(), flat.astype(np.float32))
    cw = dev(np.full(21, 1.0 / 21))
    _, g = net.grad(dev(x), dev(t), cw)
    g = g.cpu().numpy().astype(np.float64)
    lr = 1e-3
    net.train_step(dev(x), dev(t), cw, lr)
    p1 = net.get_params().cpu().numpy().astype(np.float64)
    # first Adam step: m_hat = g, v_hat = g^2, so p - lr * g / (|g| + eps)
    want = flat - lr * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(p1 - want)) < 1e-6
    net.close()


def test_training_reduces_loss(N):
    d, specs, flat, x, t, net, dev = _setup(N, 16, 16, 6, 21, 8, 3, 4, 15)
    # a smooth target the network can fit: channels are blends of the inputs
    rng = np.random.default_rng(5)
    mix = rng.standard_normal((6, 21)) / 6
    t = x @ mix
    cw = dev(np.full(21, 1.0 / 21))
    X, T = dev(x), dev(t)
    first = net.train_step(X, T, cw, 3e-3)
    for _ in range(150):
        last = net.train_step(X, T, cw, 3e-3)
    assert last < 0.1 * first, (first, last)
    net.close()


# ---- solver glue -----------------------------------------------------------

def _warm_targets_ref(F, Mx, My, Mc, f0, f1, P):
    """The target layout written out from its definition in ot_net.h."""
    C, Y, X = f0.shape
    chans = []
    for k in range(1, P):
        s = k / P
        for c in range(C):
            chans.append(F[k, c] - ((1 - s) * f0[c] + s * f1[c]))
    for M in (Mx, My, Mc):
        for k in range(P):
            for c in range(C):
                chans.append(M[k, c])
    return np.stack(chans, axis=-1)


def test_warm_targets_and_state_roundtrip(N):
    import torch
    from paper_1501_04840_amd import otdyn
    X, Y, C, P, nb = 24, 16, 3, 4, 2
    d = otdyn.ot_dyn_default_desc(X, Y, C, P)
    rng = np.random.default_rng(9)
    f0 = rng.uniform(0.1, 1, (nb, C, Y, X)).astype(np.float32)
    f1 = rng.uniform(0.1, 1, (nb, C, Y, X)).astype(np.float32)
    F = rng.standard_normal((nb, P + 1, C, Y, X)).astype(np.float32)
    Ms = [rng.standard_normal((nb, P, C, Y, X)).astype(np.float32) for _ in range(3)]
    Ms[0][..., 0] = 0          # Neumann walls (x slot 0, y slot 0); colour is periodic
    Ms[1][..., 0, :] = 0
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    dF, dM = dev(F), [dev(m) for m in Ms]
    nch = N.warm_channels(C, P)
    t = torch.empty((nb, Y, X, nch), dtype=torch.float32, device="cuda:0")
    sl = X * Y * C
    st = torch.cuda.current_stream().cuda_stream
    N.ot_warm_targets(d, nb, dev(f0), dev(f1), dF, (P + 1) * sl, *dM, P * sl, None, t, st)
    got = t.cpu().numpy()
    for b in range(nb):
        ref = _warm_targets_ref(F[b].astype(np.float64), *(m[b] for m in Ms), f0[b], f1[b], P)
        np.testing.assert_allclose(got[b], ref, rtol=1e-6, atol=1e-6)
    x = torch.empty((nb, Y, X, 2 * C), dtype=torch.float32, device="cuda:0")
    N.ot_warm_inputs(d, nb, dev(f0), dev(f1), None, x, st)
    np.testing.assert_array_equal(x.cpu().numpy(),
                                  np.concatenate([f0, f1], axis=1).transpose(0, 2, 3, 1))
    # with a base: targets subtract it, inputs append it, states add it back
    base = dev(rng.standard_normal((nb, Y, X, nch)).astype(np.float32))
    tb = torch.empty_like(t)
    N.ot_warm_targets(d, nb, dev(f0), dev(f1), dF, (P + 1) * sl, *dM, P * sl, base, tb, st)
    want = got - base.cpu().numpy()
    o0 = C * (P - 1)                      # wall slots read as 0 whatever the base
    want[:, :, 0, o0:o0 + P * C] = 0
    want[:, 0, :, o0 + P * C:o0 + 2 * P * C] = 0
    np.testing.assert_allclose(tb.cpu().numpy(), want, rtol=1e-5, atol=1e-5)
    xb = torch.empty((nb, Y, X, 2 * C + nch), dtype=torch.float32, device="cuda:0")
    N.ot_warm_inputs(d, nb, dev(f0), dev(f1), base, xb, st)
    np.testing.assert_array_equal(xb.cpu().numpy()[..., 2 * C:], base.cpu().numpy())
    # state from the targets gives back the unknowns of F and all of M
    F2 = torch.zeros_like(dF)
    M2 = [torch.zeros_like(m) for m in dM]
    N.ot_warm_state(d, nb, dev(f0), dev(f1), t, None, F2, (P + 1) * sl, *M2, P * sl, st)
    np.testing.assert_allclose(F2.cpu().numpy()[:, 1:P], F[:, 1:P], rtol=1e-6, atol=1e-6)
    for a, b in zip(M2, Ms):
        np.testing.assert_array_equal(a.cpu().numpy(), b)
    F3 = torch.zeros_like(dF)
    M3 = [torch.zeros_like(m) for m in dM]
    N.ot_warm_state(d, nb, dev(f0), dev(f1), tb, base, F3, (P + 1) * sl, *M3, P * sl, st)
    np.testing.assert_allclose(F3.cpu().numpy()[:, 1:P], F[:, 1:P], rtol=1e-5, atol=1e-5)
    for a, b in zip(M3, Ms):
        np.testing.assert_allclose(a.cpu().numpy(), b, rtol=1e-5, atol=1e-5)


def _lerp(u, n):
    i0 = int(np.floor(u))
    w = u - i0
    return min(max(i0, 0), n - 1), min(max(i0 + 1, 0), n - 1), w


def _prolong_ref(Fc, Mxc, Myc, Mcc, X, Y, P):
    """The prolongation written out from its definition in ot_net.h
    (Neumann x and y), one fine entry at a time."""
    Pc1, C, Yc, Xc = Fc.shape
    Pc = Pc1 - 1
    F = np.zeros((P + 1, C, Y, X))
    Ms = [np.zeros((P, C, Y, X)) for _ in range(3)]

    def cen(A, x, y):
        xa, xb, wx = _lerp(0.5 * x - 0.25, Xc)
        ya, yb, wy = _lerp(0.5 * y - 0.25, Yc)
        return ((1 - wy) * ((1 - wx) * A[ya, xa] + wx * A[ya, xb])
                + wy * ((1 - wx) * A[yb, xa] + wx * A[yb, xb]))

    def xface(A, x, y):
        fa = lambda row, j: 0.0 if j <= 0 or j >= Xc else row[j]
        ya, yb, wy = _lerp(0.5 * y - 0.25, Yc)
        j, w = x // 2, 0.5 * (x % 2)
        v = [(1 - w) * fa(A[yy], j) + w * fa(A[yy], j + 1) for yy in (ya, yb)]
        return (1 - wy) * v[0] + wy * v[1]

    def yface(A, x, y):
        fa = lambda col, j: 0.0 if j <= 0 or j >= Yc else col[j]
        xa, xb, wx = _lerp(0.5 * x - 0.25, Xc)
        j, w = y // 2, 0.5 * (y % 2)
        v = [(1 - w) * fa(A[:, xx], j) + w * fa(A[:, xx], j + 1) for xx in (xa, xb)]
        return (1 - wx) * v[0] + wx * v[1]

    for k in range(1, P):
        s = k * Pc / P
        j0 = min(int(np.floor(s)), Pc - 1)
        a = s - j0
        for c in range(C):
            for y in range(Y):
                for x in range(X):
                    F[k, c, y, x] = (1 - a) * cen(Fc[j0, c], x, y) + a * cen(Fc[j0 + 1, c], x, y)
    for k in range(P):
        ka, kb, wt = _lerp((k + 0.5) * Pc / P - 0.5, Pc)
        for c in range(C):
            for y in range(Y):
                for x in range(X):
                    vals = [0.0, 0.0, 0.0]
                    for kk, ww in ((ka, 1 - wt), (kb, wt)):
                        vals[0] += ww * xface(Mxc[kk, c], x, y)
                        vals[1] += ww * yface(Myc[kk, c], x, y)
                        vals[2] += ww * cen(Mcc[kk, c], x, y)
                    Ms[0][k, c, y, x] = 0.0 if x == 0 else vals[0]
                    Ms[1][k, c, y, x] = 0.0 if y == 0 else vals[1]
                    Ms[2][k, c, y, x] = vals[2]
    return F, Ms


def test_restrict_and_prolong_match_their_definitions(N):
    import torch
    from paper_1501_04840_amd import otdyn
    X, Y, C, P, Pc, nb = 12, 8, 3, 6, 4, 2
    df = otdyn.ot_dyn_default_desc(X, Y, C, P)
    dc = otdyn.ot_dyn_default_desc(X // 2, Y // 2, C, Pc)
    rng = np.random.default_rng(10)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    f = rng.uniform(0, 1, (nb, C, Y, X))
    fc = torch.empty((nb, C, Y // 2, X // 2), dtype=torch.float32, device="cuda:0")
    N.ot_warm_restrict(df, nb, dev(f), fc, st)
    ref = f.reshape(nb, C, Y // 2, 2, X // 2, 2).mean(axis=(3, 5))
    np.testing.assert_allclose(fc.cpu().numpy(), ref, rtol=1e-6)
    Fc = rng.standard_normal((nb, Pc + 1, C, Y // 2, X // 2))
    Mc = [rng.standard_normal((nb, Pc, C, Y // 2, X // 2)) for _ in range(3)]
    Mc[0][..., 0] = 0
    Mc[1][..., 0, :] = 0
    slc, slf = (X // 2) * (Y // 2) * C, X * Y * C
    F = torch.zeros((nb, P + 1, C, Y, X), dtype=torch.float32, device="cuda:0")
    Mf = [torch.zeros((nb, P, C, Y, X), dtype=torch.float32, device="cuda:0") for _ in range(3)]
    N.ot_warm_prolong(dc, df, nb, dev(Fc), (Pc + 1) * slc, *(dev(m) for m in Mc), Pc * slc,
                      F, (P + 1) * slf, *Mf, P * slf, st)
    for b in range(nb):
        Fr, Mr = _prolong_ref(Fc[b], *(m[b] for m in Mc), X, Y, P)
        np.testing.assert_allclose(F.cpu().numpy()[b, 1:P], Fr[1:P], rtol=1e-5, atol=1e-5)
        for q in range(3):
            np.testing.assert_allclose(Mf[q].cpu().numpy()[b], Mr[q], rtol=1e-5, atol=1e-5)
    # shapes that do not pair up are rejected
    bad = otdyn.ot_dyn_default_desc(X // 2 + 1, Y // 2, C, Pc)
    with pytest.raises(otdyn.OtDynError):
        N.ot_warm_prolong(bad, df, nb, dev(Fc), (Pc + 1) * slc, *(dev(m) for m in Mc), Pc * slc,
                          F, (P + 1) * slf, *Mf, P * slf, st)


def test_warm_started_batch_certifies_at_once_from_a_solution(N):
    """A batch restarted from its own certified solution (with the dual of
    the prox fixed point) certifies within a few residual checks, while a
    cold start needs far more iterations; the solutions agree."""
    import torch
    from paper_1501_04840_amd import otdyn
    X = Y = 32
    C, P = 3, 8
    pairs = [inputs.random_pair(700 + i, X, Y, C) for i in range(3)]
    d = otdyn.ot_dyn_default_desc(X, Y, C, P)
    d.tau, d.sigma = 3.0, 0.33
    d.tol_res, d.tol_div = 1e-5, 1e-6
    d.adapt = 0                  # compare like with like: fixed step sizes
    bt = otdyn.Batch(d, [(X, Y, C, P)] * 3, "cuda:0")
    bt.set_boundary([p[0] for p in pairs], [p[1] for p in pairs])
    st, rep = bt.solve(20000, 50)
    assert st == otdyn.OT_OK, rep.as_dict()
    cold_its = [bt.problem(i).iterations for i in range(3)]
    F, M = bt.packed_state()
    bt.set_state(F, M, otdyn.OT_INIT_PRIMAL_DUAL)
    st, rep = bt.solve(20000, 50)
    assert st == otdyn.OT_OK
    warm_its = [bt.problem(i).iterations for i in range(3)]
    assert max(warm_its) <= 500 and min(cold_its) >= 4 * max(warm_its), (cold_its, warm_its)
    F2, M2 = bt.packed_state()
    # both certified at tol_res 1e-5: the same solution to a few 1e-4
    assert torch.linalg.norm(F2 - F) / torch.linalg.norm(F) < 5e-3
    # a wrong mode is rejected
    with pytest.raises(otdyn.OtDynError):
        bt.set_state(F, M, otdyn.OT_INIT_COLD)
    bt.close()


def test_trained_network_gains_over_the_coarse_start(N):
    """The committed trained network (paper_1501_04840_amd/weights) on
    held-out 64 x 64 x 3 x 16 pairs: its correction brings the prolonged
    coarse solution closer to the certified solution, and the warm-started
    solves certify.  Prints the iterations to the certified tolerance from
    the cold, coarse and network starts, and checks the network's start
    saves iterations over the cold one: fewer in total, and for no pair more
    than two residual checks (200 iterations) beyond cold, room for
    rounding-order changes of the kernels (the training record's 64 held-out
    pairs: none above cold, -2.4% on average).  The gain is small: the
    iteration removes smooth relative errors quickly and sharp-feature errors
    slowly, and the network's error is of the second kind; it does not cover
    the coarse solve and the inference in wall time."""
    import json
    import torch
    from paper_1501_04840_amd import otnet
    from paper_1501_04840_amd import warmstart as W
    net = otnet.Net(W.net_desc(8), "cuda:0")
    net.set_params(torch.from_numpy(W.load_weights()))
    pairs = W.pairs_of(range(8), held_out=True)
    res = W.evaluate(pairs, ("cold", "coarse", "warm"), net, max_iters=30000, group=8,
                     net_batch=8)
    net.close()
    err = res["prediction_rel_error"]
    print(json.dumps({m: {k: v for k, v in r.items() if k != "iterations"}
                      for m, r in res.items() if isinstance(r, dict) and "wall_s" in r}))
    print(json.dumps(err))
    for g in ("f", "mx", "my"):
        assert err["warm_" + g] < 0.9 * err["coarse_" + g], (g, err)
    assert res["warm"]["certified"] == len(pairs)
    assert res["cold"]["certified"] == len(pairs)
    cold, warm = res["cold"]["iterations"], res["warm"]["iterations"]
    assert sum(warm) < sum(cold), (cold, warm)
    assert all(w <= c + 200 for c, w in zip(cold, warm)), (cold, warm)
