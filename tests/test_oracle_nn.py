"""Pins of the FP64 warm-start network oracle (oracle/nn.py).

The gradients are pinned by central finite differences of the loss, the
convolution by scipy's N-d correlation, pooling and upsampling by their
adjoint identities, and the architecture by its parameter count.
"""
import numpy as np
import pytest
from scipy import signal

from oracle import nn


def _small_net(seed=0, c_in=6, c_out=5, base=4, levels=3):
    specs = nn.layer_specs(c_in, c_out, base, levels)
    flat = nn.he_init(specs, seed)
    rng = np.random.default_rng(seed + 1)
    flat = flat + 0.05 * rng.standard_normal(flat.size)   # non-zero biases too
    return specs, flat


def test_param_count_of_the_full_network():
    # 6 -> 189 channels with widths 32, 64, 128, 256: the layer list written out
    specs = nn.layer_specs(6, 189, 32, 4)
    names = [s[0] for s in specs]
    assert names == ["e0a", "e0b", "e1a", "e1b", "e2a", "e2b", "e3a", "e3b",
                     "d2a", "d2b", "d1a", "d1b", "d0a", "d0b", "head"]
    want = (9 * 6 * 32 + 32 + 9 * 32 * 32 + 32 + 9 * 32 * 64 + 64 + 9 * 64 * 64 + 64
            + 9 * 64 * 128 + 128 + 9 * 128 * 128 + 128 + 9 * 128 * 256 + 256
            + 9 * 256 * 256 + 256 + 9 * 384 * 128 + 128 + 9 * 128 * 128 + 128
            + 9 * 192 * 64 + 64 + 9 * 64 * 64 + 64 + 9 * 96 * 32 + 32 + 9 * 32 * 32 + 32
            + 32 * 189 + 189)
    assert nn.param_count(specs) == want


@pytest.mark.parametrize("k", [1, 3])
def test_conv_matches_scipy_correlate(k):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 7, 5, 4))
    W = rng.standard_normal((k, k, 4, 3))
    b = rng.standard_normal(3)
    y = nn.conv(x, W, b)
    for bi in range(2):
        for co in range(3):
            ref = b[co] + sum(signal.correlate(x[bi, :, :, ci], W[:, :, ci, co], mode="same")
                              for ci in range(4))
            np.testing.assert_allclose(y[bi, :, :, co], ref, rtol=1e-12, atol=1e-12)


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 8, 6, 3))
    y = rng.standard_normal((2, 4, 3, 3))
    assert np.isclose(np.sum(nn.avgpool2(x) * y), np.sum(x * nn.avgpool2_backward(y)))
    assert np.isclose(np.sum(nn.upsample2(y) * x), np.sum(y * nn.upsample2_backward(x)))
    # pooling a constant keeps it; upsampling then pooling is the identity
    np.testing.assert_allclose(nn.avgpool2(np.full((1, 4, 4, 2), 3.0)), 3.0)
    np.testing.assert_allclose(nn.avgpool2(nn.upsample2(y)), y, rtol=1e-15)


def test_conv_backward_adjoint():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 6, 6, 3))
    W = rng.standard_normal((3, 3, 3, 4))
    dy = rng.standard_normal((2, 6, 6, 4))
    dx, dW, db = nn.conv_backward(x, W, dy)
    # <conv(x) - b, dy> is linear in x and in W
    lin = np.sum((nn.conv(x, W, np.zeros(4))) * dy)
    assert np.isclose(np.sum(dx * x), lin)
    assert np.isclose(np.sum(dW * W), lin)
    np.testing.assert_allclose(db, dy.sum(axis=(0, 1, 2)))


def test_network_gradient_by_finite_differences():
    specs, flat = _small_net()
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, 8, 8, 6))
    t = rng.standard_normal((2, 8, 8, 5))
    groups = [(0, 2, 1.0), (2, 5, 0.5)]

    def L(v):
        return nn.loss(nn.forward(specs, nn.unflatten(specs, v), x, 3), t, groups)

    L0, grads = nn.backward(specs, nn.unflatten(specs, flat), x, t, groups, 3)
    assert np.isclose(L0, L(flat))
    g = nn.flatten_grads(specs, grads)
    idx = rng.choice(flat.size, 60, replace=False)
    # every layer's bias and a weight of every layer are among the probes
    o = 0
    for _, k, ci, co in specs:
        idx = np.append(idx, [o, o + k * k * ci * co])
        o += k * k * ci * co + co
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        fd = (L(flat + e) - L(flat - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_loss_gradient_by_finite_differences():
    rng = np.random.default_rng(8)
    y = rng.standard_normal((1, 3, 3, 4))
    t = rng.standard_normal((1, 3, 3, 4))
    groups = [(0, 1, 2.0), (1, 4, 0.25)]
    g = nn.loss_grad(y, t, groups)
    h = 1e-6
    for i in range(y.size):
        e = np.zeros(y.size)
        e[i] = h
        e = e.reshape(y.shape)
        fd = (nn.loss(y + e, t, groups) - nn.loss(y - e, t, groups)) / (2 * h)
        assert abs(fd - g.ravel()[i]) < 1e-8
