"""FP64 reference of the warm-start network and its gradients (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The network is not
part of the paper; it predicts an initial iterate for Algorithm 1 from the
end densities.  This module defines what the GPU network computes, in plain
NumPy float64, so that the GPU forward pass and gradients can be checked
element by element.

Architecture (channels-last tensors [B, H, W, C]):
  encoder levels l = 0..L-1 with widths w_l = base * 2^l: two 3x3 convs
  (zero padding 1, bias, ReLU) per level, a 2x2 average pool between levels;
  decoder levels l = L-2..0: nearest 2x upsampling, concatenation
  [upsampled, skip_l], two 3x3 convs with ReLU; a 1x1 head (no activation).
Weights of a k x k conv are stored [k, k, C_in, C_out].

Loss: sum over channel groups g of w_g * mean((y - t)^2 over the group).
"""
from __future__ import annotations

import numpy as np


def layer_specs(c_in: int, c_out: int, base: int = 32, levels: int = 4):
    """List of (name, k, C_in, C_out) in execution order."""
    widths = [base * (2 ** l) for l in range(levels)]
    specs = []
    c = c_in
    for l, w in enumerate(widths):
        specs.append((f"e{l}a", 3, c, w))
        specs.append((f"e{l}b", 3, w, w))
        c = w
    for l in range(levels - 2, -1, -1):
        w = widths[l]
        specs.append((f"d{l}a", 3, c + w, w))
        specs.append((f"d{l}b", 3, w, w))
        c = w
    specs.append(("head", 1, c, c_out))
    return specs


def param_count(specs) -> int:
    return sum(k * k * ci * co + co for _, k, ci, co in specs)


def unflatten(specs, flat: np.ndarray):
    """Flat parameter vector -> {name: (W [k, k, ci, co], b [co])}; the flat
    order is, per layer, W (row-major) then b."""
    out, o = {}, 0
    for name, k, ci, co in specs:
        n = k * k * ci * co
        W = flat[o:o + n].reshape(k, k, ci, co)
        o += n
        b = flat[o:o + co]
        o += co
        out[name] = (W, b)
    return out


def he_init(specs, seed: int) -> np.ndarray:
    """He-normal weights and zero biases from a seeded generator."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, k, ci, co in specs:
        std = np.sqrt(2.0 / (k * k * ci))
        parts.append(rng.standard_normal(k * k * ci * co) * std)
        parts.append(np.zeros(co))
    return np.concatenate(parts)


# ---- primitive operations and their adjoints -------------------------------

def conv(x, W, b):
    """k x k convolution (cross-correlation), stride 1, zero padding k // 2."""
    k = W.shape[0]
    p = k // 2
    B, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    out = np.zeros((B, H, Wd, W.shape[3]))
    for ky in range(k):
        for kx in range(k):
            out += xp[:, ky:ky + H, kx:kx + Wd, :] @ W[ky, kx]
    return out + b


def conv_backward(x, W, dy):
    """(dx, dW, db) of conv for upstream gradient dy."""
    k = W.shape[0]
    p = k // 2
    B, H, Wd, ci = x.shape
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(k):
        for kx in range(k):
            patch = xp[:, ky:ky + H, kx:kx + Wd, :]
            dW[ky, kx] = patch.reshape(-1, ci).T @ dy.reshape(-1, dy.shape[3])
            dxp[:, ky:ky + H, kx:kx + Wd, :] += dy @ W[ky, kx].T
    db = dy.sum(axis=(0, 1, 2))
    return dxp[:, p:p + H, p:p + Wd, :], dW, db


def avgpool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_backward(dy):
    B, H, W, C = dy.shape
    return dy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


# ---- network -------------------------------------------------------------

def forward(specs, params: dict, x, levels: int = 4, keep: bool = False):
    """Network output; with keep, also the tape of intermediate tensors."""
    tape = []
    skips = []
    h = x
    i = 0
    for l in range(levels):
        for _ in range(2):
            name = specs[i][0]
            z = conv(h, *params[name])
            tape.append((name, h, z))
            h = np.maximum(z, 0.0)
            i += 1
        if l < levels - 1:
            skips.append(h)
            h = avgpool2(h)
    for l in range(levels - 2, -1, -1):
        h = np.concatenate([upsample2(h), skips[l]], axis=3)
        for _ in range(2):
            name = specs[i][0]
            z = conv(h, *params[name])
            tape.append((name, h, z))
            h = np.maximum(z, 0.0)
            i += 1
    name = specs[i][0]
    y = conv(h, *params[name])
    tape.append((name, h, y))
    return (y, tape) if keep else y


def loss(y, t, groups):
    """groups: list of (c_start, c_end, weight)."""
    L = 0.0
    for c0, c1, w in groups:
        d = y[..., c0:c1] - t[..., c0:c1]
        L += w * float(np.mean(d * d))
    return L


def loss_grad(y, t, groups):
    g = np.zeros_like(y)
    for c0, c1, w in groups:
        d = y[..., c0:c1] - t[..., c0:c1]
        g[..., c0:c1] = 2.0 * w * d / d.size
    return g


def backward(specs, params: dict, x, t, groups, levels: int = 4):
    """(loss, {name: (dW, db)}) by reverse-mode differentiation of forward."""
    y, tape = forward(specs, params, x, levels, keep=True)
    L = loss(y, t, groups)
    grads = {}
    # head
    name, h, _ = tape[-1]
    dh, dW, db = conv_backward(h, params[name][0], loss_grad(y, t, groups))
    grads[name] = (dW, db)
    ti = len(tape) - 2
    widths = [specs[2 * l][3] for l in range(levels)]
    dskips = [None] * (levels - 1)
    for l in range(0, levels - 1):
        for _ in range(2):
            name, hin, z = tape[ti]
            dz = dh * (z > 0)
            dh, dW, db = conv_backward(hin, params[name][0], dz)
            grads[name] = (dW, db)
            ti -= 1
        c_up = dh.shape[3] - widths[l]
        dskips[l] = dh[..., c_up:]
        dh = upsample2_backward(dh[..., :c_up])
    for l in range(levels - 1, -1, -1):
        if l < levels - 1:
            dh = avgpool2_backward(dh) + dskips[l]
        for _ in range(2):
            name, hin, z = tape[ti]
            dz = dh * (z > 0)
            dh, dW, db = conv_backward(hin, params[name][0], dz)
            grads[name] = (dW, db)
            ti -= 1
    return L, grads


def flatten_grads(specs, grads) -> np.ndarray:
    parts = []
    for name, _, _, _ in specs:
        dW, db = grads[name]
        parts.append(dW.ravel())
        parts.append(db.ravel())
    return np.concatenate(parts)
