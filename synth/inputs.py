"""Seeded synthetic densities shaped like the paper's workloads.

This module only draws and normalises input densities; it holds none of the
transport method's arithmetic. Both the CPU oracle and the GPU path receive
the same FP32-rounded arrays produced here (upcast to FP64 for the oracle).

The paper's own images (RGB pairs of Sec. 4, flower hue histograms of Sec. 5)
are not available, so every workload is a synthetic stand-in with the paper's
shapes: RGB densities of X x Y x 3 with a periodic colour axis, and 1D periodic
hue histograms.

Array layout: an RGB density is returned as float32 of shape (C, Y, X), x
fastest; a hue histogram as float32 of shape (n,).
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

__all__ = [
    "normalise_mean_one",
    "aniso_gaussians",
    "rgb_bumps",
    "smooth_random_field",
    "von_mises_hist",
    "cfg1_pair",
    "cfg2_pair",
    "cfg3_pair",
    "cfg4_problems",
    "cfg5_pair",
    "hue_image",
    "random_pair",
]


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.default_rng(seed)
    return np.random.default_rng(np.random.SeedSequence(int(seed)))


def normalise_mean_one(g: np.ndarray) -> np.ndarray:
    """Scale a non-negative FP64 array to mean 1 per cell, then round to FP32."""
    g = np.asarray(g, dtype=np.float64)
    return (g / g.mean()).astype(np.float32)


def aniso_gaussians(seed, X: int, Y: int, C: int = 3, n_bumps: int = 3,
                    floor: float = 1e-3) -> np.ndarray:
    """Per channel, a sum of anisotropic Gaussians plus a floor.

    Centre U[2, X-2] x U[2, Y-2] px, axis widths U[1, 4] px, angle U[0, pi),
    amplitude U[0.5, 1.5]; the sum is scaled to peak 1 before the floor is
    added, then the whole density is normalised to mean 1.
    """
    rng = _rng(seed)
    xs = np.arange(X) + 0.5
    ys = np.arange(Y) + 0.5
    gx, gy = np.meshgrid(xs, ys)                       # (Y, X)
    out = np.zeros((C, Y, X))
    for c in range(C):
        for _ in range(n_bumps):
            cx = rng.uniform(2.0, X - 2.0)
            cy = rng.uniform(2.0, Y - 2.0)
            s1, s2 = rng.uniform(1.0, 4.0, size=2)
            ang = rng.uniform(0.0, np.pi)
            amp = rng.uniform(0.5, 1.5)
            dx, dy = gx - cx, gy - cy
            ca, sa = np.cos(ang), np.sin(ang)
            r1 = ca * dx + sa * dy
            r2 = -sa * dx + ca * dy
            out[c] += amp * np.exp(-0.5 * ((r1 / s1) ** 2 + (r2 / s2) ** 2))
    out /= out.max()
    out += floor
    return normalise_mean_one(out)


def rgb_bumps(seed, X: int, Y: int, C: int = 3, n_bumps: int = 8,
              floor: float = 1e-4) -> np.ndarray:
    """Isotropic bumps with an RGB weight each, so mass has to change channel.

    sigma U[2, 10] px, centre U[0, X) x U[0, Y), amplitude U[0.5, 1.5],
    channel weights U[0, 1]^C per bump; peak scaled to 1, floor added,
    normalised to mean 1.
    """
    rng = _rng(seed)
    xs = np.arange(X) + 0.5
    ys = np.arange(Y) + 0.5
    gx, gy = np.meshgrid(xs, ys)
    out = np.zeros((C, Y, X))
    for _ in range(n_bumps):
        s = rng.uniform(2.0, 10.0)
        cx = rng.uniform(0.0, X)
        cy = rng.uniform(0.0, Y)
        amp = rng.uniform(0.5, 1.5)
        w = rng.uniform(0.0, 1.0, size=C)
        bump = amp * np.exp(-0.5 * ((gx - cx) ** 2 + (gy - cy) ** 2) / s ** 2)
        out += w[:, None, None] * bump[None]
    out /= out.max()
    out += floor
    return normalise_mean_one(out)


def smooth_random_field(seed, X: int, Y: int, C: int = 3,
                        sigma_px: float = 4.0) -> np.ndarray:
    """U[0,1) noise, Gaussian-filtered over (y, x) with reflecting edges,
    standardised, exponentiated and normalised to mean 1."""
    rng = _rng(seed)
    noise = rng.uniform(0.0, 1.0, size=(C, Y, X))
    g = ndimage.gaussian_filter(noise, sigma=(0.0, sigma_px, sigma_px),
                                mode="reflect")
    g = (g - g.mean()) / g.std()
    return normalise_mean_one(np.exp(g))


def von_mises_hist(seed, n: int, floor: float = 1e-4) -> np.ndarray:
    """Periodic histogram on n bins: a von Mises mixture at bin centres.

    K ~ U{1..4} modes, mu ~ U[0, 1), kappa ~ U[1, 20], weights ~ Dirichlet(1);
    g(theta) = sum_k w_k exp(kappa_k (cos 2 pi (theta - mu_k) - 1)); peak
    scaled to 1, floor added, normalised to mean 1.
    """
    rng = _rng(seed)
    theta = (np.arange(n) + 0.5) / n
    k = int(rng.integers(1, 5))
    mu = rng.uniform(0.0, 1.0, size=k)
    kappa = rng.uniform(1.0, 20.0, size=k)
    w = rng.dirichlet(np.ones(k))
    g = np.zeros(n)
    for i in range(k):
        g += w[i] * np.exp(kappa[i] * (np.cos(2 * np.pi * (theta - mu[i])) - 1.0))
    g /= g.max()
    g += floor
    return normalise_mean_one(g)


# ---- the five workloads -------------------------------------------------

def cfg1_pair():
    """16 x 16 x 3, P = 8: three anisotropic Gaussians per channel (seeds 101/102)."""
    return aniso_gaussians(101, 16, 16), aniso_gaussians(102, 16, 16)


def cfg2_pair(seed0: int = 201, seed1: int = 202, X: int = 64, Y: int = 64):
    """64 x 64 x 3, P = 16: eight RGB-weighted bumps (seeds 201/202)."""
    return rgb_bumps(seed0, X, Y), rgb_bumps(seed1, X, Y)


def cfg3_pair(X: int = 256, Y: int = 256):
    """256 x 256 x 3, P = 32: exponentiated smooth random fields (seeds 301/302)."""
    return smooth_random_field(301, X, Y), smooth_random_field(302, X, Y)


HUE_BINS = (64, 128, 180, 256, 360)
HUE_STEPS = (16, 32)


def cfg4_problems(count: int = 1024, seed: int = 401):
    """Batched hue problems: list of (n, T, h0, h1) with uneven n and T."""
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for ss in children:
        rng = np.random.default_rng(ss)
        n = int(rng.choice(HUE_BINS))
        T = int(rng.choice(HUE_STEPS))
        s0, s1 = ss.spawn(2)
        out.append((n, T, von_mises_hist(s0, n), von_mises_hist(s1, n)))
    return out


def cfg5_pair(index: int, held_out: bool = False):
    """Warm-start pairs: drawn as the 64 x 64 x 3 workload.

    Training pair i uses seeds (10000 + 2i, 10001 + 2i); held-out pair i uses
    (900000 + 2i, 900001 + 2i).
    """
    base = 900000 if held_out else 10000
    return rgb_bumps(base + 2 * index, 64, 64), rgb_bumps(base + 2 * index + 1, 64, 64)


def random_pair(seed: int, X: int, Y: int, C: int = 3, floor: float = 0.05):
    """Small generic positive pair for unit tests of arbitrary shapes."""
    rng = _rng(seed)
    a = rng.uniform(floor, 1.0, size=(C, Y, X))
    b = rng.uniform(floor, 1.0, size=(C, Y, X))
    return normalise_mean_one(a), normalise_mean_one(b)


def hue_image(seed: int, H: int, W: int, sigma: float = 6.0) -> np.ndarray:
    """Synthetic 8-bit RGB photograph stand-in, (H, W, 3) uint8, rows first.

    Each channel is an independent smooth random field (white noise blurred
    with a periodic Gaussian of width `sigma` pixels, stretched to 0..255),
    so hues vary smoothly over the image with a few dominant families; a
    block of grey pixels (equal channels) sits in one corner.
    """
    rng = _rng(seed)
    ch = []
    for _ in range(3):
        z = ndimage.gaussian_filter(rng.standard_normal((H, W)), sigma, mode="wrap")
        z = (z - z.min()) / max(z.max() - z.min(), 1e-12)
        ch.append(np.round(255.0 * z))
    img = np.stack(ch, axis=-1).astype(np.uint8)
    gh, gw = max(H // 8, 1), max(W // 8, 1)
    img[:gh, :gw, :] = img[:gh, :gw, :1]
    return img
