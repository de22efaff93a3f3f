"""The hue oracle's pins catch plausible mistakes: each test plants one in a
copy of an oracle function (on the CPU) and checks that the independent fact
the pin uses -- brute force over shifts and apportionments, colorsys, the
exact output histogram -- rejects it."""
import colorsys
import itertools

import numpy as np

from oracle import hue


def _case(seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(3, 9))
    N = int(rng.integers(5, 40))
    ks = np.sort(rng.integers(0, n, N))
    cs = hue.histogram(ks, n)
    dens = rng.uniform(0, 1, n).astype(np.float32)
    ct = hue.target_counts(dens, N, cs)
    return n, N, ks, cs, ct


def _brute_best(n, N, ks, ct):
    return min(hue.circle_cost(ks, hue.assign(N, ct, t), n) for t in range(-N, N + 1))


def test_wrong_shift_sign_is_caught():
    caught = 0
    for seed in range(20):
        n, N, ks, cs, ct = _case(seed)
        s = hue.circular_shift(cs, ct)
        if hue.circle_cost(ks, hue.assign(N, ct, -s), n) != _brute_best(n, N, ks, ct):
            caught += 1
    assert caught > 0


def test_rounding_instead_of_largest_remainder_is_caught():
    def rounded(h, npix):
        x = npix * np.asarray(h, np.float64) / np.sum(np.asarray(h, np.float64))
        return np.rint(x).astype(np.int64)
    caught = 0
    rng = np.random.default_rng(7)
    for _ in range(40):
        n, N = int(rng.integers(2, 5)), int(rng.integers(1, 9))
        dens = rng.uniform(0.05, 1, n).astype(np.float32)
        c = rounded(dens, N)
        x = N * dens.astype(np.float64) / dens.astype(np.float64).sum()
        best = min(sum(abs(np.array(v) - x))
                   for v in itertools.product(range(N + 1), repeat=n) if sum(v) == N)
        if c.sum() != N or abs(np.abs(c - x).sum() - best) > 1e-9:
            caught += 1
    assert caught > 0


def test_swapped_hexcone_sectors_are_caught():
    def swapped(rgb):
        h, hi, lo = hue.hue_of_rgb(rgb[..., [1, 0, 2]])     # red and green exchanged
        return h
    px = np.random.default_rng(8).integers(0, 256, size=(500, 3), dtype=np.uint8)
    h = swapped(px)
    bad = 0
    for i in range(px.shape[0]):
        ref = colorsys.rgb_to_hsv(*(int(v) / 255.0 for v in px[i]))[0]
        d = abs(float(h[i]) - ref)
        bad += min(d, 1 - d) > 2e-6
    assert bad > 0

