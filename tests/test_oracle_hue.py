"""Pins of the hue image pipeline oracle (Sec. 5 and the cited periodic
histogram specification) against independent facts: Python's colorsys
for the hexcone, brute force over every circular shift and every integer
apportionment on small inputs, and a linear program for the W1 cost on
the circle."""
import colorsys
import itertools

import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import hue
from synth import inputs


def _pixels(seed, n):
    return np.random.default_rng(seed).integers(0, 256, size=(n, 3), dtype=np.uint8)


def test_hue_matches_colorsys():
    px = _pixels(1, 20000)
    h, hi, lo = hue.hue_of_rgb(px)
    for i in range(0, px.shape[0], 7):
        r, g, b = (int(v) / 255.0 for v in px[i])
        hh, ss, vv = colorsys.rgb_to_hsv(r, g, b)
        d = abs(float(h[i]) - hh)
        assert min(d, 1 - d) < 2e-6, (px[i], h[i], hh)
        assert hi[i] == round(vv * 255)
    grey = np.array([[0, 0, 0], [17, 17, 17], [255, 255, 255]], np.uint8)
    assert np.all(hue.hue_of_rgb(grey)[0] == 0)


def test_inverse_hexcone_matches_colorsys_and_round_trips():
    px = _pixels(2, 50000)
    h, hi, lo = hue.hue_of_rgb(px)
    assert np.array_equal(hue.rgb_of_hue(h, hi, lo), px)
    rng = np.random.default_rng(3)
    hh = rng.uniform(0, 1, 4000).astype(np.float32)
    hi = rng.integers(1, 256, 4000)
    lo = (hi * rng.uniform(0, 1, 4000)).astype(np.int64)
    out = hue.rgb_of_hue(hh, hi, lo).astype(np.int64)
    for i in range(hh.size):
        ref = colorsys.hsv_to_rgb(float(hh[i]), 1 - lo[i] / hi[i], hi[i] / 255.0)
        assert np.max(np.abs(out[i] - np.array(ref) * 255)) <= 0.5 + 1e-3


def test_histogram_bins_hold_their_hues():
    px = _pixels(4, 30000)
    n = 180
    h, _, _ = hue.hue_of_rgb(px)
    k = hue.hue_bins(h, n)
    c = hue.histogram(k, n)
    assert c.sum() == px.shape[0] and c.size == n
    hd = h.astype(np.float64)
    assert np.all(hd >= k / n - 1e-6) and np.all(hd < (k + 1) / n + 1e-6)


def test_target_counts_are_the_closest_apportionment():
    rng = np.random.default_rng(5)
    for _ in range(40):
        n = int(rng.integers(2, 5))
        N = int(rng.integers(1, 9))
        dens = rng.uniform(0, 1, n).astype(np.float32)
        dens[rng.integers(0, n)] = 0
        if dens.sum() == 0:
            continue
        c = hue.target_counts(dens, N, np.zeros(n, np.int64))
        x = N * dens.astype(np.float64) / dens.astype(np.float64).sum()
        best = min(sum(abs(np.array(v) - x))
                   for v in itertools.product(range(N + 1), repeat=n) if sum(v) == N)
        assert c.sum() == N and np.all(c >= 0)
        assert abs(np.abs(c - x).sum() - best) < 1e-9
    src = np.array([5, 0, 3, 2])
    assert np.array_equal(hue.target_counts(src.astype(np.float32), 10, src), src)
    z = np.zeros(4, np.float32)
    assert np.array_equal(hue.target_counts(z, 10, src), src)
    bad = np.array([np.nan, -1, np.inf, 2], np.float32)
    assert np.array_equal(hue.target_counts(bad, 10, src), [0, 0, 0, 10])


def _w1_circle_lp(a, b):
    """W1 between two count histograms on n periodic bins (linear program)."""
    n = a.size
    cost = np.array([[min(abs(i - j), n - abs(i - j)) for j in range(n)] for i in range(n)], float)
    A = []
    for i in range(n):
        row = np.zeros((n, n)); row[i, :] = 1; A.append(row.ravel())
    for j in range(n):
        col = np.zeros((n, n)); col[:, j] = 1; A.append(col.ravel())
    res = linprog(cost.ravel(), A_eq=np.array(A), b_eq=np.concatenate([a, b]).astype(float),
                  bounds=(0, None), method="highs")
    assert res.status == 0
    return res.fun


@pytest.mark.parametrize("seed", range(12))
def test_specification_is_exact_and_optimal(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 9))
    N = int(rng.integers(5, 40))
    ks = np.sort(rng.integers(0, n, N))          # source bins in rank order
    cs = hue.histogram(ks, n)
    dens = rng.uniform(0, 1, n).astype(np.float32) * (rng.uniform(0, 1, n) > 0.3)
    if dens.sum() == 0:
        dens[0] = 1
    ct = hue.target_counts(dens, N, cs)
    s = hue.circular_shift(cs, ct)
    out = hue.assign(N, ct, s)
    assert np.array_equal(hue.histogram(out, n), ct)          # exact
    cost = hue.circle_cost(ks, out, n)
    brute = min(hue.circle_cost(ks, hue.assign(N, ct, t), n) for t in range(-N, N + 1))
    assert cost == brute
    D = hue.edges(cs) - hue.edges(ct)
    assert cost == np.abs(D - s).sum()
    assert abs(cost - _w1_circle_lp(cs, ct)) < 1e-6


def test_specification_to_own_histogram_is_identity():
    img = inputs.hue_image(7, 48, 40)
    src = hue.Source(img, 64)
    out, k, ct, s = src.render(src.counts.astype(np.float32))
    assert s == 0 and np.array_equal(k, src.bins) and np.array_equal(ct, src.counts)
    assert np.array_equal(out, img.reshape(-1, 3))


def test_rendered_frame_has_the_target_hue_histogram():
    img = inputs.hue_image(8, 64, 64)
    n = 128
    src = hue.Source(img, n)
    target = np.roll(src.density(), 17).astype(np.float32)
    out, k, ct, s = src.render(target)
    assert np.array_equal(hue.histogram(k, n), ct)
    assert np.array_equal(ct, np.roll(src.counts, 17))
    kr = hue.hue_bins(hue.hue_of_rgb(out)[0], n)
    d = np.abs(kr - k) % n
    d = np.minimum(d, n - d)
    # 8-bit rounding moves a hue by up to 0.5 / (6 (max - min)): at most one
    # bin of 128 once max - min >= 32
    grey = src.hi == src.lo
    sat = (src.hi - src.lo) >= 32
    assert np.all(d[sat] <= 1) and np.mean(d[sat] == 0) > 0.9
    assert np.array_equal(out[grey], img.reshape(-1, 3)[grey])


def test_hsv_matches_colorsys_both_ways():
    px = _pixels(9, 30000)
    hsv = hue.hsv_of_rgb(px)
    for i in range(0, px.shape[0], 11):
        r, g, b = (int(v) / 255.0 for v in px[i])
        hh, ss, vv = colorsys.rgb_to_hsv(r, g, b)
        d = abs(float(hsv[i, 0]) - hh)
        assert min(d, 1 - d) < 2e-6 and abs(hsv[i, 1] - ss) < 1e-6 and abs(hsv[i, 2] - vv) < 1e-6
    rng = np.random.default_rng(10)
    x = rng.uniform(0, 1, (5000, 3)).astype(np.float32)
    out = hue.rgb_of_hsv(x).astype(np.int64)
    for i in range(x.shape[0]):
        ref = np.array(colorsys.hsv_to_rgb(*(float(v) for v in x[i]))) * 255
        assert np.max(np.abs(out[i] - ref)) <= 0.5 + 1e-3


def test_hsv_round_trip_is_exact_on_all_8_bit_colours():
    v = np.arange(256, dtype=np.uint8)
    for r0 in range(0, 256, 8):                     # 1/8 of the cube per test run
        r = np.full(256 * 256, r0, np.uint8)
        g, b = np.meshgrid(v, v, indexing="ij")
        px = np.stack([r, g.ravel(), b.ravel()], axis=-1)
        assert np.array_equal(hue.rgb_of_hsv(hue.hsv_of_rgb(px)), px)


def test_hsv_edge_values():
    x = np.array([[1.25, 0.5, 0.5], [-0.25, 0.5, 0.5], [0.5, 2.0, -1.0],
                  [np.nan, 0.5, 0.5], [0.5, np.inf, 0.5], [0.999999, 1.0, 1.0]], np.float32)
    out = hue.rgb_of_hsv(x)
    assert np.array_equal(out[0], hue.rgb_of_hsv(np.array([[0.25, 0.5, 0.5]], np.float32))[0])
    assert np.array_equal(out[1], hue.rgb_of_hsv(np.array([[0.75, 0.5, 0.5]], np.float32))[0])
    assert np.array_equal(out[2], [0, 0, 0]) and np.array_equal(out[3], [0, 0, 0])
    assert np.array_equal(out[4], [0, 0, 0]) and np.array_equal(out[5], [255, 0, 0])
