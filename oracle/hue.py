"""Hue image pipeline of Sec. 5 (oracle; test infrastructure only).

Sec. 5 transports the normalised hue histograms of two images on the circle
with the 1D periodic solver and renders the frame at time t by giving the
first image's hue channel the histogram h^t (saturation and value kept), with
a periodic exact histogram specification that the paper only cites
([RDG11], [NS14]).  This module writes out the reading taken here, step by
step, in plain NumPy; it shares nothing with the device path.

Readings (the paper gives no formulas for this stage):

* Hue of an 8-bit RGB pixel: the textbook HSV hexcone hue in [0, 1), computed
  in FP32 from the integer channel differences (one rounded division per
  sector, then a division by 6).  Grey pixels (max = min) have hue 0.
* Histogram on n periodic bins: bin = floor(hue * n) (FP32 product), at most
  n - 1; counts are integers.
* Target counts for N pixels from a nonnegative density h on the n bins:
  x_k = N h_k / sum(h) in FP64 (sum taken bin by bin in index order), floor,
  and the remaining pixels one each to the bins with the largest fractional
  parts (equal parts: lower bin first).  A density with no mass keeps the
  source counts.
* Exact specification: pixels are put in a strict order, by hue and then by
  raster index (the tie-break of [NS14] uses local means; the index is taken
  here).  With C_s, C_t the cumulative source and target counts at the n bin
  edges, the circular shift s is the lower median of D_e = C_s[e] - C_t[e]:
  the minimiser of sum_e |D_e - s|, which is the W1 cost on the circle of a
  rotation of the monotone map ([RDG11]).  The pixel of rank r goes to the
  target bin that holds position (r - s) mod N of the target's cumulative
  counts, so the output bins have exactly the target counts.
* Rendering: the hue moves by whole bins, hue' = hue + (k_out - k_src) / n
  wrapped into [0, 1) (FP32); the pixel's max and min channels (value and
  saturation) are kept and RGB is rebuilt from the hexcone, rounded to 8 bits.

All FP32 steps are single rounded operations in a fixed order with no fused
multiply-add, so a device implementation doing the same operations matches
bit for bit.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def hue_of_rgb(rgb: np.ndarray):
    """Hue (float32, [0, 1)) and the max / min channel (int) of u8 RGB pixels.

    rgb: (..., 3) uint8.  Hexcone hue: the sector of the largest channel
    (red, then green, then blue on ties) plus the signed difference of the
    other two over max - min, divided by 6.
    """
    c = np.asarray(rgb).astype(np.int64)
    r, g, b = c[..., 0], c[..., 1], c[..., 2]
    hi = np.maximum(np.maximum(r, g), b)
    lo = np.minimum(np.minimum(r, g), b)
    d = (hi - lo).astype(F32)
    dsafe = np.where(d > 0, d, F32(1))
    with np.errstate(invalid="ignore", divide="ignore"):
        h_r = (g - b).astype(F32) / dsafe
        h_r = np.where(h_r < 0, h_r + F32(6), h_r).astype(F32)
        h_g = ((b - r).astype(F32) / dsafe + F32(2)).astype(F32)
        h_b = ((r - g).astype(F32) / dsafe + F32(4)).astype(F32)
    h6 = np.where(hi == r, h_r, np.where(hi == g, h_g, h_b)).astype(F32)
    h6 = np.where(d > 0, h6, F32(0)).astype(F32)
    h = (h6 / F32(6)).astype(F32)
    h = np.where(h >= F32(1), h - F32(1), h).astype(F32)
    return h, hi, lo


def hue_bins(h: np.ndarray, n: int) -> np.ndarray:
    """floor(h * n) in FP32, clamped to n - 1."""
    k = np.floor((h.astype(F32) * F32(n)).astype(F32)).astype(np.int64)
    return np.minimum(k, n - 1)


def histogram(bins: np.ndarray, n: int) -> np.ndarray:
    return np.bincount(bins.ravel(), minlength=n).astype(np.int64)


def target_counts(h: np.ndarray, npix: int, source: np.ndarray) -> np.ndarray:
    """Integer counts summing to npix, proportional to the density h
    (largest remainder, FP64, sum in index order).  Negative and non-finite
    entries count as zero."""
    h = [float(v) if (np.isfinite(v) and v > 0) else 0.0
         for v in np.asarray(h, dtype=np.float32)]
    S = 0.0
    for v in h:
        S += v
    if not S > 0.0:
        return np.asarray(source, dtype=np.int64).copy()
    x = [(float(npix) * v) / S for v in h]
    c = [int(np.floor(v)) for v in x]
    rem = [x[k] - c[k] for k in range(len(h))]
    left = npix - sum(c)          # in [0, n) unless rounding pushed an x_k up
    order = sorted(range(len(h)), key=lambda k: (-rem[k], k))
    for k in order[:max(left, 0)]:
        c[k] += 1
    return np.asarray(c, dtype=np.int64)


def edges(counts: np.ndarray) -> np.ndarray:
    """Cumulative counts at the n bin edges 0..n-1 (edge e: before bin e)."""
    return np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)


def circular_shift(cs: np.ndarray, ct: np.ndarray) -> int:
    """Lower median of D_e = C_s[e] - C_t[e] over the n edges."""
    D = np.sort(np.asarray(edges(cs)) - np.asarray(edges(ct)))
    return int(D[(D.size - 1) // 2])


def assign(npix: int, ct: np.ndarray, s: int) -> np.ndarray:
    """Target bin of each rank r = 0..npix-1: the bin holding (r - s) mod N."""
    q = np.mod(np.arange(npix, dtype=np.int64) - s, npix)
    cum = np.cumsum(ct)
    return np.searchsorted(cum, q, side="right").astype(np.int64)


def rgb_of_hue(h: np.ndarray, hi: np.ndarray, lo: np.ndarray) -> np.ndarray:
    """Hexcone inverse with value hi and minimum lo kept, rounded to u8."""
    h = np.asarray(h, dtype=F32)
    hiF = np.asarray(hi).astype(F32)
    loF = np.asarray(lo).astype(F32)
    d = (hiF - loF).astype(F32)
    h6 = (h * F32(6)).astype(F32)
    i = np.floor(h6).astype(np.int64)
    i = np.clip(i, 0, 5)
    f = (h6 - i.astype(F32)).astype(F32)
    x = (d * f).astype(F32)
    up = (loF + x).astype(F32)
    down = (hiF - x).astype(F32)
    r = np.choose(i, [hiF, down, loF, loF, up, hiF])
    g = np.choose(i, [up, hiF, hiF, down, loF, loF])
    b = np.choose(i, [loF, loF, up, hiF, hiF, down])
    out = np.stack([r, g, b], axis=-1).astype(F32)
    out = np.floor((out + F32(0.5)).astype(F32))
    return np.clip(out, 0, 255).astype(np.uint8)


def hsv_of_rgb(rgb: np.ndarray) -> np.ndarray:
    """HSV (float32, (..., 3)) of u8 RGB: the hexcone hue above, saturation
    (max - min) / max (0 for black), value max / 255."""
    h, hi, lo = hue_of_rgb(rgb)
    hiF = np.asarray(hi).astype(F32)
    d = (hiF - np.asarray(lo).astype(F32)).astype(F32)
    with np.errstate(invalid="ignore", divide="ignore"):
        sat = np.where(hiF > 0, (d / np.where(hiF > 0, hiF, F32(1))).astype(F32), F32(0))
    val = (hiF / F32(255)).astype(F32)
    return np.stack([h, sat.astype(F32), val], axis=-1).astype(F32)


def rgb_of_hsv(hsv: np.ndarray) -> np.ndarray:
    """u8 RGB of float HSV by the textbook hexcone: h wrapped into [0, 1),
    sector i = floor(6h), f = 6h - i, p = v (1 - s), q = v (1 - s f),
    t = v (1 - s (1 - f)); each channel floor(255 c + 0.5), clamped.  s and v
    are clamped to [0, 1]; non-finite inputs give black."""
    x = np.asarray(hsv, dtype=F32)
    h, sat, val = x[..., 0], x[..., 1], x[..., 2]
    bad = ~(np.isfinite(h) & np.isfinite(sat) & np.isfinite(val))
    h = np.where(bad, F32(0), h).astype(F32)
    sat = np.clip(np.where(bad, F32(0), sat), 0, 1).astype(F32)
    val = np.clip(np.where(bad, F32(0), val), 0, 1).astype(F32)
    h = (h - np.floor(h).astype(F32)).astype(F32)
    h = np.where(h >= F32(1), h - F32(1), h).astype(F32)
    h6 = (h * F32(6)).astype(F32)
    i = np.clip(np.floor(h6).astype(np.int64), 0, 5)
    f = (h6 - i.astype(F32)).astype(F32)
    one = F32(1)
    p = (val * (one - sat).astype(F32)).astype(F32)
    q = (val * (one - (sat * f).astype(F32)).astype(F32)).astype(F32)
    t = (val * (one - (sat * (one - f).astype(F32)).astype(F32)).astype(F32)).astype(F32)
    r = np.choose(i, [val, q, p, p, t, val])
    g = np.choose(i, [t, val, val, q, p, p])
    b = np.choose(i, [p, p, t, val, val, q])
    out = np.stack([r, g, b], axis=-1).astype(F32)
    out = np.floor(((out * F32(255)).astype(F32) + F32(0.5)).astype(F32))
    return np.clip(out, 0, 255).astype(np.uint8)


class Source:
    """The first image's hue data: hue, bins, counts and the strict order."""

    def __init__(self, rgb: np.ndarray, n: int):
        px = np.asarray(rgb, dtype=np.uint8).reshape(-1, 3)
        self.rgb = px
        self.n = n
        self.h, self.hi, self.lo = hue_of_rgb(px)
        self.bins = hue_bins(self.h, n)
        self.counts = histogram(self.bins, n)
        # strict order: by hue, equal hues by raster index (stable sort)
        self.order = np.argsort(self.h, kind="stable")
        self.rank = np.empty_like(self.order)
        self.rank[self.order] = np.arange(self.order.size)

    def density(self) -> np.ndarray:
        """Hue histogram normalised to mean one over the bins (the solver's
        density convention)."""
        N = self.rgb.shape[0]
        return self.counts.astype(np.float64) * (self.n / N)

    def specify(self, target: np.ndarray):
        """Exact periodic specification to the density `target`:
        returns (output bins per pixel, target counts, shift)."""
        N = self.rgb.shape[0]
        ct = target_counts(target, N, self.counts)
        s = circular_shift(self.counts, ct)
        k_of_rank = assign(N, ct, s)
        return k_of_rank[self.rank], ct, s

    def render(self, target: np.ndarray):
        """The frame for the density `target`: (u8 RGB (N, 3), bins, counts, shift)."""
        k_out, ct, s = self.specify(target)
        dk = (k_out - self.bins).astype(F32)
        h2 = (self.h + (dk / F32(self.n)).astype(F32)).astype(F32)
        h2 = np.where(h2 >= F32(1), h2 - F32(1), h2).astype(F32)
        h2 = np.where(h2 < F32(0), h2 + F32(1), h2).astype(F32)
        h2 = np.where(h2 >= F32(1), h2 - F32(1), h2).astype(F32)
        return rgb_of_hue(h2, self.hi, self.lo), k_out, ct, s


def circle_cost(k_src: np.ndarray, k_out: np.ndarray, n: int) -> int:
    """Sum over pixels of the circular bin distance moved."""
    d = np.abs(np.asarray(k_src) - np.asarray(k_out)) % n
    return int(np.minimum(d, n - d).sum())
