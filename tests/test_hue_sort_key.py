"""The device sorts pixels by the 24-bit key floor(h 2^24) of their FP32 hue
instead of the hue itself.  Over every 8-bit colour this key is strictly
increasing across the distinct hue values, so both give the same strict
order (ties, equal hues, are broken by the raster index either way)."""
import numpy as np

from oracle import hue


def test_24_bit_key_orders_all_8_bit_hues_like_the_hue():
    v = np.arange(256, dtype=np.uint8)
    hs = []
    for r0 in range(256):
        g, b = np.meshgrid(v, v, indexing="ij")
        px = np.stack([np.full(65536, r0, np.uint8), g.ravel(), b.ravel()], axis=-1)
        hs.append(np.unique(hue.hue_of_rgb(px)[0]))
    h = np.unique(np.concatenate(hs))                       # every attainable FP32 hue
    assert h.min() >= 0 and h.max() < 1
    key = np.floor(h.astype(np.float64) * 2.0 ** 24)        # exact: power-of-two scaling
    assert np.all(np.diff(key) > 0)
    assert key.max() < 2 ** 24
    # the smallest gap between distinct hues, against the key's resolution
    assert np.diff(h.astype(np.float64)).min() > 2.0 ** -24
