"""Display pyramid of a rendered frame, plainly (section 3: a static
high-resolution render is stored as TIFF and converted to a pyramidal tiled
TIFF for the tiled display).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module.  It shares no code with the GPU path.

Level 0: every channel of the premultiplied RGBA float image becomes
floor(clamp(v, 0, 1) * 255 + 1/2) (NaN counts as 0); in FP64 this is exact
for an FP32 v.  Level l+1: pixel (x, y) is, per channel, the rounded mean
(s + n // 2) // n of the n pixels (2x + a, 2y + b), a, b in {0, 1}, that
exist in level l.  Levels stop at the first whose sides both fit one tile.
"""
from __future__ import annotations

import numpy as np


def quantise(img) -> np.ndarray:
    v = np.asarray(img, dtype=np.float32).astype(np.float64)
    v = np.where(np.isnan(v), 0.0, v)
    v = np.clip(v, 0.0, 1.0)
    return np.floor(v * 255.0 + 0.5).astype(np.uint8)


def halve(level: np.ndarray) -> np.ndarray:
    """One 2x2 step, pixel by pixel over the output (slow, plain)."""
    h, w = level.shape[:2]
    h2, w2 = (h + 1) // 2, (w + 1) // 2
    out = np.zeros((h2, w2, 4), np.uint8)
    lv = level.astype(np.int64)
    for y in range(h2):
        for x in range(w2):
            s = np.zeros(4, np.int64)
            n = 0
            for b in (0, 1):
                for a in (0, 1):
                    if 2 * y + b < h and 2 * x + a < w:
                        s += lv[2 * y + b, 2 * x + a]
                        n += 1
            out[y, x] = (s + n // 2) // n
    return out


def pyramid(img, tile: int = 256) -> list:
    """List of levels, (h_l, w_l, 4) uint8 each."""
    levels = [quantise(img)]
    while levels[-1].shape[0] > tile or levels[-1].shape[1] > tile:
        levels.append(halve(levels[-1]))
    return levels


def pixel(img, level: int, x: int, y: int) -> np.ndarray:
    """Pixel (x, y) of pyramid level `level`, from the float image alone
    (the same rule, recursively over the 2^level-wide block it covers)."""
    h, w = np.asarray(img).shape[:2]
    if level == 0:
        return quantise(np.asarray(img)[y, x])
    hl, wl = h, w
    for _ in range(level - 1):
        hl, wl = (hl + 1) // 2, (wl + 1) // 2
    s = np.zeros(4, np.int64)
    n = 0
    for b in (0, 1):
        for a in (0, 1):
            if 2 * y + b < hl and 2 * x + a < wl:
                s += pixel(img, level - 1, 2 * x + a, 2 * y + b).astype(np.int64)
                n += 1
    return ((s + n // 2) // n).astype(np.uint8)
