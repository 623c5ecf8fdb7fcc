"""The paper's output path written out plainly (TEST INFRASTRUCTURE ONLY: imported
by the tests, never by the library).

``boolean_colour(counts, max_iter)``  -- Sec. I with Eq. (2): a pixel's colour
    follows from its count; Boolean escape time: count == max_iter (never
    escaped) -> black (0, 0, 0), otherwise white (255, 255, 255).
``ppm_bytes(rgb, m, n)``              -- Sec. III: the master writes the image to a
    PPM file; binary PPM (P6) with maxval 255: the ASCII header "P6", width,
    height, maxval, each followed by one newline, then R, G, B bytes per pixel,
    rows top to bottom.
"""
from __future__ import annotations

import numpy as np


def boolean_colour(counts, max_iter: int) -> np.ndarray:
    counts = np.asarray(counts)
    out = np.empty(counts.shape + (3,), dtype=np.uint8)
    for idx in np.ndindex(counts.shape):
        v = 0 if counts[idx] >= max_iter else 255
        out[idx] = (v, v, v)
    return out


def ppm_bytes(rgb, m: int, n: int) -> bytes:
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8).reshape(m, n, 3)
    return f"P6\n{n} {m}\n255\n".encode("ascii") + rgb.tobytes()
