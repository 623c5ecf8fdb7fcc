"""Seeded synthetic workloads (inputs only; no escape-time arithmetic here).

Both the GPU path and the CPU oracle take their inputs from this module.  It
draws sizes, zooms, iteration limits and view centres; it never iterates
z^2 + c.  View centres "on the set boundary" are exact boundary points in
closed form: the main cardioid c = e^{it}/2 - e^{2it}/4 and the period-2 disk
|c + 1| = 1/4 (both are boundaries of hyperbolic components of the set).

Workloads (the paper's own is 8000 x 8000, iterationMax 2000, escape radius
400, Sec. IV, window not stated):
  c1  640 x 480, re in [-2, 1], im in [-1.2, 1.2], R = 2, max_iter 1000
  c2  8192 x 8192, same window, R = 2, max_iter 10000
  c3  64 views, sizes uniform in {256..4096} per side, widths log-uniform in
      [1e-10, 1e-2], max_iter log-uniform in [500, 20000], R = 2 (seed 745)
  c5  one 16384 x 16384 view of width 1e-12 at a boundary point, max_iter
      50000 (seed 747), plus 4096 views of 512 x 512 drawn like c3 (seed 748)
  paper  8000 x 8000, max_iter 2000, R = 400, c1's window (assumed)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class View:
    window: tuple  # (cx0, cy0, dx, dy)
    m: int         # rows
    n: int         # columns
    max_iter: int
    R: float = 2.0

    @property
    def pixels(self) -> int:
        return self.m * self.n


def window_from_bounds(re_min: float, re_max: float, im_min: float, im_max: float,
                       m: int, n: int) -> tuple:
    """Centre and pitch of the rectangle [re_min, re_max] x [im_min, im_max] split
    into n columns and m rows."""
    return ((re_min + re_max) / 2.0, (im_min + im_max) / 2.0,
            (re_max - re_min) / n, (im_max - im_min) / m)


def c1() -> View:
    return View(window_from_bounds(-2.0, 1.0, -1.2, 1.2, 480, 640), 480, 640, 1000, 2.0)


def c2(side: int = 8192, max_iter: int = 10000) -> View:
    return View(window_from_bounds(-2.0, 1.0, -1.2, 1.2, side, side), side, side, max_iter, 2.0)


def paper_view() -> View:
    return View(window_from_bounds(-2.0, 1.0, -1.2, 1.2, 8000, 8000), 8000, 8000, 2000, 400.0)


def boundary_point(rng: np.random.Generator) -> tuple[float, float]:
    """A point of the set's boundary: main cardioid (3/4) or period-2 disk (1/4)."""
    t = rng.uniform(0.0, 2.0 * math.pi)
    if rng.random() < 0.75:
        c = complex(math.cos(t), math.sin(t)) / 2 - complex(math.cos(2 * t), math.sin(2 * t)) / 4
    else:
        c = -1 + complex(math.cos(t), math.sin(t)) / 4
    return c.real, c.imag


def random_view(rng: np.random.Generator, m: int | None = None, n: int | None = None,
                lo: int = 256, hi: int = 4096) -> View:
    if n is None:
        n = int(rng.integers(lo, hi + 1))
    if m is None:
        m = int(rng.integers(lo, hi + 1))
    cx, cy = boundary_point(rng)
    width = 10.0 ** rng.uniform(-10.0, -2.0)
    max_iter = int(round(math.exp(rng.uniform(math.log(500.0), math.log(20000.0)))))
    d = width / n
    return View((cx, cy, d, d), m, n, max_iter, 2.0)


def c3(seed: int = 745, nviews: int = 64, lo: int = 256, hi: int = 4096) -> list[View]:
    rng = np.random.default_rng(seed)
    return [random_view(rng, lo=lo, hi=hi) for _ in range(nviews)]


def c3_scaled(seed: int = 745, nviews: int = 64, scale: int = 16) -> list[View]:
    """c3's views with every side divided by `scale` (same centres, zooms, limits):
    a small batch of the same shape mix for tests."""
    out = []
    for v in c3(seed, nviews):
        m, n = max(1, v.m // scale), max(1, v.n // scale)
        w = v.window
        out.append(View((w[0], w[1], w[2] * v.n / n, w[3] * v.n / n), m, n, v.max_iter, v.R))
    return out


def c5(seed_deep: int = 747, seed_stream: int = 748, side: int = 16384, nsmall: int = 4096,
       small: int = 512) -> list[View]:
    rng = np.random.default_rng(seed_deep)
    cx, cy = boundary_point(rng)
    d = 1e-12 / side
    deep = View((cx, cy, d, d), side, side, 50000, 2.0)
    rng2 = np.random.default_rng(seed_stream)
    return [deep] + [random_view(rng2, m=small, n=small) for _ in range(nsmall)]


def training_views(seeds=range(1000, 1016), per_seed: int = 64, lo: int = 256,
                   hi: int = 4096) -> list[View]:
    """Views for cost-model training: c3's distribution, seeds disjoint from c3/c5."""
    out = []
    for s in seeds:
        out += c3(s, per_seed, lo, hi)
    return out


def out_offsets(views) -> list[int]:
    """Element offset of each view's image in one packed output buffer."""
    offs, acc = [], 0
    for v in views:
        offs.append(acc)
        acc += v.pixels
    return offs
