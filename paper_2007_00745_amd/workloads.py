"""Seeded synthetic workloads (inputs only; no escape-time arithmetic here).

Both the GPU path and the CPU oracle take their inputs from this module.  It
draws sizes, zooms, iteration limits and ray directions; it never iterates
z^2 + c.  A view "centred on the set boundary" is centred where a seeded ray
from c = 0 leaves the set: along c(t) = t (cos theta, sin theta), bisection
between t = 0 (inside) and t = 2.5 (outside) on the predicate "the escape-time
count at the view's max_iter equals max_iter" ends at two adjacent doubles t_in,
t_out, and the centre is c(t_in).  That bisection needs the escape-time count,
so it is not done here: a committed table (tests/golden/boundary_centres.json,
written by tests/golden/make_boundary_centres.py with the CPU oracle) holds the
centre of every seeded view, and this module reads it.  Each set of the table
repeats the max_iter of every view and a digest of the ray angles it was
bisected for, and a mismatch with the draws below is an error, so the table and
the draws cannot drift apart.

Every seeded view k of seed s draws from its own generator
numpy.random.default_rng([s, k]), in this order: theta ~ U[0, 2 pi), log10 of
the width ~ U[-10, -2], ln max_iter ~ U[ln 500, ln 20000] (rounded), then two
uniforms that pick the columns and rows in {lo..hi}.  Fixed sizes or limits
override the drawn ones without changing the draws.

Workloads (the paper's own is 8000 x 8000, iterationMax 2000, escape radius
400, Sec. IV, window not stated):
  c1  640 x 480, re in [-2, 1], im in [-1.2, 1.2], R = 2, max_iter 1000
  c2  8192 x 8192, same window, R = 2, max_iter 10000
  c3  64 views (seed 745), sizes uniform in {256..4096} per side, boundary
      centres, widths log-uniform in [1e-10, 1e-2], max_iter log-uniform in
      [500, 20000], R = 2
  c5  one 16384 x 16384 view of width 1e-12 at a boundary centre, max_iter
      50000 (seed 747), plus 4096 views of 512 x 512 drawn like c3 (seed 748)
  training  seeds 1000..1015, 64 views each, drawn like c3
  paper  8000 x 8000, max_iter 2000, R = 400, c1's window (assumed)
"""
from __future__ import annotations

import hashlib
import json
import math
import os
from dataclasses import dataclass

import numpy as np

CENTRES_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "tests", "golden", "boundary_centres.json")

# ray bisection: inside end c = 0, outside end at this distance
RAY_OUTSIDE_T = 2.5

# seeds whose views have bisected centres: seed -> (views, fixed max_iter or None)
BOUNDARY_SETS = {745: (64, None), 747: (1, 50000), 748: (4096, None),
                 **{s: (64, None) for s in range(1000, 1016)}}


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


@dataclass(frozen=True)
class Draw:
    theta: float     # ray angle
    width: float     # width of the view in the complex plane (columns * dx)
    max_iter: int
    u_cols: float    # uniforms in [0, 1) that pick the sizes
    u_rows: float


def draw(seed: int, k: int) -> Draw:
    """The seeded draws of view k of seed `seed` (see the module docstring)."""
    rng = np.random.default_rng([seed, k])
    theta = float(rng.uniform(0.0, 2.0 * math.pi))
    width = float(10.0 ** rng.uniform(-10.0, -2.0))
    max_iter = int(round(math.exp(rng.uniform(math.log(500.0), math.log(20000.0)))))
    u_cols, u_rows = (float(u) for u in rng.random(2))
    return Draw(theta, width, max_iter, u_cols, u_rows)


def ray_max_iter(seed: int, k: int) -> int:
    """max_iter that view k of a boundary set is bisected (and rendered) with."""
    fixed = BOUNDARY_SETS[seed][1]
    return fixed if fixed is not None else draw(seed, k).max_iter


def ray_specs():
    """(seed, k, theta, max_iter) of every view whose centre the table holds."""
    for seed, (count, _) in BOUNDARY_SETS.items():
        for k in range(count):
            yield seed, k, draw(seed, k).theta, ray_max_iter(seed, k)


_table = None
_checked: set = set()


def _centres() -> dict:
    global _table
    if _table is None:
        if not os.path.exists(CENTRES_PATH):
            raise FileNotFoundError(
                f"{CENTRES_PATH} is missing: run tests/golden/make_boundary_centres.py")
        with open(CENTRES_PATH) as f:
            _table = json.load(f)["sets"]
    return _table


def boundary_centre(seed: int, k: int) -> tuple[float, float]:
    """Bisected boundary centre of view k of seed `seed`, from the committed table."""
    sets = _centres()
    if str(seed) not in sets or k >= len(sets[str(seed)]["centre"]):
        raise KeyError(f"no bisected centre for seed {seed} view {k}")
    s = sets[str(seed)]
    if seed not in _checked:
        thetas = ",".join(draw(seed, j).theta.hex() for j in range(len(s["centre"])))
        if hashlib.sha256(thetas.encode()).hexdigest() != s["theta_sha256"]:
            raise ValueError(f"centre table for seed {seed} was bisected along other rays: "
                             f"regenerate it")
        _checked.add(seed)
    if s["max_iter"][k] != ray_max_iter(seed, k):
        raise ValueError(f"centre table entry for seed {seed} view {k} was bisected at "
                         f"another max_iter: regenerate it")
    cx, cy = s["centre"][k]
    return float.fromhex(cx), float.fromhex(cy)


def _pick(u: float, lo: int, hi: int) -> int:
    return lo + min(hi - lo, int(u * (hi - lo + 1)))


def seeded_view(seed: int, k: int, m: int | None = None, n: int | None = None,
                lo: int = 256, hi: int = 4096, width: float | None = None) -> View:
    d = draw(seed, k)
    n = _pick(d.u_cols, lo, hi) if n is None else n
    m = _pick(d.u_rows, lo, hi) if m is None else m
    cx, cy = boundary_centre(seed, k)
    pitch = (d.width if width is None else width) / n
    return View((cx, cy, pitch, pitch), m, n, ray_max_iter(seed, k), 2.0)


def c3(seed: int = 745, nviews: int = 64, lo: int = 256, hi: int = 4096) -> list[View]:
    return [seeded_view(seed, k, lo=lo, hi=hi) for k in range(nviews)]


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
    deep = seeded_view(seed_deep, 0, m=side, n=side, width=1e-12)
    return [deep] + [seeded_view(seed_stream, k, m=small, n=small) for k in range(nsmall)]


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
