"""Pins of the escape-time oracle to facts that do not come from the oracle.

Each test names the passage it follows (paper Sec. I, Eq. (1)-(2) for the
iteration and the count) and the kind of pin: exact worked orbits, closed
forms of the Mandelbrot set, exact invariants of IEEE round-to-nearest
arithmetic, asymptotic laws at the cusps, and brute force on tiny grids.
A plausible slip in the oracle -- a sign, a dropped term, >= for >, R for
R^2, an off-by-one count, a transposed pixel map, a fused multiply-add --
fails at least one of them (the comment on each test says which).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# The C1 workload: 640 x 480, re in [-2, 1], im in [-1.2, 1.2], R = 2, max_iter 1000,
# given as centre and pitch.
C1_WIN = (-0.5, 0.0, 3.0 / 640, 2.4 / 480)


def _exact_count(re, im, max_iter, R):
    """Eq. (1)-(2) in exact rational arithmetic.  Returns None once an iterate needs
    more than 52 significant bits (then binary64 would round and the exact orbit says
    nothing about the floating-point one).  Periodic orbits are detected exactly."""
    c = (Fraction(re), Fraction(im))
    x, y = Fraction(0), Fraction(0)
    R2 = Fraction(R) ** 2
    seen = {}
    for k in range(1, max_iter + 1):
        x, y = x * x - y * y + c[0], 2 * x * y + c[1]
        for v in (x, y):
            if v.denominator.bit_length() + v.numerator.bit_length() > 56:
                return None
        if x * x + y * y > R2:
            return k
        if (x, y) in seen:
            return max_iter
        seen[(x, y)] = k
    return max_iter


def _load_orbits():
    rows = []
    with open(os.path.join(GOLDEN, "exact_orbits.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            re_, im_, mi, R, exp = line.split()
            rows.append((float(re_), float(im_), int(mi), float(R), int(exp)))
    return rows


@pytest.mark.parametrize("re_,im_,mi,R,exp", _load_orbits())
def test_exact_orbits(oracle_mod, re_, im_, mi, R, exp):
    # P6: hand-derived orbits (golden file).  Catches >= vs > (ties at c=-2, 1, 2, 2i),
    # R vs R^2 (c=1), off-by-one counts (c=2), sign slips in y' (c=-1+i).
    assert oracle_mod.escape_count(re_, im_, mi, R) == exp
    # the stored values follow from exact rational arithmetic wherever the orbit is exact
    # (the orbits of 1/4 and -3/4 are not; the real segment [-2, 1/4] lies in the set)
    ex = _exact_count(re_, im_, mi, R)
    assert ex is None or ex == exp
    if (re_, im_) not in ((0.25, 0.0), (-0.75, 0.0)):
        assert ex == exp


def test_cardioid_interior(oracle_mod):
    # P2: c = mu/2 - mu^2/4 with |mu| <= 0.9 has an attracting fixed point (multiplier mu),
    # so the orbit is bounded: count = max_iter.  Catches a wrong x' or y' formula.
    rng = np.random.default_rng(7451)
    r = 0.9 * np.sqrt(rng.random(4000))
    th = rng.random(4000) * 2 * np.pi
    mu = r * np.exp(1j * th)
    c = mu / 2 - mu * mu / 4
    out = oracle_mod.escape_counts(c.real, c.imag, 2000, 2.0)
    assert np.all(out == 2000)


def test_period2_bulb(oracle_mod):
    # P3: the disk |c + 1| < 1/4 is the period-2 component; |c + 1| <= 0.2 keeps a margin.
    rng = np.random.default_rng(7452)
    r = 0.2 * np.sqrt(rng.random(4000))
    th = rng.random(4000) * 2 * np.pi
    c = -1 + r * np.exp(1j * th)
    out = oracle_mod.escape_counts(c.real, c.imag, 2000, 2.0)
    assert np.all(out == 2000)


def test_count_one_iff_c_outside(oracle_mod):
    # P4: z_1 = c exactly, so count == 1 iff fl(fl(cx^2) + fl(cy^2)) > R^2 (numpy float64
    # ufuncs round each operation once).  Points with |c| > 2 escape at once.
    rng = np.random.default_rng(7453)
    cx = rng.uniform(-3, 3, 20000)
    cy = rng.uniform(-3, 3, 20000)
    out = oracle_mod.escape_counts(cx, cy, 500, 2.0)
    s = cx * cx + cy * cy
    assert np.array_equal(out == 1, s > 4.0)
    # C1 corners (-2, +-1.2) are outside the radius-2 disk
    assert oracle_mod.escape_count(-2.0, 1.2, 1000, 2.0) == 1
    assert oracle_mod.escape_count(-2.0, -1.2, 1000, 2.0) == 1


def test_conjugation_symmetry_points(oracle_mod):
    # P5: round-to-nearest-even is sign-symmetric, so count(cx, -cy) == count(cx, cy).
    # Catches y' = 2xy - cy and similar sign slips (those break the symmetry of orbits).
    rng = np.random.default_rng(7454)
    cx = rng.uniform(-2.1, 0.6, 5000)
    cy = rng.uniform(0.0, 1.2, 5000)
    a = oracle_mod.escape_counts(cx, cy, 3000, 2.0)
    b = oracle_mod.escape_counts(cx, -cy, 3000, 2.0)
    assert np.array_equal(a, b)
    assert len(np.unique(a)) > 50  # a non-trivial sample


def test_c1_mirror_rows(oracle_mod):
    # P5 on the C1 image: cy0 = 0 and m even make row m-1-i the exact conjugate of row i.
    img = oracle_mod.render(C1_WIN, 480, 640, 1000, 2.0)
    assert np.array_equal(img, img[::-1, :])
    assert img.min() >= 1 and img.max() == 1000
    # left-right structure: the cardioid interior at c = -0.2 is in the set,
    # the point c = 0.45 is outside.  Catches a transposed (m, n) pixel map.
    i0 = 240  # row just above the real axis
    j_in = int(round((-0.2 - (-2.0)) / (3.0 / 640) - 0.5))
    j_out = int(round((0.45 - (-2.0)) / (3.0 / 640) - 0.5))
    assert img[i0, j_in] == 1000
    assert img[i0, j_out] < 100


def test_pixel_centres(oracle_mod):
    # Pixel map: centres at (j + 0.5)/n of the width and (i + 0.5)/m of the height.
    m, n = 480, 640
    cx, cy = oracle_mod.pixel_c(C1_WIN, m, n, 0, 0)
    assert abs(cx - (-2.0 + 0.5 * 3 / 640)) < 1e-15
    assert abs(cy - (-1.2 + 0.5 * 2.4 / 480)) < 1e-15
    cx, cy = oracle_mod.pixel_c(C1_WIN, m, n, m - 1, n - 1)
    assert abs(cx - (1.0 - 0.5 * 3 / 640)) < 1e-15
    assert abs(cy - (1.2 - 0.5 * 2.4 / 480)) < 1e-15
    # row i has im increasing with i; the centre window is exactly antisymmetric in im
    for i in range(m):
        a = oracle_mod.pixel_c(C1_WIN, m, n, i, 7)[1]
        b = oracle_mod.pixel_c(C1_WIN, m, n, m - 1 - i, 7)[1]
        assert a == -b
    xs = [oracle_mod.pixel_c(C1_WIN, m, n, 3, j)[0] for j in range(n)]
    assert all(b > a for a, b in zip(xs, xs[1:]))


def test_real_axis(oracle_mod):
    # P7: with cy = 0 the orbit stays real (y == +0), so the count is that of the scalar
    # recurrence x <- fl(fl(x*x) + c); every c in [-2, 1/4] is in the set; beyond 1/4
    # the count cannot increase with c (each step is monotone in x >= 0 and c).
    n = 2001
    win = (-0.875, 0.0, 3.0 / 2000, 1.0)   # m = 1: cy = 0 exactly; centres span [-2.375, 0.625]
    row = oracle_mod.render(win, 1, n, 5000, 2.0)[0]
    cxs = np.array([oracle_mod.pixel_c(win, 1, n, 0, j)[0] for j in range(n)])
    assert oracle_mod.pixel_c(win, 1, n, 0, 5)[1] == 0.0
    inside = (cxs >= -2.0) & (cxs <= 0.25)
    assert np.all(row[inside] == 5000)
    right = cxs > 0.25
    assert np.all(np.diff(row[right]) <= 0)
    for j in range(0, n, 37):
        x, k = 0.0, 0
        c = cxs[j]
        cnt = 5000
        for k in range(1, 5001):
            x = x * x + c
            if x * x > 4.0:
                cnt = k
                break
        assert row[j] == cnt


def test_prefix_property(oracle_mod):
    # P8: count(c, M1) == min(count(c, M2), M1) for M1 <= M2.
    rng = np.random.default_rng(7455)
    cx = rng.uniform(-2.0, 0.5, 3000)
    cy = rng.uniform(-1.2, 1.2, 3000)
    big = oracle_mod.escape_counts(cx, cy, 4000, 2.0)
    for M1 in (1, 2, 7, 100, 999, 4000):
        small = oracle_mod.escape_counts(cx, cy, M1, 2.0)
        assert np.array_equal(small, np.minimum(big, M1))


def test_radius_monotone(oracle_mod):
    # P9: a larger escape radius can only delay the escape when R >= 2.
    rng = np.random.default_rng(7456)
    cx = rng.uniform(-2.0, 0.5, 3000)
    cy = rng.uniform(-1.2, 1.2, 3000)
    prev = oracle_mod.escape_counts(cx, cy, 3000, 2.0)
    for R in (2.5, 4.0, 50.0, 400.0):
        cur = oracle_mod.escape_counts(cx, cy, 3000, R)
        assert np.all(cur >= prev)
        prev = cur


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8, 1e-10])
def test_cusp_quarter(oracle_mod, eps):
    # P10: at the cusp c = 1/4 + eps the escape time obeys N * sqrt(eps) -> pi, with an
    # O(1) remainder in N (allowed: 5 iterations).  Catches any change of the map itself.
    N = oracle_mod.escape_count(0.25 + eps, 0.0, 10 ** 7, 2.0)
    assert abs(N * math.sqrt(eps) - math.pi) <= 5 * math.sqrt(eps)


@pytest.mark.parametrize("eps", [1e-3, 1e-4, 1e-5, 1e-6])
def test_cusp_neck(oracle_mod, eps):
    # P10: at the neck c = -3/4 + i*eps the escape time obeys N * eps -> pi (remainder of at
    # most 5 iterations).  Exercises y' (the orbit is complex) and the cy mapping.
    N = oracle_mod.escape_count(-0.75, eps, 10 ** 8, 2.0)
    assert abs(N * eps - math.pi) <= 5 * eps


def _brute(win, m, n, max_iter, R):
    # Python floats: IEEE binary64, round-to-nearest-even per operation, never fused.
    cx0, cy0, dx, dy = win
    R2 = R * R
    out = np.zeros((m, n), dtype=np.int32)
    for i in range(m):
        cy = cy0 + ((i + 0.5) - m / 2.0) * dy
        for j in range(n):
            cx = cx0 + ((j + 0.5) - n / 2.0) * dx
            x = y = 0.0
            cnt = max_iter
            for k in range(1, max_iter + 1):
                x, y = (x * x - y * y) + cx, 2.0 * (x * y) + cy
                if x * x + y * y > R2:
                    cnt = k
                    break
            out[i, j] = cnt
    return out


def test_bruteforce_c1_small(oracle_mod):
    # P11: the C1 window at 32 x 24 with max_iter 1000, bit for bit.  Fails if the C
    # build fused a multiply-add or used extended precision.
    win = (-0.5, 0.0, 3.0 / 32, 2.4 / 24)
    assert np.array_equal(oracle_mod.render(win, 24, 32, 1000, 2.0), _brute(win, 24, 32, 1000, 2.0))


def test_bruteforce_zoomed_views(oracle_mod):
    # P11 on 16 seeded 16 x 16 zoomed views near the set (long, rounding-heavy orbits).
    rng = np.random.default_rng(745)
    for _ in range(16):
        th = rng.uniform(0, 2 * np.pi)
        mu = np.exp(1j * th)
        c = mu / 2 - mu * mu / 4          # a point of the main cardioid's boundary
        w = 10 ** rng.uniform(-6, -2)
        win = (c.real, c.imag, w / 16, w / 16)
        mi = int(rng.integers(200, 1500))
        a = oracle_mod.render(win, 16, 16, mi, 2.0)
        assert np.array_equal(a, _brute(win, 16, 16, mi, 2.0))


def test_row_bands_equal_whole(oracle_mod):
    # Splitting rows over workers changes nothing (Bernstein independence, Sec. II-A).
    win = (-0.5, 0.0, 3.0 / 96, 2.4 / 70)
    whole = oracle_mod.render(win, 70, 96, 700, 2.0)
    par, _ = oracle_mod.render_parallel(win, 70, 96, 700, 2.0, threads=5)
    assert np.array_equal(whole, par)
    idx = np.arange(0, 70 * 96, 13)
    assert np.array_equal(oracle_mod.render_pixels(win, 70, 96, 700, 2.0, idx, threads=3),
                          whole.ravel()[idx])
