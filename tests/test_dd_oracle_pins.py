"""Pins of the double-double oracle (oracle/mandel_dd_oracle.c) against facts
that do not come from it: exact rational arithmetic for the error-free
transformations and the error bounds of the operations, the hand-derived exact
orbits of tests/golden/exact_orbits.txt (no rounding happens, so the count is
the exact one in any arithmetic), the closed-form interiors, the first iterate,
conjugation symmetry, a pure-Python double-double written separately (fma
through exact rationals) on tiny grids, and the pixel centres below binary64
resolution.  Planted mistakes in copies of the C file must each fail one of the
compact pins."""
import math
import os
import subprocess
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import dd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "exact_orbits.txt")
U2 = F(1, 2 ** 106)  # (2^-53)^2


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if line:
            re_, im_, mi, R, exp = line.split()
            rows.append((float(re_), float(im_), int(mi), float(R), int(exp)))
    return rows


def _rand_doubles(rng, k, lo=-30, hi=30):
    return [float(s * m * 2.0 ** e) for s, m, e in
            zip(rng.choice([-1, 1], k), rng.uniform(1, 2, k), rng.integers(lo, hi, k))]


def _dd_pair(rng, k):
    """Normalised double-double values (hi, lo) with |lo| <= ulp(hi) / 2."""
    out = []
    for h in _rand_doubles(rng, k):
        lo = float(rng.uniform(-0.5, 0.5)) * math.ulp(h)
        s = h + lo
        out.append((s, lo - (s - h)))
    return out


# ---- error-free transformations -------------------------------------------------

def test_two_sum_and_two_prod_are_exact():
    rng = np.random.default_rng(1)
    a, b = _rand_doubles(rng, 2000), _rand_doubles(rng, 2000)
    for x, y in zip(a, b):
        s, e = dd.op("two_sum", (x, 0.0), (y, 0.0))
        assert s == x + y and F(s) + F(e) == F(x) + F(y)
        p, e = dd.op("two_prod", (x, 0.0), (y, 0.0))
        assert p == x * y and F(p) + F(e) == F(x) * F(y)
        big, small = (x, y) if abs(x) >= abs(y) else (y, x)
        s, e = dd.op("quick_two_sum", (big, 0.0), (small, 0.0))
        assert F(s) + F(e) == F(x) + F(y)


def _rel(got, exact):
    return abs(F(got[0]) + F(got[1]) - exact) / abs(exact)


def test_operations_meet_double_double_accuracy():
    # add within 2u^2, products within 8u^2 of the exact result (u = 2^-53), and
    # every result normalised: a dropped term or an unrenormalised sum costs ~u.
    rng = np.random.default_rng(2)
    A, B = _dd_pair(rng, 1500), _dd_pair(rng, 1500)
    for a, b in zip(A, B):
        fa, fb = F(a[0]) + F(a[1]), F(b[0]) + F(b[1])
        for name, exact, bound in (("add", fa + fb, 2 * U2), ("mul", fa * fb, 8 * U2),
                                   ("sqr", fa * fa, 8 * U2)):
            bb = a if name == "sqr" else b
            r = dd.op(name, a, bb)
            if exact != 0:
                assert _rel(r, exact) <= bound, (name, a, b)
            assert abs(r[1]) <= math.ulp(r[0]) / 2 or r[0] == 0, (name, r)


def _cancelling_partner(rng, a):
    """b with b.hi = -a.hi and a low part of another scale: the high parts cancel
    and a.lo + b.lo is inexact, so the result lives in the low-part sum and its
    rounding error."""
    k = int(rng.integers(5, 40))
    return (-a[0], float(rng.uniform(-0.5, 0.5)) * math.ulp(a[0]) * 2.0 ** -k)


def test_add_with_cancellation():
    # x^2 - y^2 cancels in the update: the accurate addition keeps both low parts
    rng = np.random.default_rng(3)
    for a in _dd_pair(rng, 500):
        b = _cancelling_partner(rng, a)
        r = dd.op("add", a, b)
        exact = F(a[0]) + F(a[1]) + F(b[0]) + F(b[1])
        if exact != 0:
            assert _rel(r, exact) <= 2 * U2


# ---- counts ------------------------------------------------------------------------

@pytest.mark.parametrize("re_,im_,mi,R,exp", _golden())
def test_exact_orbits(re_, im_, mi, R, exp):
    assert dd.escape_count((re_, 0.0, im_, 0.0), mi, R) == exp


def test_closed_form_interiors_and_first_iterate():
    rng = np.random.default_rng(4)
    mu = 0.9 * np.sqrt(rng.random(200)) * np.exp(2j * np.pi * rng.random(200))
    for c in mu / 2 - mu * mu / 4:                      # main cardioid
        assert dd.escape_count((c.real, 0.0, c.imag, 0.0), 400, 2.0) == 400
    r = 0.2 * np.sqrt(rng.random(200))
    t = 2 * np.pi * rng.random(200)
    for x, y in zip(-1 + r * np.cos(t), r * np.sin(t)):  # period-2 disk |c + 1| <= 0.2
        assert dd.escape_count((x, 0.0, y, 0.0), 400, 2.0) == 400
    for x, y in rng.uniform(-3, 3, (400, 2)):            # z_1 = c: count 1 iff |c|^2 > R^2
        assert (dd.escape_count((x, 0.0, y, 0.0), 50, 2.0) == 1) == (x * x + y * y > 4.0)


def test_conjugation_symmetry():
    rng = np.random.default_rng(5)
    for x, y in zip(rng.uniform(-2, 0.5, 300), rng.uniform(0, 1.2, 300)):
        lo = float(rng.uniform(-1, 1)) * 1e-18
        c = (x, lo * 1e-3, y, lo)
        cc = (x, lo * 1e-3, -y, -lo)
        assert dd.escape_count(c, 600, 2.0) == dd.escape_count(cc, 600, 2.0)


# ---- independent pure-Python double-double ------------------------------------------

def _fma(a, b, c):
    return float(F(a) * F(b) + F(c))   # exact, then one rounding to nearest even


def _py_two_sum(a, b):
    s = a + b
    v = s - a
    return s, (a - (s - v)) + (b - v)


def _py_fast(a, b):
    s = a + b
    return s, b - (s - a)


def _py_add(a, b):
    s, e = _py_two_sum(a[0], b[0])
    t, f = _py_two_sum(a[1], b[1])
    s, e = _py_fast(s, e + t)
    return _py_fast(s, e + f)


def _py_mul(a, b):
    p = a[0] * b[0]
    e = _fma(a[0], b[0], -p)
    e = _fma(a[0], b[1], e)
    e = _fma(a[1], b[0], e)
    return _py_fast(p, e)


def _py_sqr(a):
    p = a[0] * a[0]
    e = _fma(a[0], a[0], -p)
    e = _fma(a[0] + a[0], a[1], e)
    return _py_fast(p, e)


def _py_count(win, m, n, i, j, mi, R):
    offx = (j + 0.5) - n / 2.0
    offy = (i + 0.5) - m / 2.0
    px = offx * win[4]
    py = offy * win[5]
    cx = _py_add((win[0], win[1]), (px, _fma(offx, win[4], -px)))
    cy = _py_add((win[2], win[3]), (py, _fma(offy, win[5], -py)))
    x = y = (0.0, 0.0)
    for k in range(1, mi + 1):
        xx, yy, xy = _py_sqr(x), _py_sqr(y), _py_mul(x, y)
        x = _py_add(_py_add(xx, (-yy[0], -yy[1])), cx)
        y = _py_add((2 * xy[0], 2 * xy[1]), cy)
        if x[0] * x[0] + y[0] * y[0] > R * R:
            return k
    return mi


@pytest.mark.parametrize("win,m,n,mi", [
    ((-0.5, 0.0, 0.0, 0.0, 3.0 / 8, 2.4 / 6), 6, 8, 60),
    ((-0.7436438870371587, -3.2e-17, 0.1318259042053119, 1.1e-17, 4e-17, 4e-17), 4, 5, 120),
])
def test_brute_force_python_double_double(win, m, n, mi):
    got = dd.render(win, m, n, mi, 2.0)
    want = np.array([[_py_count(win, m, n, i, j, mi, 2.0) for j in range(n)] for i in range(m)])
    assert np.array_equal(got, want)


def test_pixel_centres_below_binary64_resolution():
    # dx = 1e-17 near |c| ~ 0.75: binary64 centres collapse, double-double ones are
    # distinct, ascending, and within 2u^2 of the exact centre + offset * dx
    win = (-0.7436438870371587, 2.1e-17, 0.1318259042053119, -1.3e-17, 1e-17, 1e-17)
    m, n = 3, 64
    cs = [dd.pixel_c(win, m, n, 1, j) for j in range(n)]
    vals = [F(c[0]) + F(c[1]) for c in cs]
    assert all(b > a for a, b in zip(vals, vals[1:]))
    assert len({c[0] for c in cs}) < n // 4          # the high parts alone collapse
    for i in range(m):                                 # imaginary parts, row by row
        c = dd.pixel_c(win, m, n, i, 5)
        exact = F(win[2]) + F(win[3]) + (F(i) + F(1, 2) - F(m, 2)) * F(win[5])
        assert abs(F(c[2]) + F(c[3]) - exact) <= 2 * U2 * abs(exact)
    for j, v in enumerate(vals):
        exact = F(win[0]) + F(win[1]) + (F(j) + F(1, 2) - F(n, 2)) * F(win[4])
        assert abs(v - exact) <= 2 * U2 * abs(exact)


# ---- planted mistakes --------------------------------------------------------------

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "mandel_dd_oracle.c")
MUTATIONS = {
    "dropped_cross_term": ("    e = fma(a.lo, b.hi, e);\n", ""),
    "sqr_single_cross": ("fma(a.hi + a.hi, a.lo, p.lo)", "fma(a.hi, a.lo, p.lo)"),
    "quick_sum_in_add": ("    dd s = two_sum(a.hi, b.hi);", "    dd s = quick_two_sum(a.hi, b.hi);"),
    "dropped_low_sum": ("    e = s.lo + t.lo;", "    e = s.lo;"),
    "plus_yy": ("dd_add(dd_add(xx, dd_neg(yy)), cx)", "dd_add(dd_add(xx, yy), cx)"),
    "ge_test": ("if (s > R2)", "if (s >= R2)"),
    "no_half_pixel": ("double off_x = ((double)j + 0.5) - (double)n / 2.0;",
                      "double off_x = (double)j - (double)n / 2.0;"),
    "low_centre_dropped": ("dd cx0 = {win[0], win[1]}", "dd cx0 = {win[0], 0.0}"),
}


def _compact_pins_fail(L) -> list[str]:
    import ctypes
    d, i32, i64, P = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.oracle_dd_op.argtypes = [i32, d, d, d, d, P, P]
    L.oracle_dd_escape_count.argtypes = [P, i32, d]
    L.oracle_dd_escape_count.restype = i32
    L.oracle_dd_render.argtypes = [P, i32, i32, i32, d, P]
    L.oracle_dd_pixel_c.argtypes = [P, i32, i32, i64, i64, P]

    def op(k, a, b):
        rh, rl = ctypes.c_double(), ctypes.c_double()
        L.oracle_dd_op(k, a[0], a[1], b[0], b[1], ctypes.byref(rh), ctypes.byref(rl))
        return rh.value, rl.value

    def count(c, mi, R):
        arr = np.ascontiguousarray(c, dtype=np.float64)
        return L.oracle_dd_escape_count(arr.ctypes.data, mi, R)

    def render(win, m, n, mi):
        w = np.ascontiguousarray(win, dtype=np.float64)
        out = np.empty((m, n), dtype=np.int32)
        L.oracle_dd_render(w.ctypes.data, m, n, mi, 2.0, out.ctypes.data)
        return out

    failed = []
    win = np.array([-0.7436438870371587, 2.1e-17, 0.1318259042053119, -1.3e-17, 1e-17, 1e-17])
    for i, j in ((0, 0), (2, 63), (1, 17)):
        c = np.empty(4)
        L.oracle_dd_pixel_c(win.ctypes.data, 3, 64, i, j, c.ctypes.data)
        ex = F(win[0]) + F(win[1]) + (F(j) + F(1, 2) - 32) * F(win[4])
        ey = F(win[2]) + F(win[3]) + (F(i) + F(1, 2) - F(3, 2)) * F(win[5])
        if (abs(F(c[0]) + F(c[1]) - ex) > 2 * U2 * abs(ex)
                or abs(F(c[2]) + F(c[3]) - ey) > 2 * U2 * abs(ey)):
            failed.append("pixel_centres")
            break
    rng = np.random.default_rng(9)
    A, B = _dd_pair(rng, 300), _dd_pair(rng, 300)
    for a, b in zip(A, B):
        fa, fb = F(a[0]) + F(a[1]), F(b[0]) + F(b[1])
        b2 = _cancelling_partner(rng, a)
        fb2 = F(b2[0]) + F(b2[1])
        if (_rel(op(3, a, b), fa + fb) > 2 * U2 or _rel(op(5, a, b), fa * fb) > 8 * U2
                or _rel(op(4, a, a), fa * fa) > 8 * U2
                or (fa + fb2 != 0 and _rel(op(3, a, b2), fa + fb2) > 2 * U2)):
            failed.append("accuracy")
            break
    if any(count((re_, 0.0, im_, 0.0), mi, R) != exp for re_, im_, mi, R, exp in _golden()):
        failed.append("exact_orbits")
    for win, m, n, mi in (((-0.5, 0.0, 0.0, 0.0, 3.0 / 8, 2.4 / 6), 6, 8, 60),
                          ((-0.7436438870371587, -3.2e-17, 0.1318259042053119, 1.1e-17,
                            4e-17, 4e-17), 4, 5, 120)):
        want = np.array([[_py_count(win, m, n, i, j, mi, 2.0) for j in range(n)]
                         for i in range(m)])
        if not np.array_equal(render(win, m, n, mi), want):
            failed.append("brute_force")
            break
    return failed


def _build(tmp_path, name, old, new):
    import ctypes
    src = open(SRC).read()
    if old is not None:
        assert old in src, name
        src = src.replace(old, new, 1)
    path = tmp_path / f"{name}.c"
    path.write_text(src)
    lib = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", *dd.CFLAGS, str(path), "-o", str(lib), "-lm"], check=True)
    return ctypes.CDLL(str(lib))


def test_unmodified_dd_oracle_passes(tmp_path):
    assert _compact_pins_fail(_build(tmp_path, "unmodified", None, None)) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    assert _compact_pins_fail(_build(tmp_path, name, old, new)), name
