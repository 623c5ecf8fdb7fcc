"""Planted mistakes in copies of the oracle must each fail at least one pin.

Each case rewrites one line of oracle/mandel_oracle.c (or its compile flags),
builds the copy with gcc in a temporary directory and runs a compact set of
the pins of test_oracle_pins.py against it: exact orbits, closed-form set
members, the first iterate, conjugation symmetry, the cusp law and brute
force on a tiny grid.  The unmodified oracle passes all of them."""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "oracle", "mandel_oracle.c")
BASE_FLAGS = ["-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

MUTATIONS = {
    "ge_instead_of_gt": ("if (s > R2)", "if (s >= R2)", None),
    "R_instead_of_R2": ("double R2 = R * R;", "double R2 = R;", None),
    "minus_cx": ("double xn = diff + cx;", "double xn = diff - cx;", None),
    "dropped_two": ("double twice = 2.0 * xy;", "double twice = xy;", None),
    "plus_yy": ("double diff = xx - yy;", "double diff = xx + yy;", None),
    "count_off_by_one": ("            return k;", "            return k + 1;", None),
    "sequential_update": ("double yn = twice + cy;", "double yn = 2.0 * xn * y + cy;", None),
    "no_half_pixel": ("double off_x = ((double)j + 0.5) - (double)n / 2.0;",
                      "double off_x = (double)j - (double)n / 2.0;", None),
    "rows_use_n": ("double off_y = ((double)i + 0.5) - (double)m / 2.0;",
                   "double off_y = ((double)i + 0.5) - (double)n / 2.0;", None),
    "fused_multiply_add": (None, None, ["-O2", "-std=gnu99", "-ffp-contract=fast", "-mfma",
                                        "-fPIC", "-shared"]),
}


def _build(tmp_path, name, old, new, flags):
    src = open(ORACLE_SRC).read()
    if old is not None:
        assert old in src, f"mutation {name}: pattern not found"
        src = src.replace(old, new, 1)
    path = tmp_path / f"{name}.c"
    path.write_text(src)
    lib = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", *(flags or BASE_FLAGS), str(path), "-o", str(lib)], check=True)
    L = ctypes.CDLL(str(lib))
    d, i32, i64, P = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.oracle_escape_count.argtypes = [d, d, i32, d]
    L.oracle_escape_count.restype = i32
    L.oracle_render.argtypes = [P, i32, i32, i32, d, P]
    L.oracle_render.restype = None
    return L


def _render(L, win, m, n, mi, R):
    w = np.ascontiguousarray(win, dtype=np.float64)
    out = np.empty((m, n), dtype=np.int32)
    L.oracle_render(w.ctypes.data, m, n, mi, R, out.ctypes.data)
    return out


def _brute(win, m, n, mi, R):
    cx0, cy0, dx, dy = win
    out = np.zeros((m, n), dtype=np.int32)
    for i in range(m):
        cy = cy0 + ((i + 0.5) - m / 2.0) * dy
        for j in range(n):
            cx = cx0 + ((j + 0.5) - n / 2.0) * dx
            x = y = 0.0
            c = mi
            for k in range(1, mi + 1):
                x, y = (x * x - y * y) + cx, 2.0 * (x * y) + cy
                if x * x + y * y > R * R:
                    c = k
                    break
            out[i, j] = c
    return out


def _pins_fail(L) -> list[str]:
    """Names of the compact pins that fail for library L."""
    failed = []
    golden = [(1, 0, 1000, 2, 3), (2, 0, 1000, 2, 2), (0, 2, 1000, 2, 2), (0.5, 0, 1000, 2, 5),
              (-1, 1, 1000, 2, 3), (-2.5, 0, 1000, 2, 1), (-2, 0, 1000, 2, 1000),
              (0, 1, 1000, 2, 1000), (1, 0, 1000, 1, 2), (3, 4, 1000, 400, 3)]
    if any(L.oracle_escape_count(a, b, mi, R) != e for a, b, mi, R, e in golden):
        failed.append("exact_orbits")
    rng = np.random.default_rng(1)
    mu = 0.9 * np.sqrt(rng.random(300)) * np.exp(2j * np.pi * rng.random(300))
    c = mu / 2 - mu * mu / 4
    if any(L.oracle_escape_count(z.real, z.imag, 500, 2.0) != 500 for z in c):
        failed.append("cardioid")
    pts = rng.uniform(-3, 3, (300, 2))
    if any((L.oracle_escape_count(a, b, 100, 2.0) == 1) != (a * a + b * b > 4.0) for a, b in pts):
        failed.append("first_iterate")
    pts = np.column_stack([rng.uniform(-2, 0.5, 300), rng.uniform(0, 1.2, 300)])
    if any(L.oracle_escape_count(a, b, 800, 2.0) != L.oracle_escape_count(a, -b, 800, 2.0)
           for a, b in pts):
        failed.append("conjugation")
    eps = 1e-6
    N = L.oracle_escape_count(0.25 + eps, 0.0, 10 ** 6, 2.0)
    if abs(N * math.sqrt(eps) - math.pi) > 5 * math.sqrt(eps):
        failed.append("cusp")
    win = (-0.5, 0.0, 3.0 / 24, 2.4 / 18)
    if not np.array_equal(_render(L, win, 18, 24, 300, 2.0), _brute(win, 18, 24, 300, 2.0)):
        failed.append("brute_force")
    # a zoomed view near the cardioid boundary: long, rounding-heavy orbits
    win = (-0.745, 0.113, 1e-4 / 12, 1e-4 / 12)
    if not np.array_equal(_render(L, win, 12, 12, 3000, 2.0), _brute(win, 12, 12, 3000, 2.0)):
        failed.append("brute_force_zoom")
    return failed


def test_equivalent_mutant_conjugate_c(tmp_path):
    # y' = 2xy - cy iterates z <- z^2 + conj(c), whose orbit from 0 is the exact
    # conjugate of the true one (round-to-nearest-even is sign-symmetric), so every
    # count is unchanged: not a mistake in the output, and no pin can or should see it.
    L = _build(tmp_path, "conj_c", "double yn = twice + cy;", "double yn = twice - cy;", None)
    assert _pins_fail(L) == []
    win = (-0.745, 0.113, 1e-3 / 16, 1e-3 / 16)
    ref = _build(tmp_path, "ref", None, None, None)
    assert np.array_equal(_render(L, win, 16, 16, 2000, 2.0), _render(ref, win, 16, 16, 2000, 2.0))


def test_unmodified_oracle_passes(tmp_path):
    L = _build(tmp_path, "unmodified", None, None, None)
    assert _pins_fail(L) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new, flags = MUTATIONS[name]
    L = _build(tmp_path, name, old, new, flags)
    failed = _pins_fail(L)
    assert failed, f"planted mistake {name} passed every pin"
