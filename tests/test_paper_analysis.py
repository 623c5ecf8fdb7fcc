"""Pins of the paper's speed-up analysis (oracle/analysis.py) against the values
it prints: Table I follows from the serial fraction alone, and Table II (b) from
Table II (a).  Fixture: tests/golden/paper_tables.txt (Tables I and II)."""
import math
import os

import pytest

from oracle import analysis

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.txt")


def _tables():
    t1, t2a, t2b = {}, {}, {}
    for line in open(GOLDEN):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        key = math.inf if f[1] == "inf" else int(f[1])
        vals = [float(x) for x in f[2:]]
        {"table1": t1, "table2a": t2a, "table2b": t2b}[f[0]][key] = vals
    return t1, t2a, t2b


def test_table1_from_the_serial_fraction():
    # r_s = 1 / S_inf (the p -> inf row); every finite row must then round to the print.
    t1, _, _ = _tables()
    r_s = 1.0 / t1[math.inf][0]
    assert analysis.parallel_fraction(1.0 - r_s, 1.0) == pytest.approx(0.99719, abs=1e-5)
    for p, (s,) in t1.items():
        got = analysis.amdahl_speedup(r_s, p)
        assert round(got, 5) == pytest.approx(s, abs=1e-9), p


def test_table2a_theoretical_column_is_table1():
    t1, t2a, _ = _tables()
    for n, row in t2a.items():
        assert row[0] == t1[n][0]


def test_table2b_from_table2a():
    # Each printed input carries up to 5e-6 of rounding; |dPD/dT| + |dPD/dA| =
    # 400 / (T + A), so the recomputed value may differ from the print by at most
    # 400 / (T + A) * 5e-6 plus the 5e-6 rounding of the print itself.
    _, t2a, t2b = _tables()
    for n, (T, *acts) in t2a.items():
        for A, want in zip(acts, t2b[n]):
            got = analysis.percentage_difference(T, A)
            tol = 400.0 / (T + A) * 5e-6 + 5e-6
            assert abs(got - want) <= tol, (n, A, got, want)


def test_percentage_difference_properties():
    assert analysis.percentage_difference(3.0, 3.0) == 0.0
    assert analysis.percentage_difference(2.0, 1.0) == analysis.percentage_difference(1.0, 2.0)
    assert analysis.percentage_difference(1.0, 0.0) == 200.0   # the largest possible value
    assert analysis.actual_speedup(10.0, 2.5) == 4.0
    assert analysis.amdahl_speedup(0.0, 8) == 8.0                # fully parallel
    assert analysis.amdahl_speedup(1.0, 8) == 1.0                # fully serial
