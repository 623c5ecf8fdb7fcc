"""The paper's speed-up analysis, written out plainly (TEST INFRASTRUCTURE ONLY:
imported by tests, never by the library).

``parallel_fraction(t_p, t_s)``  -- Sec. II-B, Eq. (rp): r_p = t_p / t_s, the share
                                    of the serial run spent generating the set.
``amdahl_speedup(r_s, p)``       -- Sec. II-B (Amdahl's law): S_p = 1 / (r_s + r_p / p)
                                    with r_p = 1 - r_s; p = inf gives 1 / r_s.
``actual_speedup(t_1, t_n)``     -- Sec. V, Eq. (actualvst): time of one task over the
                                    time of n tasks.
``percentage_difference(T, A)``  -- Sec. V, Eq. (percen): |T - A| / ((T + A) / 2) * 100.

These are the formulas behind Tables I and II; they do not touch the counts.
"""
from __future__ import annotations

import math


def parallel_fraction(t_p: float, t_s: float) -> float:
    return t_p / t_s


def amdahl_speedup(r_s: float, p: float) -> float:
    r_p = 1.0 - r_s
    if math.isinf(p):
        return 1.0 / r_s
    return 1.0 / (r_s + r_p / p)


def actual_speedup(t_1: float, t_n: float) -> float:
    return t_1 / t_n


def percentage_difference(T: float, A: float) -> float:
    return abs(T - A) / ((T + A) / 2.0) * 100.0
