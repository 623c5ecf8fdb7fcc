"""Writes tests/golden/boundary_centres.json: the centre of every seeded view whose
workload asks for a centre "on the set boundary" (the uneven batch, the stress
batch and the cost-model training views).

For view k of seed s, the input generator draws a ray angle theta and the view's
max_iter.  Along c(t) = (t cos theta, t sin theta) the end t_in = 0 (c = 0, which
never escapes) is inside and t_out = 2.5 (|c| > 2, which escapes at the first
update) is outside, where "inside" means that the CPU oracle's escape-time count
(Sec. I, Eq. (1)-(2), R = 2) at the view's max_iter equals max_iter.  The
midpoint t = (t_in + t_out) / 2 replaces the end with the same predicate value
until it equals one of the ends bit for bit; the centre is then c(t_in).  The
predicate need not be monotone along the ray, so the result is some place where
the count switches from max_iter to escaping between two adjacent doubles of t:
a point of the set's boundary at the resolution of binary64 and of max_iter.

Only the oracle decides the predicate; the angles and limits come from the
seeded input generator, and the products t cos theta, t sin theta are plain
binary64.  Every double is stored as a hex float; each set also keeps the
max_iter of every view and a SHA-256 of its ray angles (hex floats joined by
commas), which the generator checks on every read.

    python tests/golden/make_boundary_centres.py
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

R = 2.0


def ray_point(t: float, theta: float) -> tuple[float, float]:
    return t * math.cos(theta), t * math.sin(theta)


def bisect_ray(theta: float, max_iter: int, t_out: float, count) -> tuple[float, float, int]:
    """(t_in, t_out, steps) at the end of the bisection; count(cx, cy) is the oracle."""
    t_in = 0.0
    steps = 0
    assert count(*ray_point(t_in, theta)) == max_iter
    assert count(*ray_point(t_out, theta)) < max_iter
    while True:
        t = 0.5 * (t_in + t_out)
        if t == t_in or t == t_out:
            return t_in, t_out, steps
        steps += 1
        if count(*ray_point(t, theta)) == max_iter:
            t_in = t
        else:
            t_out = t


def main() -> int:
    import oracle
    from paper_2007_00745_amd import workloads
    t0 = time.time()
    sets: dict = {}
    for seed, k, theta, max_iter in workloads.ray_specs():
        def count(cx, cy, mi=max_iter):
            return oracle.escape_count(cx, cy, mi, R)
        t_in, t_out, steps = bisect_ray(theta, max_iter, workloads.RAY_OUTSIDE_T, count)
        cx, cy = ray_point(t_in, theta)
        s = sets.setdefault(str(seed), {"theta": [], "max_iter": [], "centre": []})
        s["theta"].append(theta.hex())
        s["max_iter"].append(max_iter)
        s["centre"].append([cx.hex(), cy.hex()])
        if k == 0:
            print(f"seed {seed}: view 0 theta {theta:.6f} max_iter {max_iter} "
                  f"t_in {t_in:.17g} after {steps} steps ({time.time() - t0:.1f} s)", flush=True)
    for s in sets.values():
        # the angles are the generator's own draws: a digest of them is enough to
        # catch a table written for other draws
        s["theta_sha256"] = hashlib.sha256(",".join(s.pop("theta")).encode()).hexdigest()
    table = {
        "recipe": "ray c(t) = (t cos theta, t sin theta); bisection on t between 0 (inside) "
                  "and 2.5 (outside); inside = oracle escape count at the view's max_iter "
                  "equals max_iter, R = 2; stop when the midpoint equals an end; centre = c(t_in)",
        "R": R,
        "t_outside": workloads.RAY_OUTSIDE_T,
        "sets": sets,
    }
    path = workloads.CENTRES_PATH
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, separators=(",", ":"))
    os.replace(tmp, path)
    print(f"wrote {path}: {sum(len(s['centre']) for s in sets.values())} centres "
          f"({time.time() - t0:.1f} s)")
    return 0


if __name__ == "__main__":
    sys.exit(main())
