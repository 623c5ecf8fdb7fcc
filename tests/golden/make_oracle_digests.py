"""Writes tests/golden/oracle_digests.json: for every view of the 640 x 480 view (c1),
the 8192 x 8192 view at max_iter 10000 (c2) and the uneven 64-view batch (c3, seed
745), the SHA-256 of the oracle's image (int32, little-endian, row-major) and its sum
of counts; and the same for the double-double oracle's image of the deep-zoom view
(dd_deep: 4096 x 4096 at pitch 1e-17 around -0.7436438870371587 + 0.1318259042053119 i,
max_iter 20000, R 2); and one digest over the concatenated images of the 4096 small
views of the stress batch (c5 without its deep view, which is beyond a CPU run).  Only the CPU oracle computes the images (one single-threaded worker per
row band); the views come from the seeded input generator.  The GPU tests compare the
digests of whole GPU images with these, so every pixel of these workloads is checked
bit for bit without re-running the oracle on the test machine.

    python tests/golden/make_oracle_digests.py [--threads T] [--only c1,c2,c3,dd_deep,c5_small]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(ROOT, "tests", "golden", "oracle_digests.json")


def digest(img) -> str:
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(img, dtype="<i4").tobytes()).hexdigest()


DD_DEEP = dict(window=(-0.7436438870371587, 0.0, 0.1318259042053119, 0.0, 1e-17, 1e-17),
               m=4096, n=4096, max_iter=20000, R=2.0)


def dd_deep(threads: int) -> dict:
    """The double-double oracle's image of the deep-zoom view, in bands of rows."""
    import numpy as np

    import oracle.dd as dd
    d = DD_DEEP
    m, n = d["m"], d["n"]
    img = np.empty((m, n), dtype=np.int32)
    t0 = time.time()
    band = 64
    for r0 in range(0, m, band):
        r1 = min(m, r0 + band)
        idx = np.arange(r0 * n, r1 * n, dtype=np.int64)
        img[r0:r1] = dd.render_pixels(d["window"], m, n, d["max_iter"], d["R"], idx,
                                      threads=threads).reshape(r1 - r0, n)
        if r0 % 1024 == 0:
            print(f"dd_deep rows {r0}..{r1} ({time.time() - t0:.0f} s)", flush=True)
    return {"view": 0, "m": m, "n": n, "max_iter": d["max_iter"], "R": d["R"],
            "window": [float(x).hex() for x in d["window"]],
            "sha256": digest(img), "sum": int(img.sum(dtype="int64"))}


def c5_small(threads: int) -> dict:
    """One digest over the images of the stress batch's small views, concatenated in
    submission order (views 1 .. 4096 of c5), and their total sum of counts."""
    import oracle
    from paper_2007_00745_amd import workloads
    views = workloads.c5()[1:]
    h = hashlib.sha256()
    total = 0
    t0 = time.time()
    for k, v in enumerate(views):
        img, _ = oracle.render_parallel(v.window, v.m, v.n, v.max_iter, v.R, threads=threads)
        h.update(img.astype("<i4", copy=False).tobytes())
        total += int(img.sum(dtype="int64"))
        if k % 256 == 0:
            print(f"c5_small view {k + 1} ({time.time() - t0:.0f} s)", flush=True)
    return {"views": len(views), "first_view": 1, "sha256": h.hexdigest(), "sum": total,
            "m": views[0].m, "n": views[0].n}


def main() -> int:
    import oracle
    from paper_2007_00745_amd import workloads
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", default="c1,c2,c3")
    args = ap.parse_args()
    table = json.load(open(OUT)) if os.path.exists(OUT) else {}
    sets = {"c1": lambda: [workloads.c1()], "c2": lambda: [workloads.c2()],
            "c3": workloads.c3}
    for name in args.only.split(","):
        rows = []
        t0 = time.time()
        if name == "dd_deep":
            rows.append(dd_deep(args.threads))
        elif name == "c5_small":
            rows.append(c5_small(args.threads))
        else:
            for k, v in enumerate(sets[name]()):
                img, _ = oracle.render_parallel(v.window, v.m, v.n, v.max_iter, v.R,
                                                threads=args.threads)
                rows.append({"view": k, "m": v.m, "n": v.n, "max_iter": v.max_iter, "R": v.R,
                             "window": [float(x).hex() for x in v.window],
                             "sha256": digest(img), "sum": int(img.sum(dtype="int64"))})
                print(f"{name} view {k}: {v.m}x{v.n} max_iter {v.max_iter} "
                      f"sum {rows[-1]['sum']} ({time.time() - t0:.0f} s)", flush=True)
        table[name] = rows
        tmp = OUT + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, OUT)
    return 0


if __name__ == "__main__":
    sys.exit(main())
