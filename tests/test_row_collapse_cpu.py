"""Host planning of collapsed rows (paper_2007_00745_amd/csrc/row_collapse.h), built
on its own with g++ and checked against numpy: the rendered rows are the distinct
row coordinates (cy0 + ((i + 0.5) - m/2) dy, as the kernels form them; keyed by |cy|
when conjugate rows merge), in order of first occurrence and written to that first
row; every other row is copied from the first row of its key, once; no copy source
is a copy destination, so the copies may run in any order, in place.  A row's count
depends only on its c (Sec. I, Eq. (1)-(2)), and conjugate points have equal counts
(the oracle's conjugation pin), so these copies reproduce the whole image."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2007_00745_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "row_collapse.h"
int main(int argc, char **argv) {
    double cy0, dy;
    std::sscanf(argv[1], "%la", &cy0);
    std::sscanf(argv[2], "%la", &dy);
    const int m = std::atoi(argv[3]);
    const bool mirror = std::atoi(argv[4]) != 0;
    mandel::RowCollapse rc;
    mandel::plan_row_collapse(cy0, dy, m, mirror, rc);
    std::printf("%zu %zu\n", rc.cy.size(), rc.pairs.size() / 2);
    for (size_t r = 0; r < rc.cy.size(); ++r) std::printf("%a %d\n", rc.cy[r], rc.first[r]);
    for (size_t q = 0; q < rc.pairs.size(); q += 2) std::printf("%d %d\n", rc.pairs[q], rc.pairs[q + 1]);
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("collapse")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-I", CSRC, str(src),
                    "-o", str(exe)], check=True)
    return str(exe)


def _plan(driver, cy0, dy, m, mirror):
    out = subprocess.run([driver, float(cy0).hex(), float(dy).hex(), str(m), str(int(mirror))],
                         check=True, capture_output=True, text=True).stdout.split("\n")
    nr, np_ = (int(x) for x in out[0].split())
    rows = [out[1 + r].split() for r in range(nr)]
    cy = [float.fromhex(a) for a, _ in rows]
    first = [int(b) for _, b in rows]
    pairs = [tuple(int(x) for x in out[1 + nr + q].split()) for q in range(np_)]
    return cy, first, pairs


CASES = [
    # (cy0, dy, m, mirror)
    (0.5627737049654734, 1e-17, 157, False),      # ~11 rows per coordinate
    (0.5627737049654734, 1.08e-16, 200, False),   # pitch just below the spacing: scattered merges
    (0.5627737049654734, 1e-12, 64, False),       # nothing merges
    (0.0, 0.0375, 64, True),                      # centred on the real axis, even m
    (0.0, 1e-3, 37, True),                        # odd m: the axis row stays alone
    (0.0, 0.0375, 64, False),                     # same window without mirroring: all distinct
    (0.3, 0.01, 100, True),                       # off-axis window that crosses it: partial mirror
    (-0.25, 5e-3, 100, True),                     # crossing below the axis
    (1e-300, 1e-310, 50, True),                   # subnormal pitch near zero
    (0.1, 0.0, 9, False),                         # zero pitch: one coordinate
    (0.7, 0.2, 1, True),                          # one row
    (0.7, 0.2, 0, True),                          # no rows
]


@pytest.mark.parametrize("cy0,dy,m,mirror", CASES)
def test_row_collapse_plan(driver, cy0, dy, m, mirror):
    cy, first, pairs = _plan(driver, cy0, dy, m, mirror)
    i = np.arange(m, dtype=np.float64)
    rows = cy0 + ((i + 0.5) - m / 2.0) * dy            # the kernels' operation order
    key = np.abs(rows) if mirror else rows + 0.0
    # rendered rows: the distinct keys in order of first occurrence, at their first row
    _, idx = np.unique(key, return_index=True)
    assert first == sorted(idx.tolist())
    assert [c.hex() for c in cy] == [float(rows[f]).hex() for f in first]
    # copies: every other row once, from the first row of its key
    assert len(first) + len(pairs) == m
    dsts = [d for d, _ in pairs]
    assert dsts == sorted(set(dsts)) and not set(dsts) & set(first)
    firsts = set(first)
    for d, s in pairs:
        assert s in firsts and s < d and key[d] == key[s]


def test_row_collapse_counts(driver):
    # the reductions the GPU tests rely on: a 1e-17 pitch near 0.56 merges rows about
    # 11-fold; a full window centred on the axis renders half its rows (plus the axis row)
    cy, first, pairs = _plan(driver, 0.5627737049654734, 1e-17, 157, False)
    assert len(first) < 157 // 5
    assert len(_plan(driver, 0.0, 0.0375, 64, True)[1]) == 32
    assert len(_plan(driver, 0.0, 1e-3, 37, True)[1]) == 19
