"""Pins of the paper's row partitions (oracle/partition.py) and of the load
imbalance that motivates them, against what the paper states:

* naive rows (Sec. III-A, Eq. (stp), (etp), (rem)): rank r starts at
  floor(rows/N)*r, every rank but the last has floor(rows/N) contiguous rows,
  the last also has the rows mod N leftover rows; all ranks together cover every
  row exactly once, in order;
* alternating rows (Sec. III-C): rank r has rows r, r+N, ... (floor(rows/N) of
  them) and the master (rank 0) the leftover rows; again every row exactly once;
* message counts (Eq. (naive_m), (fcfs_m), (al_m)): N - 1, 2 * rows, N - 1 --
  for FCFS independent of N;
* the observation driving the paper (Sec. III-A, Sec. V): the top and bottom of
  the image are cheap and the middle expensive, so the naive partition leaves
  the outer ranks nearly idle while the alternating one evens out the work.
The last point is computed from oracle counts of the 640 x 480 view."""
import numpy as np
import pytest

import oracle
from oracle import partition
from paper_2007_00745_amd import workloads

CASES = [(480, 1), (480, 2), (480, 7), (480, 16), (480, 32), (8000, 32), (7, 7), (5, 8), (101, 10)]


@pytest.mark.parametrize("rows,N", CASES)
def test_naive_rows(rows, N):
    q = rows // N
    got = [partition.naive_rows(rows, N, r) for r in range(N)]
    for r, mine in enumerate(got):
        want_len = q + (rows % N if r == N - 1 else 0)
        assert len(mine) == want_len
        if mine:
            assert mine[0] == q * r and mine == list(range(mine[0], mine[0] + len(mine)))
    assert [row for mine in got for row in mine] == list(range(rows))


@pytest.mark.parametrize("rows,N", CASES)
def test_alternating_rows(rows, N):
    q = rows // N
    got = [partition.alternating_rows(rows, N, r) for r in range(N)]
    for r, mine in enumerate(got):
        assert mine[:q] == [r + k * N for k in range(q)]
        assert mine[q:] == (list(range(q * N, rows)) if r == 0 else [])
    assert sorted(row for mine in got for row in mine) == list(range(rows))


def test_message_counts():
    for N in (2, 4, 8, 16, 32):
        assert partition.naive_message_count(N) == N - 1
        assert partition.alternating_message_count(N) == N - 1
    # FCFS: one row index out and one row back per row, whatever N is
    assert partition.fcfs_message_count(8000) == 16000


def test_middle_rows_cost_more_and_alternating_balances():
    v = workloads.c1()
    img = oracle.render(v.window, v.m, v.n, v.max_iter, v.R).astype(np.int64)
    row_cost = img.sum(axis=1)
    m = v.m
    outer = row_cost[: m // 4].sum() + row_cost[3 * m // 4:].sum()
    middle = row_cost[m // 4: 3 * m // 4].sum()
    assert middle > 3 * outer
    for N in (4, 8, 16):
        naive = np.array([row_cost[partition.naive_rows(m, N, r)].sum() for r in range(N)])
        alt = np.array([row_cost[partition.alternating_rows(m, N, r)].sum() for r in range(N)])
        assert naive.max() / naive.min() > 5          # outer ranks nearly idle
        assert alt.max() / alt.min() < 1.1            # interleaving evens the work out
        assert naive.sum() == alt.sum() == row_cost.sum()
