"""The paper's row partitions, written out plainly (TEST INFRASTRUCTURE ONLY).

``naive_rows``        -- Sec. III-A, Eq. (stp), (etp), (rem): rank r of N takes
                         the contiguous rows S_r .. E_r, S_r = floor(rows/N)*r,
                         E_r = floor(rows/N)*(r+1) - 1, and the last rank also
                         takes the rows - N*floor(rows/N) leftover rows.
                         The printed Eq. (etp) reads "(r x 1)"; it is taken as
                         (r + 1), the only reading under which consecutive
                         ranks tile the image.
``alternating_rows``  -- Sec. III-C: rank r takes rows r, r+N, r+2N, ... for
                         floor(rows/N) rows; the master (rank 0) also takes the
                         leftover rows N*floor(rows/N) .. rows-1.
``fcfs_message_count`` etc. -- Sec. III, Eq. (naive_m), (fcfs_m), (al_m).
"""
from __future__ import annotations


def naive_rows(rows: int, N: int, r: int) -> list[int]:
    q = rows // N
    start = q * r
    end = q * (r + 1) - 1
    if r == N - 1:
        end += rows % N
    return list(range(start, end + 1))


def alternating_rows(rows: int, N: int, r: int) -> list[int]:
    q = rows // N
    mine = [r + k * N for k in range(q)]
    if r == 0:
        mine += list(range(q * N, rows))
    return mine


def naive_message_count(N: int) -> int:
    return N - 1


def fcfs_message_count(rows: int) -> int:
    return 2 * rows


def alternating_message_count(N: int) -> int:
    return N - 1
