"""Reference of the descending bucket order of tile keys (TEST INFRASTRUCTURE ONLY).

The paper has no tile order: its first-come-first-served partition hands rows out
in index order (Sec. III-B).  The library adds longest-processing-time-first list
scheduling (Graham), where the queue visits tiles by predicted cost, descending.
Its order is a counting sort on a fixed grid of buckets, so this module states
which bucket each key falls in, and what every valid order must look like:

  * B = 4096 buckets.  Numbers use buckets 0 .. B - 2: key k goes to
        floor(clamp((HI - k) * S, 0, B - 2)),   HI = 50, LO = -2,
        S = (B - 1) / (HI - LO) = 4095 / 52 = 78.75 (exact in binary32),
    with HI - k and the product each rounded to binary32 (the precision in which
    the order is taken), so k = HI lands in bucket 0, k = LO (and below, and -inf)
    in bucket B - 2, keys above HI (and +inf) in bucket 0.
  * NaN keys go to bucket B - 1, after every number.
  * A valid order is a permutation whose bucket sequence is non-decreasing, i.e.
    equal to the sorted list of all keys' buckets; the order inside one bucket is
    free.
"""
from __future__ import annotations

import numpy as np

BUCKETS = 4096
KEY_LO = np.float32(-2.0)
KEY_HI = np.float32(50.0)
SCALE = np.float32(BUCKETS - 1) / (KEY_HI - KEY_LO)   # binary32 78.75


def bucket(keys) -> np.ndarray:
    """Bucket index of every key (binary32 keys; see the module docstring)."""
    k = np.asarray(keys, dtype=np.float32)
    with np.errstate(invalid="ignore", over="ignore"):
        u = (KEY_HI - k) * SCALE                       # two binary32 roundings
        u = np.where(np.isnan(k), np.float32(0), u)    # NaN keys are placed below
        b = np.floor(np.minimum(np.maximum(u, np.float32(0)), np.float32(BUCKETS - 2)))
    return np.where(np.isnan(k), BUCKETS - 1, b).astype(np.int64)


def order_desc(keys) -> np.ndarray:
    """One valid order: tiles by bucket, ties in index order."""
    return np.argsort(bucket(keys), kind="stable")


def bucket_sequence(keys) -> np.ndarray:
    """The bucket sequence that every valid order of these keys visits."""
    return np.sort(bucket(keys))


def is_valid_order(keys, perm) -> bool:
    """perm is a permutation of range(len(keys)) visiting buckets in ascending order."""
    perm = np.asarray(perm, dtype=np.int64)
    n = len(np.asarray(keys))
    if perm.shape != (n,) or not np.array_equal(np.sort(perm), np.arange(n)):
        return False
    return bool(np.array_equal(bucket(np.asarray(keys, dtype=np.float32)[perm]),
                               bucket_sequence(keys)))
