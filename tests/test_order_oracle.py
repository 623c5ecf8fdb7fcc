"""Pins of the bucket-order reference (oracle/order.py) to hand-computed buckets:
with HI = 50 and a scale of exactly 78.75 buckets per unit, a key k lands in
floor((50 - k) * 78.75) wherever that product is exact, the ends clamp, infinities
go to the end buckets and NaN after every number.  Valid orders are recognised and
invalid ones rejected."""
import math

import numpy as np
import pytest

from oracle import order


def test_scale_is_exact():
    assert float(order.SCALE) == 78.75 == 4095 / 52


@pytest.mark.parametrize("key, want", [
    (50.0, 0), (49.0, 78), (48.0, 157), (49.5, 39), (0.0, 3937), (-1.0, 4016),
    (10.0, 3150), (-1.5, 4055), (-2.0, 4094), (-3.0, 4094), (-1e30, 4094), (51.0, 0),
    (1e30, 0), (math.inf, 0), (-math.inf, 4094), (math.nan, 4095),
    # a key just below 50: (50 - k) * 78.75 < 1, still bucket 0
    (np.nextafter(np.float32(50), np.float32(0)), 0),
    # products that are exact integers land on the bucket they name (floor, not round)
    (42.0, 630), (46.0, 315), (49.75, 19), (34.0, 1260),
])
def test_hand_computed_buckets(key, want):
    assert int(order.bucket([key])[0]) == want


def test_buckets_monotone_in_key():
    k = np.sort(np.random.default_rng(1).uniform(-5, 55, 20000).astype(np.float32))[::-1]
    assert np.all(np.diff(order.bucket(k)) >= 0)


def test_order_desc_is_valid_and_descending():
    rng = np.random.default_rng(2)
    keys = rng.uniform(-3, 52, 5000).astype(np.float32)
    keys[rng.choice(5000, 7, replace=False)] = np.nan
    keys[:3] = [np.inf, -np.inf, 50.0]
    p = order.order_desc(keys)
    assert order.is_valid_order(keys, p)
    kk = keys[p]
    assert np.all(np.isnan(kk[-7:])) and not np.any(np.isnan(kk[:-7]))
    # whole-bucket granularity: inside [LO, HI] keys decrease up to one bucket width
    fin = kk[:-7][(kk[:-7] >= -2) & (kk[:-7] <= 50)]
    assert np.all(np.diff(fin) <= 1.0 / 78.75 + 1e-5)
    # out-of-range keys sit in the end buckets, with the in-range keys of those buckets
    b = order.bucket(kk)
    assert np.all(b[kk > 50] == 0) and np.all(b[kk < -2] == order.BUCKETS - 2)


def test_invalid_orders_rejected():
    keys = np.array([1.0, 40.0, 20.0, np.nan], dtype=np.float32)
    assert order.is_valid_order(keys, [1, 2, 0, 3])
    assert not order.is_valid_order(keys, [2, 1, 0, 3])   # ascending pair
    assert not order.is_valid_order(keys, [1, 2, 3, 0])   # NaN before a number
    assert not order.is_valid_order(keys, [1, 2, 0])      # not a permutation
    assert not order.is_valid_order(keys, [1, 1, 0, 3])
    # equal keys, or keys sharing a bucket, may come in any order
    same = np.array([3.0, 3.0, 3.001], dtype=np.float32)
    assert order.is_valid_order(same, [0, 1, 2]) and order.is_valid_order(same, [2, 1, 0])
