"""Pins of the oracle's group bounds (the inputs of the group-wise Eq. 2 test):
the members' exact FP32 bounding box, amin = the smallest member |a_old| and
dA = delta_acc * amin rounded to FP32.

Independent references: hand-built groups whose accelerations are
Pythagorean quadruples (every square, sum and root exact in FP32, so amin is
known exactly), numpy min/max over each group's own index range, and |a| in
FP64 for random accelerations (amin within one FP32 ulp of it). Neighbours
outside every group carry extreme coordinates and the smallest |a|, so a
range that is off by one member changes the box and amin."""
import numpy as np
import pytest

import oracle


def _groups(begin, count):
    b = np.asarray(begin, np.int64)
    c = np.asarray(count, np.int64)
    return oracle.Groups(b, c, np.zeros_like(b))


def test_group_bounds_hand_built(orc):
    # sorted particles 0..9; groups [1, 4) and [5, 9); particles 0, 4, 9 lie
    # outside every group with far-away positions and the smallest |a|
    x = np.array([-100, 0.5, 2.0, -1.0, 100, 3.0, 3.0, 2.5, 4.0, 100], np.float32)
    y = np.array([-100, 1.0, -2.0, 0.0, 100, 0.0, 1.0, -1.0, 0.5, -100], np.float32)
    z = np.array([100, 0.0, 0.25, -0.5, -100, 7.0, 6.0, 8.0, 6.5, 100], np.float32)
    # |a| = 1, 9, 3, 7 | 5 | 13, 3, 9, 15 | 1   (Pythagorean quadruples)
    a = np.array([[0, 0, 1], [1, 4, 8], [1, 2, 2], [2, 3, 6], [3, 4, 0],
                  [3, 4, 12], [2, 1, 2], [4, 4, 7], [2, 10, 11], [1, 0, 0]], np.float32)
    grp = _groups([1, 5], [3, 4])
    for dacc in (2.0 ** -9, 0.1):
        lo, hi, amin, dA = orc.group_bounds(grp, x, y, z, a, dacc)
        # group 0: members 1..3, smallest |a| = 3 at its second member
        np.testing.assert_array_equal(lo[0], [-1.0, -2.0, -0.5])
        np.testing.assert_array_equal(hi[0], [2.0, 1.0, 0.25])
        # group 1: members 5..8, smallest |a| = 3 at its second member
        np.testing.assert_array_equal(lo[1], [2.5, -1.0, 6.0])
        np.testing.assert_array_equal(hi[1], [4.0, 1.0, 8.0])
        np.testing.assert_array_equal(amin, np.array([3.0, 3.0], np.float32))
        want = np.float32(dacc) * np.float32(3.0)  # one FP32 rounding of the product
        np.testing.assert_array_equal(dA, np.array([want, want], np.float32))
    # 0.1f * 3 is inexact in FP32: the stored value is the rounded product
    assert float(np.float32(np.float32(0.1) * np.float32(3.0))) != 0.1 * 3.0


def test_group_bounds_single_member_and_no_acceleration(orc):
    x = np.array([1.0, -2.0, 5.0], np.float32)
    y = np.array([0.0, 3.0, 5.0], np.float32)
    z = np.array([4.0, 4.0, 5.0], np.float32)
    a = np.array([[6, 2, 3], [0, 0, 0], [1, 1, 1]], np.float32)  # |a| = 7, 0, sqrt 3
    grp = _groups([0, 1, 2], [1, 1, 1])
    lo, hi, amin, dA = orc.group_bounds(grp, x, y, z, a, 0.5)
    np.testing.assert_array_equal(lo, np.stack([x, y, z], 1))
    np.testing.assert_array_equal(hi, np.stack([x, y, z], 1))
    assert amin[0] == 7.0 and amin[1] == 0.0
    assert amin[2] == np.float32(np.sqrt(3.0))  # correctly rounded root of an exact 3
    np.testing.assert_array_equal(dA, np.float32(0.5) * amin)
    # no previous acceleration (bootstrap): amin = dA = 0, the box unchanged
    lo2, hi2, amin2, dA2 = orc.group_bounds(grp, x, y, z, None, 0.5)
    np.testing.assert_array_equal(lo2, lo)
    np.testing.assert_array_equal(hi2, hi)
    assert (amin2 == 0).all() and (dA2 == 0).all()


@pytest.mark.parametrize("seed", [0, 1])
def test_group_bounds_random_against_numpy(orc, seed):
    rng = np.random.default_rng(seed)
    n = 5000
    x, y, z = (rng.normal(size=n).astype(np.float32) for _ in range(3))
    a = (rng.normal(size=(n, 3)) * rng.lognormal(size=(n, 1))).astype(np.float32)
    # contiguous groups of 1..64 members with gaps of 0..2 particles between them
    begin, count, s = [], [], 0
    while True:
        s += int(rng.integers(0, 3))
        c = int(rng.integers(1, 65))
        if s + c > n:
            break
        begin.append(s)
        count.append(c)
        s += c
    grp = _groups(begin, count)
    dacc = 2.0 ** -9
    lo, hi, amin, dA = orc.group_bounds(grp, x, y, z, a, dacc)
    amag = np.sqrt((a.astype(np.float64) ** 2).sum(1))
    for g, (b, c) in enumerate(zip(begin, count)):
        sl = slice(b, b + c)
        np.testing.assert_array_equal(lo[g], [x[sl].min(), y[sl].min(), z[sl].min()])
        np.testing.assert_array_equal(hi[g], [x[sl].max(), y[sl].max(), z[sl].max()])
        ref = amag[sl].min()
        assert abs(float(amin[g]) - ref) <= np.spacing(np.float32(ref)), (g, amin[g], ref)
        # the smallest member, not the largest or the first
        k = int(np.argmin(amag[sl]))
        assert abs(float(amin[g]) - amag[b + k]) <= np.spacing(np.float32(ref))
    np.testing.assert_array_equal(dA, (np.float32(dacc) * amin).astype(np.float32))
