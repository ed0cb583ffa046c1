"""Host logic of bench.py (CPU): the lane-slot count of a walk, from per-group
list lengths and sizes, by the walk's own rules: blocks of 64 list entries,
S = 8, 4, 2, 1 lane streams for groups of at most 8, 16, 32, 64 members, a
block's entries padded to a multiple of 4 S."""
import importlib.util
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _slots_by_hand(e, c):
    S = 8 if c <= 8 else 4 if c <= 16 else 2 if c <= 32 else 1
    total = 0
    while e > 0:
        blk = min(64, e)
        padded = -(-blk // (4 * S)) * (4 * S)
        total += padded // S
        e -= blk
    return total


def test_walk_lane_slots_cases():
    b = _bench()
    # a 64-member group with 130 entries: two full blocks (128 slots) and 2
    # entries padded to 4
    assert b.walk_lane_slots(np.array([130]), np.array([64])) == 132
    # 8 members (8 streams): a full block is 8 slots; 36 entries pad to 64
    assert b.walk_lane_slots(np.array([100]), np.array([8])) == 16
    # 20 members (2 streams): one full block, 32 slots
    assert b.walk_lane_slots(np.array([64]), np.array([20])) == 32
    assert b.walk_lane_slots(np.array([0]), np.array([5])) == 0


def test_walk_lane_slots_matches_blockwise_count():
    b = _bench()
    rng = np.random.default_rng(11)
    e = rng.integers(0, 5000, 500)
    c = rng.integers(1, 65, 500)
    assert b.walk_lane_slots(e, c) == sum(_slots_by_hand(int(x), int(y)) for x, y in zip(e, c))
