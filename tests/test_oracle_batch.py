"""Pins of the oracle's batch of independent systems in one tree: the system
digits on top of the key, a spatial part equal to each system's own Morton
key cut to 21 - r levels (checked against a plain bit-interleave), system
roots at level r, and forces, lists and groups identical to separate runs of
each system (when no single-system cell needs more than 21 - r levels)."""
import numpy as np
import pytest

import nbody_inputs as I


def _batch(n_sys, seed, lo=7.0, hi=10.5):
    ps = I.cluster_batch(n_sys, seed, log2_min=lo, log2_max=hi)
    off = np.concatenate([[0], np.cumsum([p.n for p in ps])]).astype(np.int64)
    cat = lambda k: np.concatenate([p.f32()[k] for p in ps])  # noqa: E731
    return ps, off, cat(0), cat(1), cat(2), cat(6)


def test_system_digits(orc):
    assert [orc.system_digits(s) for s in (1, 2, 8, 9, 64, 65, 512, 513)] == \
        [0, 1, 1, 2, 2, 3, 3, 4]


def _interleave(qx, qy, qz, bits):
    k = 0
    for b in range(bits):
        k |= ((qx >> b) & 1) << (3 * b + 2)
        k |= ((qy >> b) & 1) << (3 * b + 1)
        k |= ((qz >> b) & 1) << (3 * b)
    return k


def test_batch_keys(orc):
    ps, off, x, y, z, m = _batch(9, 3)
    k, boxes, r = orc.batch_keys(x, y, z, off)
    assert r == 2
    bits = 21 - r
    for s in range(9):
        a, b = off[s], off[s + 1]
        assert np.all((k[a:b] >> np.uint64(3 * bits)) == s)
        box = orc.root_cube(x[a:b], y[a:b], z[a:b])
        np.testing.assert_array_equal(boxes[s], box)
        k21, _ = orc.keys(x[a:b], y[a:b], z[a:b])
        np.testing.assert_array_equal(k[a:b] & np.uint64((1 << (3 * bits)) - 1),
                                      k21 >> np.uint64(3 * r))
        for i in range(a, min(b, a + 20)):
            q = [min(int(np.floor((float(c) - box[j]) * 2.0 ** bits / box[3])), 2 ** bits - 1)
                 for j, c in enumerate((x[i], y[i], z[i]))]
            assert int(k[i]) == (s << (3 * bits)) | _interleave(*q, bits)


# (the second batch holds systems of 2 to about 3000 particles: neighbouring
# system roots small enough to be group cells, which must not be joined)
@pytest.mark.parametrize("merge", [0, 1])
@pytest.mark.parametrize("S,seed,lo,hi", [(9, 5, 7.0, 10.5), (40, 7, 1.0, 12.0)])
def test_batch_equals_separate_systems(orc, merge, S, seed, lo, hi):
    ps, off, x, y, z, m = _batch(S, seed, lo, hi)
    r = orc.system_digits(S)
    rb = orc.tree_forces(x, y, z, m, a_old=None, systems=off, group_merge=merge)
    cl = rb.cells
    # every cell above the system digits is split; the level-r cells are the
    # system roots, holding exactly their systems' particles
    assert np.all(cl.n_child[cl.level < r] > 0)
    roots = np.flatnonzero(cl.level == r)
    np.testing.assert_array_equal(cl.pbegin[roots], off[:-1])
    np.testing.assert_array_equal(cl.pcount[roots], np.diff(off))
    a_old = rb.acc.astype(np.float32)
    rb = orc.tree_forces(x, y, z, m, a_old=a_old, systems=off, group_merge=merge)
    # no group spans two systems
    sys_of = np.searchsorted(off, rb.grp.begin, side="right") - 1
    assert np.all(rb.grp.begin + rb.grp.count <= off[sys_of + 1])
    for s in range(S):
        a, b = off[s], off[s + 1]
        rs = orc.tree_forces(x[a:b], y[a:b], z[a:b], m[a:b], a_old=a_old[a:b],
                             group_merge=merge)
        if (rs.cells.level[rs.cells.n_child > 0] >= 21 - r).any():
            pytest.skip("a single-system cell below level 21 - r is split")
        np.testing.assert_array_equal(rb.acc[a:b], rs.acc)
        sel = sys_of == s
        np.testing.assert_array_equal(rb.gentries[sel], rs.gentries)
        np.testing.assert_array_equal(rb.grp.count[sel], rs.grp.count)
