"""Pins of the joined i-groups: consecutive sibling group cells joined greedily
while the count stays within group_max. Checked against the cell table: a
partition in particle order, every group a run of consecutive siblings that
are group cells, and no group could absorb the next sibling group cell."""
import numpy as np
import pytest

import nbody_inputs as I


@pytest.mark.parametrize("n,seed,gmax", [(30000, 4, 64), (20000, 5, 32), (777, 6, 16)])
def test_merged_groups_definition(orc, n, seed, gmax):
    g = I.galaxy(n, seed)
    x, y, z = (g.pos[:, k].astype(np.float32) for k in range(3))
    k, _ = orc.keys(x, y, z)
    perm, ks = orc.sort(k)
    cells = orc.build_tree(ks, min(16, gmax))
    base = orc.groups(cells, gmax, 0)
    mg = orc.groups(cells, gmax, 1)
    # partition in particle order, sizes within bound
    assert mg.begin[0] == 0 and (mg.begin + mg.count)[-1] == n
    np.testing.assert_array_equal(mg.begin[1:], (mg.begin + mg.count)[:-1])
    assert mg.count.max() <= gmax
    # every joined group is a union of consecutive base groups with one parent
    starts = set(base.begin.tolist())
    bidx = {b: i for i, b in enumerate(base.begin.tolist())}
    par = cells.parent[base.cell]
    for gi in range(mg.n):
        b, e = mg.begin[gi], mg.begin[gi] + mg.count[gi]
        assert b in starts
        i = bidx[b]
        members = []
        while i < base.n and base.begin[i] < e:
            members.append(i)
            i += 1
        assert base.begin[members[-1]] + base.count[members[-1]] == e
        assert len({int(par[j]) for j in members}) == 1 or len(members) == 1
        # consecutive siblings: child indices increase by one
        cid = base.cell[members]
        assert np.all(np.diff(cid) == 1)
        # greedy maximality: the next base group, if it is the next sibling
        # group cell, did not fit
        if i < base.n and len(members) >= 1:
            nxt = i
            same_parent = par[nxt] == par[members[-1]] and base.cell[nxt] == cid[-1] + 1
            if same_parent and cells.pcount[base.cell[nxt]] <= gmax:
                assert mg.count[gi] + base.count[nxt] > gmax
    assert mg.n <= base.n
