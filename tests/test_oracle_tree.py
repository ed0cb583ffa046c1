"""Pins of the oracle's tree pieces: keys, sort, level-order octree, moments,
groups, the Eq. 2 acceptance test and the walk.

Independent references used here: hand-computed keys, geometric cell
membership (coordinates against cell midpoints, no keys), numpy's stable
argsort, a recursive geometric octree built from coordinates, brute-force
member maxima, Eq. 2 in its undivided FP64 form, and the direct sum."""
import numpy as np
import pytest

import nbody_inputs as I


# ------------------------------------------------------------------ keys
def test_keys_hand_computed(orc):
    # cube [0, 1]^3 (extent exactly 1 -> L = 1); the point at the upper corner
    # is clamped to q = 2^21 - 1 on every axis (key = 2^63 - 1).
    x = np.array([0, 1, 0.5, 0, 0, 0.25, 0.75, 0.5], np.float32)
    y = np.array([0, 1, 0, 0.5, 0, 0, 0.25, 0.5], np.float32)
    z = np.array([0, 1, 0, 0, 0.5, 0, 0.5, 0.5], np.float32)
    k, box = orc.keys(x, y, z)
    assert list(box) == [0.0, 0.0, 0.0, 1.0]
    assert k[0] == 0
    assert k[1] == (1 << 63) - 1
    assert k[2] == 1 << 62  # x half -> top bit of the x digit
    assert k[3] == 1 << 61
    assert k[4] == 1 << 60
    assert k[5] == 1 << 59  # x quarter -> x bit of the level-2 digit
    # (0.75, 0.25, 0.5): qx = 3*2^19, qy = 2^19, qz = 2^20
    # x bits 20,19 -> key bits 62,59; y bit 19 -> 58; z bit 20 -> 60
    assert k[6] == (1 << 62) | (1 << 59) | (1 << 58) | (1 << 60)
    assert k[7] == (1 << 62) | (1 << 61) | (1 << 60)


def test_root_cube_power_of_two(orc):
    x = np.array([-3.0, 2.5], np.float32)
    y = np.array([0.0, 0.1], np.float32)
    z = np.array([1.0, 1.0], np.float32)
    box = orc.root_cube(x, y, z)
    assert list(box) == [-3.0, 0.0, 1.0, 8.0]  # ext 5.5 -> L = 8
    box = orc.root_cube(np.array([0.0, 0.125], np.float32), np.zeros(2, np.float32),
                        np.zeros(2, np.float32))
    assert box[3] == 0.125  # exact power of two is kept
    box = orc.root_cube(np.ones(3, np.float32), np.ones(3, np.float32), np.ones(3, np.float32))
    assert box[3] == 1.0  # zero extent
    with pytest.raises(ValueError):
        orc.root_cube(np.array([0, np.nan], np.float32), np.zeros(2, np.float32),
                      np.zeros(2, np.float32))


def test_key_prefix_is_geometric_cell(orc):
    # two particles share the level-l key prefix iff they fall in the same
    # cell of a 2^l grid over the root cube (computed from coordinates)
    p = I.plummer(3000, 3)
    x, y, z = (p.pos[:, k].astype(np.float32) for k in range(3))
    k, box = orc.keys(x, y, z)
    lo, L = box[:3], box[3]
    rng = np.random.default_rng(0)
    ii = rng.integers(0, 3000, 4000)
    jj = np.concatenate([rng.integers(0, 3000, 3000), (ii[3000:] + 1) % 3000])
    P = np.stack([x, y, z], 1).astype(np.float64)
    for lvl in (1, 2, 3, 5, 8):
        cell = np.floor((P - lo) * (2.0 ** lvl / L)).astype(np.int64)
        cell = np.minimum(cell, 2 ** lvl - 1)
        same_geo = np.all(cell[ii] == cell[jj], axis=1)
        sh = np.uint64(63 - 3 * lvl)
        same_key = (k[ii] >> sh) == (k[jj] >> sh)
        np.testing.assert_array_equal(same_geo, same_key)
    # the top octal digit is the octant index 4*[x high] + 2*[y high] + [z high]
    half = (P - lo) >= L / 2
    top = (k >> np.uint64(60)).astype(np.int64)
    np.testing.assert_array_equal(top, 4 * half[:, 0] + 2 * half[:, 1] + half[:, 2])


def test_sort_is_stable_argsort(orc):
    rng = np.random.default_rng(1)
    k = rng.integers(0, 50, 5000).astype(np.uint64) << np.uint64(40)
    perm, ks = orc.sort(k)
    np.testing.assert_array_equal(perm, np.argsort(k, kind="stable"))
    np.testing.assert_array_equal(ks, np.sort(k))


# ------------------------------------------------------------------ tree
def _geometric_octree(P, lo, L, leaf_max):
    """Recursive octree from coordinates (no keys): children in octant order
    (x, then y, then z as the high, middle, low bit); returns level-order list
    of (level, sorted tuple of member caller indices)."""
    n = P.shape[0]
    out = []
    frontier = [(0, np.zeros(3), np.arange(n))]
    while frontier:
        nxt = []
        for lvl, org, mem in frontier:
            out.append((lvl, mem))
            if len(mem) > leaf_max and lvl < 21:
                h = L / 2.0 ** (lvl + 1)
                rel = P[mem] - lo - org
                bits = (rel >= h).astype(np.int64)
                octs = 4 * bits[:, 0] + 2 * bits[:, 1] + bits[:, 2]
                for o in range(8):
                    sel = mem[octs == o]
                    if len(sel):
                        off = np.array([(o >> 2) & 1, (o >> 1) & 1, o & 1]) * h
                        nxt.append((lvl + 1, org + off, sel))
        frontier = nxt
    # within a level, order by position of first member in key order is the
    # prefix order; the frontier order above already is the prefix order
    return out


@pytest.mark.parametrize("n,leaf_max,seed", [(1, 16, 0), (17, 16, 1), (200, 4, 2),
                                             (512, 16, 3), (512, 1, 4), (300, 8, 5)])
def test_build_matches_geometric_octree(orc, n, leaf_max, seed):
    p = I.plummer(n, seed)
    x, y, z = (p.pos[:, k].astype(np.float32) for k in range(3))
    k, box = orc.keys(x, y, z)
    perm, ks = orc.sort(k)
    cells = orc.build_tree(ks, leaf_max)
    P = np.stack([x, y, z], 1).astype(np.float64)
    ref = _geometric_octree(P, box[:3], box[3], leaf_max)
    assert cells.n == len(ref)
    for c, (lvl, mem) in enumerate(ref):
        assert cells.level[c] == lvl
        got = np.sort(perm[cells.pbegin[c]:cells.pbegin[c] + cells.pcount[c]])
        np.testing.assert_array_equal(got, np.sort(mem))


def _check_tree_invariants(cells, n, leaf_max):
    assert cells.pbegin[0] == 0 and cells.pcount[0] == n and cells.parent[0] == -1
    assert np.all(np.diff(cells.level) >= 0)  # level order
    for c in range(cells.n):
        if cells.n_child[c]:
            f, e = cells.first_child[c], cells.first_child[c] + cells.n_child[c]
            assert cells.pcount[c] > leaf_max and cells.level[c] < 21
            assert np.all(cells.parent[f:e] == c)
            assert np.all(cells.level[f:e] == cells.level[c] + 1)
            assert cells.pbegin[f] == cells.pbegin[c]
            ends = cells.pbegin[f:e] + cells.pcount[f:e]
            np.testing.assert_array_equal(cells.pbegin[f + 1:e], ends[:-1])
            assert ends[-1] == cells.pbegin[c] + cells.pcount[c]
            assert 1 <= cells.n_child[c] <= 8
        else:
            assert cells.pcount[c] <= leaf_max or cells.level[c] == 21


def test_tree_invariants_galaxy(orc):
    g = I.galaxy(20000, 3)
    x, y, z = (g.pos[:, k].astype(np.float32) for k in range(3))
    k, _ = orc.keys(x, y, z)
    perm, ks = orc.sort(k)
    for lm in (1, 8, 16):
        _check_tree_invariants(orc.build_tree(ks, lm), 20000, lm)


def test_tree_coincident_particles(orc):
    # 100 identical positions plus a few others: level-21 leaves exceed leaf_max
    x = np.concatenate([np.full(100, 0.3), [0.0, 1.0, 0.7]]).astype(np.float32)
    y = np.concatenate([np.full(100, 0.6), [0.0, 1.0, 0.1]]).astype(np.float32)
    z = np.concatenate([np.full(100, 0.2), [0.0, 1.0, 0.9]]).astype(np.float32)
    k, _ = orc.keys(x, y, z)
    perm, ks = orc.sort(k)
    cells = orc.build_tree(ks, 16)
    _check_tree_invariants(cells, 103, 16)
    big = np.where(cells.pcount == 100)[0]
    assert cells.level[big[-1]] == 21 and cells.n_child[big[-1]] == 0
    grp = orc.groups(cells, 32)
    assert grp.count.max() <= 32 and grp.count.sum() == 103
    np.testing.assert_array_equal(grp.begin[1:], (grp.begin + grp.count)[:-1])


# --------------------------------------------------------------- moments
def test_moments_against_brute_force(orc):
    p = I.plummer(3000, 7)
    x, y, z, _, _, _, m = p.f32()
    m = np.full(3000, 2.0 ** -12, np.float32)  # exact sums
    k, _ = orc.keys(x, y, z)
    perm, ks = orc.sort(k)
    sx, sy, sz, sm = x[perm], y[perm], z[perm], m[perm]
    cells = orc.build_tree(ks, 8)
    mom = orc.moments(cells, sx, sy, sz, sm, G=1.0)
    P = np.stack([sx, sy, sz], 1).astype(np.float64)
    # root: exact total mass, centre of mass = FP64 system centre of mass
    assert mom.M[0] == 3000 * 2.0 ** -12
    com = (P * sm[:, None].astype(np.float64)).sum(0) / mom.M[0]
    np.testing.assert_allclose(mom.com[0], com.astype(np.float32), rtol=2e-7, atol=1e-9)
    for c in range(cells.n):
        b, e = cells.pbegin[c], cells.pbegin[c] + cells.pcount[c]
        # b^2 is the largest member distance^2 to the stored centre of mass
        d = P[b:e] - mom.com[c].astype(np.float64)
        d2 = (d * d).sum(1)
        assert np.all(d2 <= mom.b2[c] * (1 + 1e-6) + 1e-30)
        assert mom.b2[c] <= d2.max() * (1 + 1e-6) + 1e-30
        if e - b == 1:  # single particle: exact position, zero size
            assert np.all(mom.com[c] == P[b].astype(np.float32)) and mom.b2[c] == 0
        if e - b == 2:  # two equal masses: midpoint
            mid = 0.5 * (P[b] + P[b + 1])
            np.testing.assert_allclose(mom.com[c], mid, rtol=1e-7, atol=1e-9)
        assert abs(mom.M[c] - (e - b) * 2.0 ** -12) == 0
        assert mom.q[c] == np.float32(mom.m32[c]) * mom.b2[c]


# --------------------------------------------------------------- groups
def test_groups_definition(orc):
    g = I.galaxy(30000, 4)
    x, y, z = (g.pos[:, k].astype(np.float32) for k in range(3))
    k, _ = orc.keys(x, y, z)
    perm, ks = orc.sort(k)
    cells = orc.build_tree(ks, 16)
    for gmax in (16, 32, 64):
        grp = orc.groups(cells, gmax)
        assert grp.begin[0] == 0 and (grp.begin + grp.count)[-1] == 30000
        np.testing.assert_array_equal(grp.begin[1:], (grp.begin + grp.count)[:-1])
        assert grp.count.max() <= gmax and grp.count.min() >= 1
        # each group is a cell with count <= gmax whose parent has count > gmax
        for gi in range(grp.n):
            c = grp.cell[gi]
            assert cells.pbegin[c] == grp.begin[gi] and cells.pcount[c] == grp.count[gi]
            assert cells.pcount[c] <= gmax
            assert cells.parent[c] == -1 or cells.pcount[cells.parent[c]] > gmax
        # and every such cell is a group
        is_grp = (cells.pcount <= gmax) & ((cells.parent < 0) |
                                          (cells.pcount[np.maximum(cells.parent, 0)] > gmax))
        assert is_grp.sum() == grp.n


# ------------------------------------------------------------------ MAC
def test_mac_matches_eq2_undivided(orc):
    """accept <=> d > b and G m b^2 / d^4 <= dacc |a|  (Eq. 2), FP64 reference,
    for cases whose relative margin exceeds 1e-4."""
    rng = np.random.default_rng(3)
    n_ok = 0
    for _ in range(4000):
        lo = rng.uniform(-1, 1, 3).astype(np.float32)
        hi = (lo + rng.uniform(0, 0.5, 3)).astype(np.float32)
        com = rng.uniform(-4, 4, 3).astype(np.float32)
        b2 = np.float32(rng.uniform(0, 1) ** 2)
        m = np.float32(rng.uniform(0.01, 1))
        amin = np.float32(rng.uniform(0.05, 2))
        dacc = np.float32(2.0 ** -rng.integers(1, 12))
        dA = np.float32(dacc * amin)
        q = np.float32(m * b2)
        t = np.maximum(np.maximum(lo.astype(float) - com, com - hi.astype(float)), 0)
        d2 = float(t @ t)
        lhs = float(m) * float(b2) / d2 ** 2 if d2 > 0 else np.inf
        rhs = float(dacc) * float(amin)
        if d2 > 0 and abs(lhs / rhs - 1) < 1e-4:
            continue
        if abs(d2 - float(b2)) <= 1e-4 * max(d2, 1e-30):
            continue
        expect = (d2 > float(b2)) and (lhs <= rhs)
        assert orc.mac(lo, hi, dA, False, com, b2, q) == expect
        n_ok += 1
        # bootstrap: d > 2 b
        if abs(d2 - 4 * float(b2)) > 1e-4 * max(d2, 1e-30):
            assert orc.mac(lo, hi, dA, True, com, b2, q) == (d2 > 4 * float(b2))
    assert n_ok > 3000


def test_mac_inside_group_never_accepts(orc):
    lo = np.array([0, 0, 0], np.float32)
    hi = np.array([1, 1, 1], np.float32)
    # centre of mass inside the box: d = 0, never accepted (even b = 0)
    assert not orc.mac(lo, hi, 1e9, False, np.array([0.5, 0.5, 0.5]), 0.0, 0.0)
    assert not orc.mac(lo, hi, 1e9, True, np.array([0.5, 0.5, 0.5]), 0.0, 0.0)


# ------------------------------------------------------------------ walk
def _brute_entries(orc, tr, g, bootstrap):
    """Interaction list of group g by enumeration: a cell is an entry iff it is
    accepted and no ancestor is accepted; particles of leaves that are not
    accepted and have no accepted ancestor are entries."""
    cells, mom = tr.cells, tr.mom
    lo, hi, dA = tr.glo[g], tr.ghi[g], tr.gdA[g]
    acc = np.array([orc.mac(lo, hi, dA, bootstrap, mom.com[c], mom.b2[c], mom.q[c])
                    for c in range(cells.n)])
    blocked = np.zeros(cells.n, bool)  # some ancestor accepted
    for c in range(1, cells.n):
        pa = cells.parent[c]
        blocked[c] = blocked[pa] or acc[pa]
    ids = [c for c in range(cells.n) if acc[c] and not blocked[c]]
    for c in range(cells.n):
        if cells.n_child[c] == 0 and not acc[c] and not blocked[c]:
            ids += [(1 << 40) + s for s in range(cells.pbegin[c],
                                                  cells.pbegin[c] + cells.pcount[c])]
    return ids


@pytest.mark.parametrize("n,seed,boot", [(256, 1, True), (256, 2, False), (200, 3, False)])
def test_walk_entries_brute_force(orc, n, seed, boot):
    p = I.plummer(n, seed)
    x, y, z, _, _, _, m = p.f32()
    a_old = None if boot else orc.direct(p.pos.astype(np.float32), m).astype(np.float32)
    tr = orc.tree_forces(x, y, z, m, a_old=a_old, delta_acc=2.0 ** -4, leaf_max=4,
                         group_max=16)
    for g in range(tr.grp.n):
        ids = _brute_entries(orc, tr, g, boot)
        assert tr.gentries[g] == len(ids)
        h = sum(orc.mix64(i) for i in ids) % (1 << 64)
        assert int(tr.ghash[g]) == h
    # each member's acceleration is Eq. 1 over its group's entries (FP64)
    P = np.stack([x, y, z], 1).astype(np.float64)
    for g in (0, tr.grp.n // 2, tr.grp.n - 1):
        ids = _brute_entries(orc, tr, g, boot)
        src = np.array([P[tr.perm[i - (1 << 40)]] if i >= 1 << 40 else tr.mom.com[i]
                        for i in ids],
                       np.float64)
        ms = np.array([m[tr.perm[i - (1 << 40)]] if i >= 1 << 40 else tr.mom.m32[i]
                       for i in ids], np.float64)
        for s in range(tr.grp.begin[g], tr.grp.begin[g] + tr.grp.count[g]):
            d = src - P[tr.perm[s]]
            r2 = (d * d).sum(1) + 2.0 ** -14
            expect = (ms[:, None] * d / r2[:, None] ** 1.5).sum(0)
            np.testing.assert_allclose(tr.acc_sorted[s], expect, rtol=1e-12, atol=1e-14)


def test_walk_zero_delta_is_direct(orc):
    # delta_acc = 0 accepts only zero-size cells, so the list is every particle
    g = I.galaxy(3000, 9)
    x, y, z, _, _, _, m = g.f32()
    ad, phid = orc.direct(np.stack([x, y, z], 1), m, want_phi=True)
    tr = orc.tree_forces(x, y, z, m, a_old=ad, delta_acc=0.0)
    np.testing.assert_allclose(tr.acc, ad, rtol=1e-11, atol=1e-13)
    # the potential over the same lists leaves out each particle's own entry
    np.testing.assert_allclose(tr.phi, phid, rtol=1e-12)
    assert tr.interactions() == 3000 * 3000


def test_walk_potential_plummer_energy(orc):
    # the tree potential at delta_acc = 2^-9: W = sum m phi / 2 against the
    # Plummer model's -3 pi / 32 (G = M = a = 1; softening 2^-7 and the
    # truncation at u <= 0.999 move it by well under 1 %), and per particle
    # within the walk's error of the direct potential
    p = I.plummer(1 << 14, 21)
    x, y, z, _, _, _, m = p.f32()
    ad, phid = orc.direct(np.stack([x, y, z], 1), m, want_phi=True)
    tr = orc.tree_forces(x, y, z, m, a_old=ad.astype(np.float32), delta_acc=2.0 ** -9)
    W = 0.5 * float((m * tr.phi).sum())
    assert abs(W / (-3 * np.pi / 32) - 1) < 0.02, W
    assert np.abs(tr.phi / phid - 1).max() < 2e-3
    assert (tr.phi < 0).all()


def test_walk_monotone_and_converging(orc):
    p = I.plummer(4096, 4)
    x, y, z, _, _, _, m = p.f32()
    ad = orc.direct(np.stack([x, y, z], 1), m)
    prev_n, prev_e = None, None
    for k in (1, 3, 5, 7, 9, 12, 16, 20):
        tr = orc.tree_forces(x, y, z, m, a_old=ad.astype(np.float32), delta_acc=2.0 ** -k)
        e = np.linalg.norm(tr.acc - ad, axis=1) / np.linalg.norm(ad, axis=1)
        e99 = np.percentile(e, 99)
        if prev_n is not None:
            assert tr.interactions() >= prev_n
            assert e99 <= prev_e * 1.05
        prev_n, prev_e = tr.interactions(), e99
    assert prev_e < 2e-5  # 99th percentile at delta_acc = 2^-20
