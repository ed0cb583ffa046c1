"""GPU parity at full size: the galaxy of 2^23 particles in the launch
configuration the benchmark times (eps 2^-6, delta_acc 2^-9, leaf 16, groups
of at most 64 with sibling joining, default tile, wavefronts and split).

Whole arrays, bit-exact against the oracle: sorted keys, permutation, cell
table, groups, group boxes / min |a_old| / delta_acc |a_old|, and for every
group (the oracle walks all of them) the list length and entry hash; forces
of every particle under the tree-parity rule. Block time steps at this
size: the walk split chosen by queue length gives the same bits as an
unsplit walk, step after step."""
import sys

import numpy as np
import pytest

import nbody_inputs as I

pytestmark = pytest.mark.gpu

N = 1 << 23
EPS, DACC = 2.0 ** -6, 2.0 ** -9
TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def nb(torch):
    import paper_1811_02761_amd as nb

    nb.lib()
    return nb


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def galaxy():
    return I.galaxy(N, 3)


def _walk(orc, pipe, sel, sa):
    """The oracle's walk of groups `sel` (bootstrap criterion when sa is None);
    returns sorted-order accelerations (only the members of sel set),
    per-group list lengths and entry hashes."""
    sx, sy, sz, sm, cells, mom, grp = pipe
    g = orc.Groups(grp.begin[sel], grp.count[sel], grp.cell[sel])
    lo, hi, _, dA = orc.group_bounds(g, sx, sy, sz, sa, DACC)
    n = sx.shape[0]
    ax, ay, az = (np.zeros(n) for _ in range(3))
    ent = np.empty(g.n, np.int64)
    gh = np.empty(g.n, np.uint64)
    orc.lib().orc_walk(n, sx, sy, sz, sm, cells.n, cells.pbegin, cells.pcount,
                       cells.first_child, cells.n_child, mom.m32,
                       np.ascontiguousarray(mom.com[:, 0]), np.ascontiguousarray(mom.com[:, 1]),
                       np.ascontiguousarray(mom.com[:, 2]), mom.b2, mom.q, g.n, g.begin, g.count,
                       np.ascontiguousarray(lo.reshape(-1)), np.ascontiguousarray(hi.reshape(-1)),
                       dA, None, int(sa is None), 1.0, EPS, ax, ay, az, None, ent, gh,
                       orc.nthreads_default())
    return np.stack([ax, ay, az], 1), ent, gh


def test_fullsize_tree_and_sampled_walk(nb, torch, orc, galaxy):
    x, y, z, _, _, _, m = galaxy.f32()
    _say("oracle pipeline, n = %d" % N)
    k, box = orc.keys(x, y, z)
    perm, ks = orc.sort(k)
    sx, sy, sz, sm = x[perm], y[perm], z[perm], m[perm]
    cells = orc.build_tree(ks, 16)
    mom = orc.moments(cells, sx, sy, sz, sm, 1.0)
    grp = orc.groups(cells, 64, 1)
    pipe = (sx, sy, sz, sm, cells, mom, grp)
    # a_old: the oracle's own bootstrap walk of every group, rounded to FP32
    _say("oracle bootstrap walk of %d groups" % grp.n)
    a0s, _, _ = _walk(orc, pipe, np.arange(grp.n), None)
    a0s = a0s.astype(np.float32)
    a_old = np.empty_like(a0s)
    a_old[perm] = a0s

    _say("GPU build + walk")
    ctx = nb.Context(nb.Params(eps=EPS, delta_acc=DACC, leaf_max=16, group_max=64, checks=1),
                     n_max=N)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")  # noqa: E731
    ctx.build_tree(dev(x), dev(y), dev(z), dev(m))
    acc = ctx.calc_acc(tuple(dev(a_old[:, j]) for j in range(3)))
    ctx.sync()
    a_gpu = np.stack([_np(t) for t in acc], 1)

    np.testing.assert_array_equal(_np(ctx.export(nb.X.KEYS)), ks)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.PERM)).astype(np.int64), perm)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.BOX)), box)
    st = ctx.stats()
    assert st["ncell"] == cells.n and st["ngroup"] == grp.n
    np.testing.assert_array_equal(_np(ctx.export(nb.X.LEVEL)), cells.level)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.PCOUNT)), cells.pcount)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.FCHILD)), cells.first_child)
    node = _np(ctx.export(nb.X.NODE)).reshape(-1, 4)
    mq = _np(ctx.export(nb.X.MQ)).reshape(-1, 2)
    np.testing.assert_array_equal(node[:, :3], mom.com)
    np.testing.assert_array_equal(node[:, 3], mom.b2)
    np.testing.assert_array_equal(mq[:, 0], mom.m32)
    np.testing.assert_array_equal(mq[:, 1], mom.q)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.GBEGIN)).astype(np.int64), grp.begin)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.GCOUNT)).astype(np.int64), grp.count)
    lo, hi, amin, dA = orc.group_bounds(grp, sx, sy, sz, a0s, DACC)
    gbox = _np(ctx.export(nb.X.GBOX)).reshape(-1, 8)
    np.testing.assert_array_equal(gbox[:, 0:3], lo)
    np.testing.assert_array_equal(gbox[:, 4:7], hi)
    np.testing.assert_array_equal(gbox[:, 3], dA)
    np.testing.assert_array_equal(gbox[:, 7], amin)

    # every group: the oracle walks all of them with the same a_old
    _say("oracle walk of all %d groups" % grp.n)
    a_ref_s, ent, gh = _walk(orc, pipe, np.arange(grp.n), a0s)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.GENTRIES)).astype(np.int64), ent)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.GHASH)), gh)
    a_ref = np.empty_like(a_ref_s)
    a_ref[perm] = a_ref_s
    d = np.linalg.norm(a_gpu.astype(np.float64) - a_ref, axis=1)
    e = d / np.linalg.norm(a_ref, axis=1)
    # |a_i| <= A_i, so e~_i <= e_i: the scale A_i (a direct sum over all N)
    # is needed only where e_i exceeds the bound, plus a random sample
    rng = np.random.default_rng(11)
    tgt = np.union1d(np.flatnonzero(e > TOL), rng.choice(N, size=4096, replace=False))
    pos = np.stack([x, y, z], 1).astype(np.float64)
    _, A = orc.direct(pos, m, eps=EPS, targets=tgt, want_aabs=True)
    et = d[tgt] / A
    _say("all %d particles: p99.9 e %.3g, max e %.3g; %d with e > 1e-5, max e~ there %.3g"
         % (N, np.percentile(e, 99.9), e.max(), int((e > TOL).sum()), et.max()))
    assert et.max() <= TOL and np.percentile(e, 99.9) <= TOL


def test_fullsize_block_steps_split_bit_identical(nb, torch, galaxy):
    # the benchmark's integration (block steps dt_max 2^-3, eta 0.025); block
    # steps walk short queues of heavy groups, which the automatic split
    # shares among 2 or 4 wavefronts
    states = []
    for split in (0, 1):
        ctx = nb.Context(nb.Params(eps=EPS, delta_acc=DACC, walk_split=split), n_max=N)
        st = nb.State.from_numpy(galaxy.pos, galaxy.vel, galaxy.mass, dt=2.0 ** -3,
                                 block_steps=True, eta=0.025)
        ctx.step(st, 12)
        ctx.sync()
        s = ctx.stats()
        _say("walk_split %d: %d walks, %d queued groups in all, tick %d"
             % (split, s["walk_calls"], s["queued_sum"], st.tick))
        states.append([_np(t) for t in (st.x, st.y, st.z, st.vx, st.vy, st.vz, st.ax, st.ay,
                                        st.az, st.level)])
        del ctx
    for u, v in zip(*states):
        np.testing.assert_array_equal(u, v)
