"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bit-exact: Morton keys, sort permutation, cell table, FP64 and FP32 moments,
group table and boxes, per-group interaction-list lengths and entry hashes
(every MAC decision). Toleranced: accelerations, under the rule
  max_i |da_i| / A_i <= 1e-5  and  99.9th percentile of |da_i| / |a_i| <= 1e-5
with A_i = sum_j G m_j |r_ij| / (r_ij^2 + eps^2)^(3/2) (the conditioning of
the sum: FP32 cannot give a per-particle relative bound where |a_i| << A_i).
"""
import math
import sys

import numpy as np
import pytest

import nbody_inputs as I

pytestmark = pytest.mark.gpu

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


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


def _run(nb, torch, x, y, z, m, params, a_old=None, n_max=None):
    params.checks = 1  # record per-group entry hashes
    ctx = nb.Context(params, n_max=n_max or len(x))
    X, Y, Z, M = (_dev(torch, a.astype(np.float32)) for a in (x, y, z, m))
    ctx.build_tree(X, Y, Z, M)
    ao = None if a_old is None else tuple(_dev(torch, a_old[:, k].astype(np.float32)) for k in range(3))
    acc = ctx.calc_acc(ao)
    ctx.sync()
    return ctx, np.stack([_np(a) for a in acc], 1)


def _ref(orc, x, y, z, m, params, a_old=None):
    """The oracle's tree forces under the same parameters as the HIP call."""
    return orc.tree_forces(x, y, z, m, a_old=a_old, eps=params.eps,
                           delta_acc=params.delta_acc, leaf_max=params.leaf_max,
                           group_max=params.group_max, group_merge=params.group_merge)


def _compare_tree(nb, ctx, ref, torch):
    keys = _np(ctx.export(nb.X.KEYS))
    perm = _np(ctx.export(nb.X.PERM)).astype(np.int64)
    np.testing.assert_array_equal(keys, ref.keys_sorted)
    np.testing.assert_array_equal(perm, ref.perm)
    box = _np(ctx.export(nb.X.BOX))
    np.testing.assert_array_equal(box, ref.box)
    st = ctx.stats()
    assert st["ncell"] == ref.cells.n
    assert st["ngroup"] == ref.grp.n
    c = ref.cells
    np.testing.assert_array_equal(_np(ctx.export(nb.X.LEVEL)), c.level)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.PBEGIN)), c.pbegin)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.PCOUNT)), c.pcount)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.FCHILD)), c.first_child)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.NCHILD)), c.n_child)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.PARENT)), c.parent)
    node = _np(ctx.export(nb.X.NODE)).reshape(-1, 4)
    mq = _np(ctx.export(nb.X.MQ)).reshape(-1, 2)
    mom = _np(ctx.export(nb.X.MOM64)).reshape(-1, 4)
    np.testing.assert_array_equal(mom[:, 0], ref.mom.M)
    np.testing.assert_array_equal(mom[:, 1:], ref.mom.S)
    np.testing.assert_array_equal(node[:, :3], ref.mom.com)
    np.testing.assert_array_equal(node[:, 3], ref.mom.b2)
    np.testing.assert_array_equal(mq[:, 0], ref.mom.m32)
    np.testing.assert_array_equal(mq[:, 1], ref.mom.q)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.GBEGIN)), ref.grp.begin)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.GCOUNT)), ref.grp.count)


def _compare_walk(nb, ctx, ref, acc_gpu, pos, m, eps, G=1.0, check_bounds=True):
    gbox = _np(ctx.export(nb.X.GBOX)).reshape(-1, 8)
    if check_bounds:
        np.testing.assert_array_equal(gbox[:, 0:3], ref.glo)
        np.testing.assert_array_equal(gbox[:, 4:7], ref.ghi)
        np.testing.assert_array_equal(gbox[:, 3], ref.gdA)
        np.testing.assert_array_equal(gbox[:, 7], ref.gamin)
    ent = _np(ctx.export(nb.X.GENTRIES)).astype(np.int64)
    gh = _np(ctx.export(nb.X.GHASH))
    np.testing.assert_array_equal(ent, ref.gentries)
    np.testing.assert_array_equal(gh, ref.ghash)
    return acc_errors(ref.acc, acc_gpu, pos, m, eps, G)


def acc_errors(a_ref, a_gpu, pos, m, eps, G=1.0, A=None):
    import oracle

    if A is None:
        _, A = oracle.direct(pos.astype(np.float32).astype(np.float64), m, eps=eps, G=G,
                             want_aabs=True)
    d = np.linalg.norm(a_gpu.astype(np.float64) - a_ref, axis=1)
    e = d / np.linalg.norm(a_ref, axis=1)
    et = d / A
    return e, et


def _assert_rule(e, et):
    assert et.max() <= TOL, et.max()
    assert np.percentile(e, 99.9) <= TOL, np.percentile(e, 99.9)


CASES = [
    ("plummer", 1 << 13, 1, 16, 64),
    ("galaxy", 40000, 3, 16, 64),
    ("plummer", 5000, 7, 8, 32),
    ("galaxy", 3001, 9, 4, 16),
    ("plummer", 777, 2, 1, 8),
    ("plummer", 40, 4, 16, 64),  # the root is the only group, and it is split
]


@pytest.mark.parametrize("merge", [0, 1])
@pytest.mark.parametrize("model,n,seed,leaf,gmax", CASES)
def test_tree_and_walk_parity(nb, torch, orc, model, n, seed, leaf, gmax, merge):
    # calcNode with one launch per level (merge 0) and with the persistent
    # grid-barrier launch (merge 1)
    _say("case", model, n, seed, leaf, gmax, merge)
    p = I.plummer(n, seed) if model == "plummer" else I.galaxy(n, seed)
    x, y, z, _, _, _, m = p.f32()
    eps = 2.0 ** -7
    params = nb.Params(eps=eps, delta_acc=2.0 ** -9, leaf_max=leaf, group_max=gmax,
                       group_merge=merge, calcnode_sync=1 + merge)
    # bootstrap pass (no a_old)
    ctx, acc0 = _run(nb, torch, x, y, z, m, params)
    ref0 = _ref(orc, x, y, z, m, params)
    _compare_tree(nb, ctx, ref0, torch)
    e, et = _compare_walk(nb, ctx, ref0, acc0, np.stack([x, y, z], 1), m, eps)
    _assert_rule(e, et)
    # MAC pass with a_old = the oracle's bootstrap acceleration (FP32)
    a_old = ref0.acc.astype(np.float32)
    ctx1, acc1 = _run(nb, torch, x, y, z, m, params, a_old=a_old)
    ref1 = _ref(orc, x, y, z, m, params, a_old)
    e, et = _compare_walk(nb, ctx1, ref1, acc1, np.stack([x, y, z], 1), m, eps)
    _say("  max e~ %.3g  p99.9 e %.3g  entries %d" % (et.max(), np.percentile(e, 99.9),
                                                     ref1.gentries.sum()))
    _assert_rule(e, et)


@pytest.mark.parametrize("sync", [1, 2])
@pytest.mark.parametrize("n", [1, 2, 3, 17, 65, 257])
def test_tiny_and_ragged(nb, torch, orc, n, sync):
    _say("tiny", n, "calcnode_sync", sync)
    p = I.plummer(n, 100 + n)
    x, y, z, _, _, _, m = p.f32()
    params = nb.Params(leaf_max=4, group_max=16, calcnode_sync=sync)
    a_old = np.ones((n, 3), np.float32)
    ctx, acc = _run(nb, torch, x, y, z, m, params, a_old=a_old)
    ref = _ref(orc, x, y, z, m, params, a_old)
    _compare_tree(nb, ctx, ref, torch)
    if n > 1:
        e, et = _compare_walk(nb, ctx, ref, acc, np.stack([x, y, z], 1), m, 2.0 ** -7)
        _assert_rule(e, et)
    else:
        assert np.all(acc == 0)


def test_coincident_particles(nb, torch, orc):
    # 300 identical positions: level-21 leaves beyond leaf_max, groups cut
    # into pieces of group_max
    rng = np.random.default_rng(5)
    x = np.concatenate([np.full(300, 0.25), rng.uniform(-1, 1, 700)]).astype(np.float32)
    y = np.concatenate([np.full(300, -0.5), rng.uniform(-1, 1, 700)]).astype(np.float32)
    z = np.concatenate([np.full(300, 0.125), rng.uniform(-1, 1, 700)]).astype(np.float32)
    m = np.full(1000, 1e-3, np.float32)
    a_old = np.ones((1000, 3), np.float32)
    for merge, sync in ((0, 1), (1, 2), (1, 1)):
        params = nb.Params(leaf_max=8, group_max=32, group_merge=merge, calcnode_sync=sync)
        ctx, acc = _run(nb, torch, x, y, z, m, params, a_old=a_old)
        ref = _ref(orc, x, y, z, m, params, a_old)
        _compare_tree(nb, ctx, ref, torch)
        e, et = _compare_walk(nb, ctx, ref, acc, np.stack([x, y, z], 1), m, 2.0 ** -7)
        _assert_rule(e, et)


def test_zero_delta_equals_direct(nb, torch, orc):
    g = I.galaxy(6000, 11)
    x, y, z, _, _, _, m = g.f32()
    pos = np.stack([x, y, z], 1)
    ad, A = orc.direct(pos.astype(np.float64), m, want_aabs=True)
    params = nb.Params(delta_acc=0.0)
    ctx, acc = _run(nb, torch, x, y, z, m, params, a_old=ad.astype(np.float32))
    st = ctx.stats()
    assert st["interactions"] == 6000 * 6000
    e, et = acc_errors(ad, acc, pos, m, 2.0 ** -7, A=A)
    _assert_rule(e, et)
    # GPU direct kernel
    X, Y, Z, M = (_dev(torch, a) for a in (x, y, z, m))
    dd = np.stack([_np(t) for t in ctx.direct(X, Y, Z, M)], 1)
    e, et = acc_errors(ad, dd, pos, m, 2.0 ** -7, A=A)
    _assert_rule(e, et)


def test_results_independent_of_tile_waves_frontier_and_split(nb, torch, orc):
    # the walk's summation order is fixed by the group alone: list tile,
    # resident wavefronts, stack capacity (with its retry pass) and the number
    # of wavefronts sharing a group never change a bit
    g = I.galaxy(30000, 12)
    x, y, z, _, _, _, m = g.f32()
    a_old = _ref(orc, x, y, z, m, nb.Params()).acc.astype(np.float32)
    outs = []
    for tile, waves, fc, split in ((256, 8, 0, 1), (64, 4, 4096, 1), (2048, 16, 1 << 18, 2),
                                   (320, 12, 0, 4), (192, 32, 0, 0), (128, 32, 64, 4),
                                   (192, 32, 64, 2)):
        params = nb.Params(list_tile=tile, waves_per_cu=waves, frontier_cap=fc, walk_split=split)
        _, acc = _run(nb, torch, x, y, z, m, params, a_old=a_old)
        outs.append(acc)
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_compensated_sum_parity_and_not_worse(nb, torch, orc):
    """Both summations, plain and compensated (Neumaier), under the
    element-wise tree-parity rule against the oracle's tree; the compensated
    sum is also no worse in RMS relative error."""
    g = I.galaxy(20000, 13)
    x, y, z, _, _, _, m = g.f32()
    pos = np.stack([x, y, z], 1)
    a_old = _ref(orc, x, y, z, m, nb.Params()).acc.astype(np.float32)
    ref = _ref(orc, x, y, z, m, nb.Params(delta_acc=2.0 ** -16), a_old)
    _, A = orc.direct(pos.astype(np.float64), m, eps=nb.Params().eps, want_aabs=True)
    errs = []
    for comp in (0, 1):
        ctx, acc = _run(nb, torch, x, y, z, m,
                        nb.Params(delta_acc=2.0 ** -16, compensated=comp), a_old=a_old)
        np.testing.assert_array_equal(_np(ctx.export(nb.X.GENTRIES)).astype(np.int64),
                                      ref.gentries)
        d = np.linalg.norm(acc.astype(np.float64) - ref.acc, axis=1)
        e = d / np.linalg.norm(ref.acc, axis=1)
        _say("compensated %d: max e~ %.3g, p99.9 e %.3g, max e %.3g"
             % (comp, (d / A).max(), np.percentile(e, 99.9), e.max()))
        assert (d / A).max() <= TOL
        assert np.percentile(e, 99.9) <= TOL
        errs.append(e)
    _say("plain rms %.3g comp rms %.3g" % (np.sqrt((errs[0] ** 2).mean()),
                                          np.sqrt((errs[1] ** 2).mean())))
    assert np.sqrt((errs[1] ** 2).mean()) <= np.sqrt((errs[0] ** 2).mean())


def test_nonfinite_input_is_reported(nb, torch):
    x = np.zeros(100, np.float32)
    x[17] = np.nan
    y = np.linspace(0, 1, 100).astype(np.float32)
    ctx = nb.Context(nb.Params(), n_max=100)
    X, Y, M = _dev(torch, x), _dev(torch, y), _dev(torch, np.ones(100, np.float32))
    ctx.build_tree(X, Y, Y, M)
    with pytest.raises(nb.NbodyError) as ei:
        ctx.sync()
    assert ei.value.code == nb.NBODY_ENONFINITE
    # sticky: later calls fail with the same code
    with pytest.raises(nb.NbodyError):
        ctx.build_tree(Y, Y, Y, M)


def test_frontier_overflow_is_walked_again(nb, torch, orc):
    # delta_acc = 0 opens every cell: with a 64-cell frontier every group
    # overflows and is walked again by the retry pass; results bit-identical
    g = I.galaxy(20000, 14)
    x, y, z, _, _, _, m = g.f32()
    a_old = np.ones((20000, 3), np.float32)
    outs = []
    for fc in (64, 0):
        ctx, acc = _run(nb, torch, x, y, z, m, nb.Params(frontier_cap=fc, delta_acc=0.0),
                        a_old=a_old)
        st = ctx.stats()
        _say("frontier %d: retried %d of %d groups" % (fc, st["retried"], st["ngroup"]))
        if fc == 64:
            assert st["retried"] == st["ngroup"]
        else:
            assert st["retried"] == 0
        outs.append((acc, _np(ctx.export(nb.X.GENTRIES)), _np(ctx.export(nb.X.GHASH))))
    for u, v in zip(*outs):
        np.testing.assert_array_equal(u, v)
    ref = _ref(orc, x, y, z, m, nb.Params(delta_acc=0.0), a_old)
    np.testing.assert_array_equal(outs[0][1].astype(np.int64), ref.gentries)


def test_calc_before_build_and_workspace_limits(nb, torch):
    ctx = nb.Context(nb.Params(), n_max=1000)
    out = tuple(torch.empty(10, dtype=torch.float32, device="cuda") for _ in range(3))
    rc = nb.lib().nbody_calc_acc(ctx._h, None, None, None, *[nb._ptr(t) for t in out])
    assert rc == nb.NBODY_ENOTREE
    big = torch.zeros(2000, dtype=torch.float32, device="cuda")
    with pytest.raises(nb.NbodyError) as ei:
        ctx.build_tree(big, big, big, big)
    assert ei.value.code == nb.NBODY_ENOMEM


def test_kdk_step_matches_oracle(nb, torch, orc):
    p = I.plummer(4096, 21)
    eps, dt = 2.0 ** -7, 2.0 ** -7
    st = nb.State.from_numpy(p.pos, p.vel, p.mass, dt=dt, rebuild_interval=1)
    ctx = nb.Context(nb.Params(eps=eps), n_max=4096)
    ctx.step(st, 2)
    ctx.sync()
    m = p.mass.astype(np.float32)

    def force_tree(state={"a": None}):
        def f(p32):
            r = _ref(orc, p32[:, 0], p32[:, 1], p32[:, 2], m, nb.Params(eps=eps),
                     state["a"])
            state["a"] = r.acc.astype(np.float32)
            return state["a"]
        return f

    f = force_tree()
    x = p.pos.copy()
    a = f(x.astype(np.float32))  # bootstrap
    a = f(x.astype(np.float32))  # MAC pass with a_old
    v = p.vel.astype(np.float32)
    for _ in range(2):
        x, v, a = orc.kdk_step(x, v, a, m, dt, f)
    xg = np.stack([_np(st.x), _np(st.y), _np(st.z)], 1)
    vg = np.stack([_np(st.vx), _np(st.vy), _np(st.vz)], 1)
    # the GPU forces differ from the oracle's by FP32 rounding, and a_old
    # rounding can flip a few MAC decisions (a change of order delta_acc |a|)
    assert np.abs(xg - x).max() < 1e-6 * np.abs(x).max()
    assert np.abs(vg - v).max() < 1e-4 * np.abs(v).max()
    assert st.t == 2 * dt


def test_direct64_matches_oracle(nb, torch, orc):
    """The FP64 direct sum on the GPU (the accuracy reference of the tree
    walk) against the oracle's FP64 direct sum: only the summation order
    differs, so they agree to about 1e-13 relative."""
    g = I.galaxy(20000, 41)
    x, y, z, _, _, _, m = g.f32()
    rng = np.random.default_rng(8)
    tgt = np.concatenate([[0, 19999], rng.choice(20000, 700, replace=False)]).astype(np.int64)
    eps = 2.0 ** -6
    ctx = nb.Context(nb.Params(eps=eps), n_max=16)
    acc, aabs, phi = ctx.direct64(*(_dev(torch, a) for a in (x, y, z, m)), _dev(torch, tgt))
    ctx.sync()
    pos = np.stack([x, y, z], 1).astype(np.float64)
    ra, rA, rphi = orc.direct(pos, m, eps=eps, targets=tgt, want_aabs=True, want_phi=True)
    for got, ref in ((_np(acc), ra), (_np(aabs), rA), (_np(phi), rphi)):
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # an index outside [0, n) gives zeros
    bad = _dev(torch, np.array([3, 20000], np.int64))
    acc2, aabs2, phi2 = ctx.direct64(*(_dev(torch, a) for a in (x, y, z, m)), bad)
    ctx.sync()
    assert (_np(acc2)[1] == 0).all() and _np(aabs2)[1] == 0 and _np(phi2)[1] == 0
    r3 = orc.direct(pos, m, eps=eps, targets=np.array([3]))
    assert np.abs(_np(acc2)[0] - r3[0]).max() <= 1e-12 * np.abs(r3).max()


def test_potential_matches_oracle(nb, torch, orc):
    """nbody_calc_acc_pot: the potential from the same interaction lists
    against the oracle tree's FP64 potential (all terms share one sign, so
    the rule is a plain relative error per particle), accelerations
    bit-identical to nbody_calc_acc, lists exact."""
    g = I.galaxy(20000, 43)
    x, y, z, _, _, _, m = g.f32()
    eps = 2.0 ** -6
    params = nb.Params(eps=eps, checks=1)
    a_old = _ref(orc, x, y, z, m, params).acc.astype(np.float32)
    ref = _ref(orc, x, y, z, m, params, a_old)
    ctx, acc = _run(nb, torch, x, y, z, m, params, a_old=a_old)
    (ax, ay, az), phi = ctx.calc_acc_pot(tuple(_dev(torch, a_old[:, k]) for k in range(3)))
    ctx.sync()
    acc2 = np.stack([_np(ax), _np(ay), _np(az)], 1)
    np.testing.assert_array_equal(acc2, acc)
    np.testing.assert_array_equal(_np(ctx.export(nb.X.GENTRIES)).astype(np.int64),
                                  ref.gentries)
    rel = np.abs(_np(phi).astype(np.float64) - ref.phi) / np.abs(ref.phi)
    _say("potential: max rel %.3g" % rel.max())
    assert rel.max() <= TOL
    W = 0.5 * float((m * _np(phi)).sum())
    assert abs(W / (0.5 * float((m * ref.phi).sum())) - 1) < 1e-6
