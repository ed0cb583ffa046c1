"""GPU parity of individual block time steps through the C ABI.

Each step starts the HIP path and the oracle from the same state (the
oracle's), so the comparison stays exact: positions (opening kicks and the
drift) and the velocities of inactive particles bit for bit, the set of
active particles and the walked groups exactly, the interaction lists of the
walked groups exactly, new levels exactly (a flip is accepted only where the
oracle's |a| lies within 1e-5 of a level threshold), accelerations of the
active particles under the tree-parity rule."""
import sys

import numpy as np
import pytest

import nbody_inputs as I

pytestmark = pytest.mark.gpu


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


def _load(torch, st, X, V, A, LV):
    for t, a in ((st.x, X[:, 0]), (st.y, X[:, 1]), (st.z, X[:, 2]), (st.vx, V[:, 0]),
                 (st.vy, V[:, 1]), (st.vz, V[:, 2]), (st.ax, A[:, 0]), (st.ay, A[:, 1]),
                 (st.az, A[:, 2]), (st.level, LV)):
        t.copy_(torch.as_tensor(np.ascontiguousarray(a)))


def _get(st):
    f = lambda *ts: np.stack([t.cpu().numpy() for t in ts], 1)  # noqa: E731
    return (f(st.x, st.y, st.z), f(st.vx, st.vy, st.vz), f(st.ax, st.ay, st.az),
            None if st.level is None else st.level.cpu().numpy())


def _near_threshold(a, dt, eta, eps, tol=1e-5):
    am = np.linalg.norm(a.astype(np.float64), axis=1)
    lim = np.sqrt(2 * eta * float(np.float32(eps)) / am)
    r = (dt / lim)[:, None] / 2.0 ** np.arange(11)[None, :]
    return (np.abs(r - 1) < tol).any(axis=1)


@pytest.mark.parametrize("model,n,dt", [("plummer", 4096, 0.25), ("galaxy", 20000, 2.0 ** -3)])
def test_block_steps_match_oracle(nb, torch, orc, model, n, dt):
    _say("block", model, n, dt)
    p = I.plummer(n, 5) if model == "plummer" else I.galaxy(n, 6)
    x, y, z, _, _, _, m = p.f32()
    eps, dacc, eta = 2.0 ** -7, 2.0 ** -9, 0.025
    params = nb.Params(eps=eps, delta_acc=dacc, checks=1)
    ref = lambda px, py, pz, ao: orc.tree_forces(  # noqa: E731
        px, py, pz, m, a_old=ao, eps=eps, delta_acc=dacc, leaf_max=params.leaf_max,
        group_max=params.group_max, group_merge=params.group_merge)
    a = ref(x, y, z, ref(x, y, z, None).acc.astype(np.float32)).acc.astype(np.float32)
    LV = orc.block_level(a, dt, eta, eps, 0)
    assert len(np.unique(LV)) >= 3, np.bincount(LV)
    X, V, A = p.pos.copy(), p.vel.astype(np.float32), a
    st = nb.State.from_numpy(X, V, p.mass, dt=dt, rebuild_interval=1, block_steps=True, eta=eta)
    st.have_acc = 1
    ctx = nb.Context(params, n_max=n)
    last = {}

    def force(p32, a_old):
        last["r"] = ref(p32[:, 0], p32[:, 1], p32[:, 2], a_old)
        return last["r"].acc.astype(np.float32)

    tick = 0
    for s in range(4):
        _load(torch, st, X, V, A, LV)
        st.tick = tick
        ctx.step(st, 1)
        X, V, A, LV, tick, act = orc.block_step(X, V, A, LV, dt, tick, force, eta=eta, eps=eps)
        gx, gv, ga, gl = _get(st)
        _say("  step %d tick %d active %d" % (s, tick, act.sum()))
        assert st.tick == tick
        np.testing.assert_array_equal(gx, X)
        np.testing.assert_array_equal(gv[~act], V[~act])
        np.testing.assert_array_equal(ga[~act], A[~act])
        bad = gl != LV
        assert not (bad & ~act).any()
        if bad.any():
            assert _near_threshold(A[bad], dt, eta, eps).all(), np.flatnonzero(bad)
        r = last["r"]
        stats = ctx.stats()
        assert stats["active"] == act.sum()
        q = ctx.export(nb.X.QUEUE).cpu().numpy()
        gact = np.array([act[r.perm[b:b + c]].any() for b, c in zip(r.grp.begin, r.grp.count)])
        np.testing.assert_array_equal(q, np.flatnonzero(gact))
        gent = ctx.export(nb.X.GENTRIES).cpu().numpy().astype(np.int64)
        np.testing.assert_array_equal(gent[q], r.gentries[q])
        gh = ctx.export(nb.X.GHASH).cpu().numpy()
        np.testing.assert_array_equal(gh[q], r.ghash[q])
        _, Aabs = orc.direct(X.astype(np.float32).astype(np.float64), m, eps=eps,
                             want_aabs=True)
        err = np.linalg.norm(ga[act] - A[act], axis=1) / Aabs[act]
        assert err.max() <= 1e-5, err.max()
        dv = np.linalg.norm(gv[act] - V[act], axis=1)
        assert dv.max() <= 1e-5 * np.linalg.norm(V, axis=1).max()


def test_single_level_block_equals_global_kdk(nb, torch):
    p = I.plummer(8192, 7)
    dt_max, k = 2.0 ** -4, 3
    ctx = nb.Context(nb.Params(), n_max=8192)
    sb = nb.State.from_numpy(p.pos, p.vel, p.mass, dt=dt_max, rebuild_interval=1,
                             block_steps=True, level_min=k, level_max=k)
    ctx.step(sb, 3)
    ctx2 = nb.Context(nb.Params(), n_max=8192)
    sg = nb.State.from_numpy(p.pos, p.vel, p.mass, dt=dt_max / 2 ** k, rebuild_interval=1)
    ctx2.step(sg, 3)
    ctx.sync()
    ctx2.sync()
    for a, b in zip(_get(sb)[:3], _get(sg)[:3]):
        np.testing.assert_array_equal(a, b)
    assert (sb.level.cpu().numpy() == k).all()
    assert sb.tick == 3 * 2 ** (10 - k)
    assert sb.t == sg.t == 3 * dt_max / 2 ** k


def test_block_steps_auto_rebuild_and_time(nb, torch):
    g = I.galaxy(50000, 8)
    ctx = nb.Context(nb.Params(eps=2.0 ** -6), n_max=50000)
    st = nb.State.from_numpy(g.pos, g.vel, g.mass, dt=2.0 ** -3, rebuild_interval=0,
                             block_steps=True)
    ctx.step(st, 12)
    ctx.sync()
    s = ctx.stats()
    assert s["steps"] == 12 and 0 < s["active"] <= 50000 and 0 < s["queued"] <= s["ngroup"]
    assert st.t == st.tick * st.dt / 1024
    lev = st.level.cpu().numpy()
    assert lev.min() >= 0 and lev.max() <= 10
    # every particle has a step boundary at or after the time reached
    assert np.isfinite(_get(st)[0]).all()


def test_bad_levels_are_reported(nb, torch):
    p = I.plummer(1000, 9)
    ctx = nb.Context(nb.Params(), n_max=1000)
    st = nb.State.from_numpy(p.pos, p.vel, p.mass, dt=2.0 ** -5, block_steps=True,
                             level_max=4)
    ctx.step(st, 1)
    ctx.sync()
    st.level[7] = 9  # beyond level_max
    with pytest.raises(nb.NbodyError) as ei:
        ctx.step(st, 1)
        ctx.sync()
    assert ei.value.code == nb.NBODY_ECORRUPT


def test_equal_keys_keep_caller_order_across_calls(nb, torch, orc):
    # Particles in identical pairs share one 63-bit key. Within one call the
    # block steps sort the state from the tree's previous key order (slot s
    # holds the caller index the tree's permutation names). After the caller
    # permutes its arrays between two calls, about half of the pairs reach
    # that sort in the opposite of caller order. The tree must still break
    # every tie by caller index, exactly as the oracle's stable sort does.
    n0 = 1500
    p = I.plummer(n0, 9)
    pos, vel, mass = (np.concatenate([a, a]) for a in (p.pos, p.vel, p.mass))
    n = 2 * n0
    params = nb.Params(eps=2.0 ** -7, delta_acc=2.0 ** -9)
    st = nb.State.from_numpy(pos, vel, mass, dt=2.0 ** -4, rebuild_interval=1,
                             block_steps=True, eta=0.025)
    ctx = nb.Context(params, n_max=n)
    ctx.set_step_layout(1)  # key order for these short calls too
    ctx.step(st, 2)
    ctx.sync()
    idx = torch.as_tensor(np.random.default_rng(4).permutation(n), device=st.x.device)
    for t in (st.x, st.y, st.z, st.vx, st.vy, st.vz, st.m, st.ax, st.ay, st.az, st.level):
        t.copy_(t[idx])
    ctx.step(st, 2)
    ctx.sync()
    x, y, z = (t.cpu().numpy().astype(np.float32) for t in (st.x, st.y, st.z))
    k, _ = orc.keys(x, y, z)
    perm, ks = orc.sort(k)
    # the twins stayed identical: every pair is still a tie
    assert int((ks[1:] == ks[:-1]).sum()) >= n0
    np.testing.assert_array_equal(ctx.export(nb.X.KEYS).cpu().numpy(), ks)
    np.testing.assert_array_equal(ctx.export(nb.X.PERM).cpu().numpy().astype(np.int64), perm)


def test_layouts_bit_identical(nb, torch):
    # the state kept in key order, or in the caller's arrays, during a call of
    # block steps: the same arithmetic, so the same bits (rebuild every 3rd
    # step: the automatic rule depends on timings). Between calls the caller
    # changes two values in place (a key-ordered context must notice and
    # gather again), then leaves the state alone (it may reuse its own copy).
    p = I.galaxy(20000, 8)
    params = nb.Params(eps=2.0 ** -7, delta_acc=2.0 ** -9)
    out = []
    for layout in (1, 2, 0):
        st = nb.State.from_numpy(p.pos, p.vel, p.mass, dt=2.0 ** -3, rebuild_interval=3,
                                 block_steps=True, eta=0.025)
        ctx = nb.Context(params, n_max=len(p.mass))
        ctx.set_step_layout(layout)
        ctx.step(st, 9)
        st.vx[17] += 2.0 ** -10
        st.ay[4321] *= 0.5
        ctx.step(st, 3)
        ctx.step(st, 8)
        ctx.sync()
        out.append(([t.cpu().numpy() for t in (st.x, st.y, st.z, st.vx, st.vy, st.vz, st.ax,
                                                st.ay, st.az, st.level)],
                    ctx.export(nb.X.PERM).cpu().numpy(), st.tick, ctx.stats()["rebuilds"]))
    for o in out[1:]:
        for a, b in zip(out[0][0], o[0]):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(out[0][1], o[1])
        assert out[0][2:] == o[2:]


@pytest.mark.parametrize("n", [1, 3, 63, 257, 1000])
def test_layouts_bit_identical_small_and_ragged(nb, torch, n):
    # the key-ordered layout moves the state in tiles of 256 particles (and
    # hashes it per workgroup): tiny and ragged counts in both layouts, bit
    # for bit, across two calls with an in-place change between them
    _say("step layouts, n", n)
    p = I.plummer(n, 300 + n)
    params = nb.Params(eps=2.0 ** -6, delta_acc=2.0 ** -9, leaf_max=4, group_max=16)
    out = []
    for layout in (1, 2):
        st = nb.State.from_numpy(p.pos, p.vel, p.mass, dt=2.0 ** -4, rebuild_interval=2,
                                 block_steps=True, eta=0.025)
        ctx = nb.Context(params, n_max=n)
        ctx.set_step_layout(layout)
        ctx.step(st, 5)
        st.vx[n - 1] += 2.0 ** -10
        ctx.step(st, 4)
        ctx.sync()
        out.append(([t.cpu().numpy() for t in (st.x, st.y, st.z, st.vx, st.vy, st.vz, st.ax,
                                                st.ay, st.az, st.level)],
                    ctx.export(nb.X.PERM).cpu().numpy(), st.tick))
    for a, b in zip(out[0][0], out[1][0]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]
    for a in out[0][0][:9]:
        assert np.all(np.isfinite(a))
