"""GPU parity of the multi-step path that the benchmark times: the tree kept
across steps (moments recomputed on the kept topology, the drift writing
positions straight into the key order), the acceleration mirror carried from
step to step and across rebuilds, and fixed or automatic rebuild intervals.

The HIP path steps one context without ever reloading its state. Before each
step the test copies the GPU's state and lets the oracle take the same step
from it, with the force of the oracle's tree whose keys, order, cells and
groups come from the positions at the GPU's last rebuild (its moments, group
boxes and forces from the current positions): the tree kept across steps of
Sec. 1 and 4.1 (topology rebuilt every few steps, calcNode every step).
Checked per step: positions bit for bit; inactive velocities, accelerations
and levels bit for bit; the sorted keys of the kept tree; the walked groups,
their list lengths and entry hashes exactly; accelerations of the active
particles under the tree-parity rule (max |da|/A <= 1e-5 and the 99.9th
percentile of |da|/|a| <= 1e-5); levels exactly except where |a| is within
1e-5 of a level threshold.

Block steps alternate the state's layout during a call (the tree's key
order, or the caller's arrays through the tree's permutation) from step to
step. A second context runs the same steps in ONE nbody_step call in key
order (the form the benchmark times) and must end bit-identical to the
step-by-step run.
"""
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


def _get(st):
    f = lambda *ts: np.stack([t.cpu().numpy() for t in ts], 1)  # noqa: E731
    return (f(st.x, st.y, st.z), f(st.vx, st.vy, st.vz), f(st.ax, st.ay, st.az),
            None if st.level is None else st.level.cpu().numpy())


def _near_threshold(a, dt, eta, eps, tol=1e-5):
    am = np.linalg.norm(a.astype(np.float64), axis=1)
    lim = np.sqrt(2 * eta * float(np.float32(eps)) / am)
    r = (dt / lim)[:, None] / 2.0 ** np.arange(11)[None, :]
    return (np.abs(r - 1) < tol).any(axis=1)


def _model(name, n, seed):
    return I.plummer(n, seed) if name == "plummer" else I.galaxy(n, seed)


CASES = [
    # model, n, seed, dt (dt_max for block steps), eps, steps, block
    ("galaxy", 20000, 6, 2.0 ** -3, 2.0 ** -6, 8, True),
    ("plummer", 6000, 5, 0.25, 2.0 ** -7, 6, True),
    ("plummer", 8192, 12, 2.0 ** -5, 2.0 ** -7, 6, False),
]


@pytest.mark.parametrize("interval", [3, 0])
@pytest.mark.parametrize("case", CASES, ids=["galaxy-block", "plummer-block", "plummer-kdk"])
def test_multistep_matches_oracle(nb, torch, orc, case, interval):
    model, n, seed, dt, eps, nsteps, block = case
    _say("multistep", model, n, "block" if block else "kdk", "interval", interval)
    p = _model(model, n, seed)
    m = p.mass.astype(np.float32)
    dacc, eta = 2.0 ** -9, 0.025
    params = nb.Params(eps=eps, delta_acc=dacc, checks=1)

    def tree(pos32, a_old, topo32):
        return orc.tree_forces(pos32[:, 0], pos32[:, 1], pos32[:, 2], m, a_old=a_old,
                               eps=eps, delta_acc=dacc, leaf_max=params.leaf_max,
                               group_max=params.group_max, group_merge=params.group_merge,
                               topo=(topo32[:, 0], topo32[:, 1], topo32[:, 2]))

    def fresh_state():
        return nb.State.from_numpy(p.pos, p.vel, p.mass, dt=dt, rebuild_interval=interval,
                                   block_steps=block, eta=eta)

    ctx = nb.Context(params, n_max=n)
    st = fresh_state()
    ctx.step(st, 0)  # the first force evaluation (bootstrap walk, then Eq. 2 walk)
    ctx.sync()
    topo = p.pos.astype(np.float32)  # the tree of the first evaluation
    rebuilds = ctx.stats()["rebuilds"]
    seen_rebuild = 0
    for s in range(nsteps):
        X, V, A, LV = _get(st)
        tick = st.tick
        # block steps alternate the state's layout (key order, caller order)
        ctx.set_step_layout(1 + s % 2)
        ctx.step(st, 1)
        ctx.sync()
        stats = ctx.stats()
        rebuilt = stats["rebuilds"] > rebuilds
        rebuilds = stats["rebuilds"]
        seen_rebuild += rebuilt
        last = {}

        def force(p32, a_old=None):
            nonlocal topo
            if rebuilt:
                topo = p32.copy()
            a_old = A if a_old is None else a_old
            last["r"] = tree(p32, a_old, topo)
            return last["r"].acc.astype(np.float32)

        if block:
            Xo, Vo, Ao, LVo, tick1, act = orc.block_step(X, V, A, LV, dt, tick, force, eta=eta,
                                                          eps=eps)
            assert st.tick == tick1
        else:
            Xo, Vo, Ao = orc.kdk_step(X, V, A, m, dt, force)
            act = np.ones(n, bool)
        gx, gv, ga, gl = _get(st)
        r = last["r"]
        _say("  step %d rebuilt %s active %d" % (s, rebuilt, act.sum()))
        np.testing.assert_array_equal(gx, Xo)
        np.testing.assert_array_equal(ctx.export(nb.X.KEYS).cpu().numpy(), r.keys_sorted)
        np.testing.assert_array_equal(gv[~act], Vo[~act])
        np.testing.assert_array_equal(ga[~act], Ao[~act])
        if block:
            q = ctx.export(nb.X.QUEUE).cpu().numpy()
            gact = np.array([act[r.perm[b:b + c]].any()
                             for b, c in zip(r.grp.begin, r.grp.count)])
            np.testing.assert_array_equal(q, np.flatnonzero(gact))
            assert stats["active"] == act.sum()
            bad = gl != LVo
            assert not (bad & ~act).any()
            if bad.any():
                assert _near_threshold(Ao[bad], dt, eta, eps).all(), np.flatnonzero(bad)
        else:
            q = np.arange(r.grp.n)
        gent = ctx.export(nb.X.GENTRIES).cpu().numpy().astype(np.int64)
        np.testing.assert_array_equal(gent[q], r.gentries[q])
        gh = ctx.export(nb.X.GHASH).cpu().numpy()
        np.testing.assert_array_equal(gh[q], r.ghash[q])
        _, Aabs = orc.direct(Xo.astype(np.float32).astype(np.float64), m, eps=eps,
                             want_aabs=True)
        d = np.linalg.norm(ga[act].astype(np.float64) - r.acc[act], axis=1)
        assert (d / Aabs[act]).max() <= TOL, (d / Aabs[act]).max()
        e = d / np.linalg.norm(r.acc[act], axis=1)
        assert np.percentile(e, 99.9) <= TOL, np.percentile(e, 99.9)
        dv = np.linalg.norm(gv[act] - Vo[act], axis=1)
        assert dv.max() <= 1e-5 * np.linalg.norm(Vo, axis=1).max()
    if interval:  # steps interval, 2 interval, ... (0-based) rebuild
        assert seen_rebuild == (nsteps - 1) // interval
    # the same steps in one call on a fresh context: bit-identical end state
    ctx2 = nb.Context(params, n_max=n)
    ctx2.set_step_layout(1)  # key order whatever the step count
    st2 = fresh_state()
    ctx2.step(st2, 0)
    ctx2.step(st2, nsteps)
    ctx2.sync()
    assert ctx2.stats()["rebuilds"] == rebuilds or interval == 0
    if interval:
        for a, b in zip(_get(st2), _get(st)):
            if a is not None:
                np.testing.assert_array_equal(a, b)
        assert st2.tick == st.tick and st2.t == st.t


def test_refit_matches_oracle_on_kept_topology(nb, torch, orc):
    """nbody_refit: moments, group boxes, lists and forces of new positions on
    the tree of old ones, against the oracle's tree of the old positions."""
    n = 30000
    g = I.galaxy(n, 21)
    rng = np.random.default_rng(3)
    p0 = g.pos.astype(np.float32)
    p1 = (g.pos + 2.0 ** -7 * g.vel + 1e-4 * rng.standard_normal((n, 3))).astype(np.float32)
    m = g.mass.astype(np.float32)
    eps, dacc = 2.0 ** -6, 2.0 ** -9
    params = nb.Params(eps=eps, delta_acc=dacc, checks=1)
    kw = dict(eps=eps, delta_acc=dacc, leaf_max=params.leaf_max, group_max=params.group_max,
              group_merge=params.group_merge)
    a_old = orc.tree_forces(*p1.T, m, a_old=None, **kw).acc.astype(np.float32)
    ref = orc.tree_forces(*p1.T, m, a_old=a_old, topo=tuple(p0.T), **kw)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")  # noqa: E731
    ctx = nb.Context(params, n_max=n)
    ctx.build_tree(*(dev(c) for c in p0.T), dev(m))
    ctx.refit(*(dev(c) for c in p1.T), dev(m))
    acc = ctx.calc_acc(tuple(dev(c) for c in a_old.T))
    ctx.sync()
    np.testing.assert_array_equal(ctx.export(nb.X.KEYS).cpu().numpy(), ref.keys_sorted)
    np.testing.assert_array_equal(ctx.export(nb.X.PERM).cpu().numpy().astype(np.int64), ref.perm)
    mom = ctx.export(nb.X.MOM64).cpu().numpy().reshape(-1, 4)
    np.testing.assert_array_equal(mom[:, 0], ref.mom.M)
    np.testing.assert_array_equal(mom[:, 1:], ref.mom.S)
    node = ctx.export(nb.X.NODE).cpu().numpy().reshape(-1, 4)
    np.testing.assert_array_equal(node[:, :3], ref.mom.com)
    np.testing.assert_array_equal(node[:, 3], ref.mom.b2)
    mq = ctx.export(nb.X.MQ).cpu().numpy().reshape(-1, 2)
    np.testing.assert_array_equal(mq[:, 0], ref.mom.m32)
    np.testing.assert_array_equal(mq[:, 1], ref.mom.q)
    box = ctx.export(nb.X.GBOX).cpu().numpy().reshape(-1, 8)
    np.testing.assert_array_equal(box[:, 0:3], ref.glo)
    np.testing.assert_array_equal(box[:, 4:7], ref.ghi)
    np.testing.assert_array_equal(box[:, 3], ref.gdA)
    np.testing.assert_array_equal(box[:, 7], ref.gamin)
    np.testing.assert_array_equal(ctx.export(nb.X.GENTRIES).cpu().numpy().astype(np.int64),
                                  ref.gentries)
    np.testing.assert_array_equal(ctx.export(nb.X.GHASH).cpu().numpy(), ref.ghash)
    got = np.stack([a.cpu().numpy() for a in acc], 1)
    _, Aabs = orc.direct(p1.astype(np.float64), m, eps=eps, want_aabs=True)
    d = np.linalg.norm(got.astype(np.float64) - ref.acc, axis=1)
    assert (d / Aabs).max() <= TOL
    assert np.percentile(d / np.linalg.norm(ref.acc, axis=1), 99.9) <= TOL
