"""GPU parity of the second-order Runge-Kutta integrator (predict / correct,
Heun's method; nbody_state.integrator = 1) through the C ABI.

The HIP path steps one context without reloading its state; before each
step the test copies the GPU's state and the oracle takes the same step from
it. The oracle is fed the GPU's predicted-position accelerations a_p
(NBODY_X_APRED) for the correction and as the a_old of the second force
evaluation, so both sides take the same decisions after it. Checked per step:
positions and velocities bit for bit (their arithmetic sees identical
inputs), the kept tree's sorted keys, the GPU's a_p against the oracle's
tree at the predicted positions and the new accelerations against the
oracle's tree at the corrected positions (both under the tree-parity rule),
and the second walk's list lengths and entry hashes exactly."""
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
    return f(st.x, st.y, st.z), f(st.vx, st.vy, st.vz), f(st.ax, st.ay, st.az)


def _rule(orc, got, ref, pos32, m, eps):
    _, A = orc.direct(pos32.astype(np.float64), m, eps=eps, want_aabs=True)
    d = np.linalg.norm(got.astype(np.float64) - ref, axis=1)
    et, e = d / A, d / np.linalg.norm(ref, axis=1)
    assert et.max() <= TOL, et.max()
    assert np.percentile(e, 99.9) <= TOL, np.percentile(e, 99.9)
    return et.max()


@pytest.mark.parametrize("model,n,seed,dt,interval", [("plummer", 6000, 31, 2.0 ** -6, 2),
                                                       ("galaxy", 12000, 32, 2.0 ** -7, 1)])
def test_rk2_steps_match_oracle(nb, torch, orc, model, n, seed, dt, interval):
    _say("rk2", model, n, dt, interval)
    p = I.plummer(n, seed) if model == "plummer" else I.galaxy(n, seed)
    m = p.mass.astype(np.float32)
    eps, dacc = 2.0 ** -7, 2.0 ** -9
    params = nb.Params(eps=eps, delta_acc=dacc, checks=1)
    kw = dict(eps=eps, delta_acc=dacc, leaf_max=params.leaf_max, group_max=params.group_max,
              group_merge=params.group_merge)
    st = nb.State.from_numpy(p.pos, p.vel, p.mass, dt=dt, rebuild_interval=interval,
                             integrator=1)
    ctx = nb.Context(params, n_max=n)
    ctx.step(st, 0)  # first force evaluation
    ctx.sync()
    topo = p.pos.astype(np.float32)
    rebuilds = ctx.stats()["rebuilds"]
    for s in range(4):
        X, V, A = _get(st)
        ctx.step(st, 1)
        ctx.sync()
        stats = ctx.stats()
        rebuilt = stats["rebuilds"] > rebuilds
        rebuilds = stats["rebuilds"]
        ap_gpu = ctx.export(nb.X.APRED).cpu().numpy().reshape(3, n).T.copy()
        calls = []

        def force(p32, a_old):
            nonlocal topo
            if rebuilt and not calls:
                topo = p32.copy()  # the rebuild is at the predicted positions
            r = orc.tree_forces(*p32.T, m, a_old=a_old, topo=tuple(topo.T), **kw)
            calls.append((p32.copy(), r))
            return r.acc.astype(np.float32)

        Xo, Vo, Ao, _ = orc.rk2_step(X, V, A, dt, force, a_pred_in=ap_gpu)
        gx, gv, ga = _get(st)
        _say("  step %d rebuilt %s" % (s, rebuilt))
        np.testing.assert_array_equal(gx, Xo)
        np.testing.assert_array_equal(gv, Vo)
        (xp32, r1), (xn32, r2) = calls
        np.testing.assert_array_equal(ctx.export(nb.X.KEYS).cpu().numpy(), r2.keys_sorted)
        e1 = _rule(orc, ap_gpu, r1.acc, xp32, m, eps)
        e2 = _rule(orc, ga, r2.acc, xn32, m, eps)
        np.testing.assert_array_equal(ctx.export(nb.X.GENTRIES).cpu().numpy().astype(np.int64),
                                      r2.gentries)
        np.testing.assert_array_equal(ctx.export(nb.X.GHASH).cpu().numpy(), r2.ghash)
        _say("    max e~ predicted %.3g corrected %.3g" % (e1, e2))
    assert st.t == 4 * dt


def test_rk2_rejects_block_steps_and_graphs(nb, torch):
    p = I.plummer(512, 3)
    ctx = nb.Context(nb.Params(), n_max=512)
    st = nb.State.from_numpy(p.pos, p.vel, p.mass, block_steps=True, integrator=1)
    with pytest.raises(nb.NbodyError) as ei:
        ctx.step(st, 1)
    assert ei.value.code == nb.NBODY_EINVAL
    st2 = nb.State.from_numpy(p.pos, p.vel, p.mass, rebuild_interval=1, integrator=1)
    with pytest.raises(nb.NbodyError):
        ctx.step_graph(st2, 1)
    st3 = nb.State.from_numpy(p.pos, p.vel, p.mass, integrator=2)
    with pytest.raises(nb.NbodyError):
        ctx.step(st3, 1)
