"""Pins of the oracle's individual block time steps and of a tree kept across
steps (topology from earlier positions, moments from the current ones).

Level rule: closed forms where every quantity is a power of two, and a
brute-force sqrt comparison away from ties. Step structure: one level held
for all particles equals kick-drift-kick leapfrog bit for bit; in a constant
field every particle lands exactly on the closed-form parabola at its own
step boundaries (all values dyadic, so exact)."""
import math

import numpy as np
import pytest

import nbody_inputs as I


def test_level_closed_form(orc):
    # 2 eta eps = 2^-9, dt_max = 2^-7, a = (2^p, 0, 0):
    # dt_k^4 a^2 <= 2^-18  <=>  k >= (p - 5) / 2
    eta, eps, dt = 2.0 ** -4, 2.0 ** -6, 2.0 ** -7
    ps = np.arange(-12, 32)
    a = np.zeros((len(ps), 3), np.float32)
    a[:, 0] = np.ldexp(1.0, ps)
    lev = orc.block_level(a, dt, eta, eps, 0)
    want = np.clip([-((5 - p) // 2) for p in ps], 0, 10)
    np.testing.assert_array_equal(lev, want)
    # the axis does not matter, a zero acceleration takes the lowest level
    lev_z = orc.block_level(a[:, ::-1].copy(), dt, eta, eps, 0)
    np.testing.assert_array_equal(lev_z, want)
    assert orc.block_level(np.zeros((1, 3), np.float32), dt, eta, eps, 0, 2, 9)[0] == 2


def test_level_brute_force(orc):
    rng = np.random.default_rng(3)
    a = (rng.standard_normal((4000, 3)) * np.exp(rng.uniform(-4, 9, (4000, 1)))).astype(np.float32)
    eta, eps, dt = 0.025, 2.0 ** -6, 2.0 ** -7
    lev = orc.block_level(a, dt, eta, eps, 0)
    for i in range(len(a)):
        am = math.sqrt(sum(float(c) ** 2 for c in a[i]))
        lim = math.sqrt(2 * eta * eps / am)
        ks = [k for k in range(11) if dt / 2 ** k <= lim]
        k = ks[0] if ks else 10
        # skip near-ties, where FP64 rounding of the two forms may differ
        if k > 0 and abs(dt / 2 ** (k - 1) / lim - 1) < 1e-12:
            continue
        if abs(dt / 2 ** k / lim - 1) < 1e-12:
            continue
        assert lev[i] == k, (i, lev[i], k)


@pytest.mark.parametrize("tick,k_align", [(0, 0), (1024, 0), (512, 1), (768, 2), (1, 10),
                                          (1024 + 96, 5)])
def test_level_alignment(orc, tick, k_align):
    a = np.zeros((1, 3), np.float32)  # wants level 0
    assert orc.block_level(a, 2.0 ** -7, 0.025, 2.0 ** -6, tick)[0] == k_align


def _direct_force(orc, m, eps):
    def f(p32, a_old):
        a = orc.direct(p32.astype(np.float64), m, eps=eps)
        return a.astype(np.float32)
    return f


def test_single_level_is_leapfrog(orc):
    p = I.plummer(64, 8)
    m = p.mass.astype(np.float32)
    eps, dt_max, k = 2.0 ** -7, 2.0 ** -7, 3
    f = _direct_force(orc, m, eps)
    x0 = p.pos.copy()
    v0 = p.vel.astype(np.float32)
    a0 = f(x0.astype(np.float32), None)
    xb, vb, ab = x0.copy(), v0.copy(), a0.copy()
    lev = np.full(64, k, np.int8)
    tick = 0
    xl, vl, al = x0.copy(), v0.copy(), a0.copy()
    for _ in range(5):
        xb, vb, ab, lev, tick, act = orc.block_step(xb, vb, ab, lev, dt_max, tick, f,
                                                    eta=0.025, eps=eps, level_min=k,
                                                    level_max=k)
        assert act.all()
        xl, vl, al = orc.kdk_step(xl, vl, al, m, dt_max / 2 ** k, lambda q: f(q, None))
        np.testing.assert_array_equal(xb, xl)
        np.testing.assert_array_equal(vb, vl)
        np.testing.assert_array_equal(ab, al)
    assert tick == 5 * 2 ** (10 - k)


def test_constant_field_two_levels(orc):
    # 2 eta eps = 2^-9 and dt_max = 2^-4: dt_k^4 a^2 <= 2^-18 gives level 0
    # for |a| = 2^-6 and level 1 for |a| = 2 (k >= (1 + p) / 2 with a = 2^p)
    dt = 2.0 ** -4
    eta, eps = 2.0 ** -4, 2.0 ** -6
    a = np.array([[2.0 ** -6, 0, 0], [0, 2.0, 0]], np.float32)
    lev = orc.block_level(a, dt, eta, eps, 0, 0, 1)
    np.testing.assert_array_equal(lev, [0, 1])
    x0 = np.array([[1.0, 2.0, -1.0], [0.5, -0.25, 4.0]])
    v0 = np.array([[0.5, -1.0, 0.25], [2.0, 0.125, -0.5]], np.float32)
    force = lambda p32, a_old: a  # noqa: E731  constant field per particle
    x, v, acc, tick = x0.copy(), v0.copy(), a.copy(), 0
    A, V = a.astype(np.float64), v0.astype(np.float64)
    seen = []
    for _ in range(2):
        x, v, acc, lev, tick, act = orc.block_step(x, v, acc, lev, dt, tick, force,
                                                   eta=eta, eps=eps, level_min=0,
                                                   level_max=1)
        np.testing.assert_array_equal(lev, [0, 1])
        seen.append(act.copy())
        if tick == 512:
            # particle 1 at its boundary lies on the parabola; particle 0
            # drifted with its half-kicked velocity (all values dyadic: exact)
            h = dt / 2
            np.testing.assert_array_equal(x[1], x0[1] + V[1] * h + A[1] * h * h / 2)
            np.testing.assert_array_equal(x[0], x0[0] + (V[0] + A[0] * dt / 2) * h)
    assert tick == 1024
    np.testing.assert_array_equal(seen[0], [False, True])
    np.testing.assert_array_equal(seen[1], [True, True])
    # a common boundary: both exactly on the parabola, v = v0 + a dt
    np.testing.assert_array_equal(x, x0 + V * dt + A * dt * dt / 2)
    np.testing.assert_array_equal(v, (V + A * dt).astype(np.float32))


def test_each_level_active_once_per_step(orc):
    rng = np.random.default_rng(9)
    n = 40
    lev0 = rng.integers(0, 6, n).astype(np.int8)
    lev0[0] = 5
    a = np.zeros((n, 3), np.float32)
    x, v = np.zeros((n, 3)), np.zeros((n, 3), np.float32)
    force = lambda p32, a_old: a  # noqa: E731
    count = np.zeros(n, int)
    tick = 0
    while tick < 1024:
        x, v, a, lev, tick, act = orc.block_step(x, v, a, lev0, 2.0 ** -7, tick, force,
                                                 eta=0.025, eps=2.0 ** -6, level_min=0,
                                                 level_max=5)
        count += act
    np.testing.assert_array_equal(count, 2 ** lev0.astype(int))


def test_kept_topology(orc):
    g = I.galaxy(3000, 17)
    x, y, z, vx, vy, vz, m = g.f32()
    dt = np.float32(2.0 ** -5)
    x1, y1, z1 = (x + vx * dt).astype(np.float32), (y + vy * dt).astype(np.float32), \
        (z + vz * dt).astype(np.float32)
    # topology from the same positions = a fresh tree
    a = orc.tree_forces(x1, y1, z1, m, a_old=None)
    b = orc.tree_forces(x1, y1, z1, m, a_old=None, topo=(x1, y1, z1))
    np.testing.assert_array_equal(a.acc, b.acc)
    np.testing.assert_array_equal(a.gentries, b.gentries)
    # topology from earlier positions: the groups still partition the particles,
    # b^2 still encloses every member, and delta_acc = 0 still gives direct
    c = orc.tree_forces(x1, y1, z1, m, a_old=np.ones((3000, 3), np.float32),
                        delta_acc=0.0, topo=(x, y, z))
    s = np.stack([x1, y1, z1], 1)[c.perm]
    cl = c.cells
    for j in range(cl.n):
        b0, nn = cl.pbegin[j], cl.pcount[j]
        d = (s[b0:b0 + nn] - c.mom.com[j]).astype(np.float64)
        r2 = (d * d).sum(axis=1)
        assert r2.max() <= c.mom.b2[j] * (1 + 1e-6)
    ad, A = orc.direct(np.stack([x1, y1, z1], 1).astype(np.float64), m, want_aabs=True)
    assert (np.linalg.norm(c.acc - ad, axis=1) / A).max() < 1e-12
