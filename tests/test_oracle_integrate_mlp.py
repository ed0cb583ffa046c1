"""Pins of the oracle's leapfrog step (time reversal, second-order
convergence on a circular orbit) and of the MLP cost model's analytic
gradient (central finite differences)."""
import math

import numpy as np

import nbody_inputs as I


def _direct_force(orc, m, eps):
    def f(p32):
        return orc.direct(p32, m, eps=eps).astype(np.float32)
    return f


def test_kdk_time_reversal(orc):
    p = I.plummer(256, 3)
    m = p.mass.astype(np.float32)
    force = _direct_force(orc, m, 2.0 ** -5)
    x0 = p.pos.copy()
    v0 = p.vel.astype(np.float32)
    a0 = force(x0.astype(np.float32))
    x, v, a = x0, v0, a0
    for _ in range(16):
        x, v, a = orc.kdk_step(x, v, a, m, 2.0 ** -7, force)
    v = -v
    for _ in range(16):
        x, v, a = orc.kdk_step(x, v, a, m, 2.0 ** -7, force)
    assert np.abs(x - x0).max() < 1e-5 * np.abs(x0).max()
    assert np.abs(-v - v0).max() < 1e-4 * np.abs(v0).max()


def test_kdk_second_order_circular_orbit(orc):
    # two equal masses m = 1/2 on a circular orbit of separation 1 (G = 1,
    # eps -> tiny): angular speed w = 1, each body at radius 1/2, speed 1/2.
    eps = 1e-4
    m = np.array([0.5, 0.5], np.float32)
    force = _direct_force(orc, m, eps)
    T = 2 * math.pi / math.sqrt(1.0 / (1 + eps * eps) ** 1.5)
    errs = []
    for nstep in (64, 128, 256):
        dt = T / 4 / nstep
        x = np.array([[0.5, 0, 0], [-0.5, 0, 0]], np.float64)
        w = 1.0 / (1 + eps * eps) ** 0.75
        v = np.array([[0, 0.5 * w, 0], [0, -0.5 * w, 0]], np.float32)
        a = force(x.astype(np.float32))
        for _ in range(nstep):
            x, v, a = orc.kdk_step(x, v, a, m, dt, force)
        # after a quarter period body 0 sits at (0, 1/2)
        errs.append(np.linalg.norm(x[0] - np.array([0.0, 0.5, 0.0])))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, errs


def test_mlp_gradient_finite_differences(orc):
    H = 8
    rng = np.random.default_rng(0)
    npar = orc.mlp_nparams(H)
    assert npar == 8 + 4 * H + H + H * H + H + H + 1
    w = rng.normal(0, 0.5, npar)
    f = rng.normal(0, 1, (16, 4))
    t = rng.normal(0, 1, 16)
    loss, g = orc.mlp_grad(w, f, t, hidden=H)
    y = orc.mlp_forward(w, f, hidden=H)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-14
    h = 1e-6
    num = np.empty(npar)
    for k in range(npar):
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        num[k] = (orc.mlp_grad(wp, f, t, hidden=H)[0] - orc.mlp_grad(wm, f, t, hidden=H)[0]) / (2 * h)
    # the standardisation entries are constants (gradient 0); the rest match
    # central differences
    np.testing.assert_array_equal(g[:8], 0.0)
    np.testing.assert_allclose(g[8:], num[8:], rtol=1e-6, atol=1e-9)


def test_mlp_forward_special_case(orc):
    # all weights zero except the output bias: the network is the constant b3,
    # and the prediction is b3 plus the size-based estimate f0 + f3; with
    # W1 = 0 and b1 = atanh(0.5), every hidden unit of layer 1 is 0.5.
    H = 4
    npar = orc.mlp_nparams(H)
    w = np.zeros(npar)
    w[4:8] = 1.0  # identity standardisation
    w[-1] = 2.5
    f = np.random.default_rng(1).normal(size=(5, 4))
    skip = f[:, 0] + f[:, 3]
    np.testing.assert_array_equal(orc.mlp_forward(w, f, hidden=H), 2.5 + skip)
    o = 8
    w[o + 4 * H:o + 5 * H] = math.atanh(0.5)  # b1
    w[o + 5 * H:o + 5 * H + H * H] = 1.0  # W2 = ones -> layer 2 pre-activation = H * 0.5
    w[o + 5 * H + H * H + H:o + 5 * H + H * H + 2 * H] = 1.0  # W3 = ones
    y = orc.mlp_forward(w, f, hidden=H)
    np.testing.assert_allclose(y, 2.5 + H * math.tanh(H * 0.5) + skip, rtol=1e-14, atol=1e-14)


def test_mlp_standardisation(orc):
    # the standardised network equals the plain one on pre-standardised inputs
    H = 8
    rng = np.random.default_rng(3)
    f = rng.normal(5.0, 3.0, (40, 4))
    w = rng.normal(0, 0.5, orc.mlp_nparams(H))
    w = orc.mlp_standardize(w, f)
    np.testing.assert_allclose(w[:4], f.mean(0), rtol=1e-14)
    np.testing.assert_allclose(w[4:8], 1 / f.std(0), rtol=1e-14)
    z = (f - f.mean(0)) / f.std(0)
    w_id = w.copy()
    w_id[:4] = 0.0
    w_id[4:8] = 1.0
    # (the size-based term is added to the network's output from the raw inputs)
    np.testing.assert_allclose(orc.mlp_forward(w, f, hidden=H) - (f[:, 0] + f[:, 3]),
                               orc.mlp_forward(w_id, z, hidden=H) - (z[:, 0] + z[:, 3]),
                               rtol=1e-12, atol=1e-12)
