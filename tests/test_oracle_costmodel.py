"""Pins of the oracle's cost-model pieces: Adam against its closed form under a
constant gradient and on a quadratic, training that overfits a small set,
and the group features and target on hand-built groups."""
import numpy as np

import nbody_inputs as I


def test_adam_constant_gradient_closed_form(orc):
    # with a constant gradient the bias-corrected moments equal g and g^2, so
    # every step moves by lr g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 7.0])
    w = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr = 0.01
    for t in range(1, 6):
        w, m, v = orc.adam_step(w, g, m, v, t, lr)
        np.testing.assert_allclose(w, -t * lr * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_quadratic(orc):
    w = np.array([10.0])
    m = np.zeros(1)
    v = np.zeros(1)
    for t in range(1, 3001):
        g = 2.0 * (w - 3.0)
        w, m, v = orc.adam_step(w, g, m, v, t, 0.05)
    assert abs(w[0] - 3.0) < 1e-3


def test_mlp_overfits_small_set(orc):
    H = 16
    rng = np.random.default_rng(4)
    f = rng.standard_normal((16, 4))
    t = rng.standard_normal(16)
    w0 = I.mlp_init(orc.mlp_nparams(H), orc.mlp_fan_in(H), 1).astype(np.float64)
    _, losses = orc.mlp_train(w0, f, t, hidden=H, steps=1500, lr=1e-2)
    assert losses[-1] < 1e-3 * losses[0], (losses[0], losses[-1])


def test_fan_in_layout(orc):
    for H in (8, 32):
        fan = orc.mlp_fan_in(H)
        assert fan.shape == (orc.mlp_nparams(H),)
        assert fan[0] == 1 and fan[8] == 4 and fan[-1] == H


class _G:
    def __init__(self, begin, count):
        self.begin = np.asarray(begin)
        self.count = np.asarray(count)
        self.n = len(begin)


def test_features_hand_built(orc):
    sx = np.array([0.0, 2.0, 5.0], np.float32)
    sy = np.zeros(3, np.float32)
    sz = np.zeros(3, np.float32)
    sm = np.array([0.5, 0.5, 0.25], np.float32)
    prev = np.array([3.0, 5.0, 0.0])
    f = orc.cost_features(_G([0, 2], [2, 1]), sx, sy, sz, sm, prev)
    # group 0: two particles 2 apart -> h = 1, mass 1, mean previous length 4
    np.testing.assert_allclose(f[0], [1.0, np.log2(1 + 2.0 ** -40), -3 * np.log2(1 + 2.0 ** -40),
                                      np.log2(5.0)], rtol=0, atol=1e-15)
    # group 1: one particle -> h = 0, the floor 2^-40
    np.testing.assert_allclose(f[1], [0.0, -40.0, -2.0 + 120.0, 0.0], rtol=0, atol=1e-12)
    t = orc.cost_target(_G([0, 2], [2, 1]), np.array([16, 0]))
    np.testing.assert_array_equal(t, [5.0, 0.0])
