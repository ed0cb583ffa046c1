"""Pins of the oracle's second-order Runge-Kutta step (Heun's predict /
correct form) against what the mathematics fixes, not against itself:

- a linear force a = -W x (anisotropic harmonic oscillator): one step of any
  two-stage second-order Runge-Kutta method on y' = J y is the Taylor
  polynomial I + hJ + (hJ)^2/2 of exp(hJ), written out here per component;
- a constant force: the step is exact (the parabola x + v t + a t^2/2);
- second-order convergence on a circular two-body orbit (error ratio 4 when
  the step halves), with the oracle's own direct sum as the force;
- the previous-acceleration input of each force evaluation (the a_old of
  Eq. 2): a for the predicted positions, a_p for the corrected ones."""
import math

import numpy as np


def test_rk2_linear_force_is_taylor_polynomial(orc):
    rng = np.random.default_rng(4)
    n = 50
    w2 = np.array([1.0, 2.5, 0.25], np.float64)  # omega^2 per axis
    x = rng.normal(size=(n, 3))
    v = rng.normal(size=(n, 3)).astype(np.float32)

    def force(p32, a_old):
        return (-(w2.astype(np.float32)) * p32).astype(np.float32)

    a = force(x.astype(np.float32), None)
    for h in (0.1, 0.03):
        xn, vn, an, ap = orc.rk2_step(x, v, a, h, force)
        X = x.astype(np.float32).astype(np.float64)  # the force sees FP32 positions
        V = v.astype(np.float64)
        x_ref = x + h * V - 0.5 * h * h * w2 * X
        v_ref = V - h * w2 * X - 0.5 * h * h * w2 * V
        assert np.abs(xn - x_ref).max() <= 1e-6 * np.abs(x).max(), np.abs(xn - x_ref).max()
        assert np.abs(vn - v_ref).max() <= 1e-6 * np.abs(V).max(), np.abs(vn - v_ref).max()
        # a' is the force at the corrected positions
        np.testing.assert_array_equal(an, force(xn.astype(np.float32), None))


def test_rk2_constant_force_is_exact(orc):
    g = np.array([0.5, -1.25, 2.0], np.float32)
    x = np.array([[1.0, 2.0, -3.0], [0.0, 0.0, 0.0]])
    v = np.array([[0.25, 0.5, -0.75], [1.0, -1.0, 0.5]], np.float32)

    def force(p32, a_old):
        return np.broadcast_to(g, p32.shape).astype(np.float32)

    a = force(x, None)
    h = 0.125  # powers of two: every product and sum below is exact
    xn, vn, _, _ = orc.rk2_step(x, v, a, h, force)
    np.testing.assert_array_equal(xn, x + v.astype(np.float64) * h + 0.5 * g * h * h)
    np.testing.assert_array_equal(vn, v + g * np.float32(h))


def test_rk2_second_order_circular_orbit(orc):
    eps = 1e-4
    m = np.array([0.5, 0.5], np.float32)

    def force(p32, a_old):
        return orc.direct(p32, m, eps=eps).astype(np.float32)

    T = 2 * math.pi / math.sqrt(1.0 / (1 + eps * eps) ** 1.5)
    errs = []
    for nstep in (64, 128, 256):
        dt = T / 4 / nstep
        x = np.array([[0.5, 0, 0], [-0.5, 0, 0]], np.float64)
        w = 1.0 / (1 + eps * eps) ** 0.75
        v = np.array([[0, 0.5 * w, 0], [0, -0.5 * w, 0]], np.float32)
        a = force(x.astype(np.float32), None)
        for _ in range(nstep):
            x, v, a, _ = orc.rk2_step(x, v, a, dt, force)
        errs.append(np.linalg.norm(x[0] - np.array([0.0, 0.5, 0.0])))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, errs


def test_rk2_previous_acceleration_inputs(orc):
    seen = []

    def force(p32, a_old):
        seen.append(np.array(a_old))
        return (-p32).astype(np.float32)

    x = np.array([[1.0, 0.0, 0.0]])
    v = np.array([[0.0, 1.0, 0.0]], np.float32)
    a = np.array([[-1.0, 0.0, 0.0]], np.float32)
    _, _, _, ap = orc.rk2_step(x, v, a, 0.1, force)
    np.testing.assert_array_equal(seen[0], a)
    np.testing.assert_array_equal(seen[1], ap)
    # a_p supplied from outside replaces the computed one in the correction
    fixed = np.array([[-2.0, 0.0, 0.0]], np.float32)
    _, vn, _, ap2 = orc.rk2_step(x, v, a, 0.1, force, a_pred_in=fixed)
    np.testing.assert_array_equal(ap2, fixed)
    np.testing.assert_array_equal(vn, v + ((a + fixed) * np.float32(0.05)).astype(np.float32))
