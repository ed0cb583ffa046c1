"""Pins of the oracle's direct summation (Eq. 1, Sec. 1) against closed forms,
symmetry and Newton's third law."""
import math

import numpy as np
import pytest

import nbody_inputs as I


def test_two_body_closed_form(orc):
    # a_1 = G m_2 r_12 / (r_12^2 + eps^2)^(3/2), for several eps (incl. 0)
    pos = np.array([[0.3, -1.2, 2.0], [1.7, 0.4, -0.5]])
    m = np.array([0.25, 3.0])
    for eps in (0.0, 0.01, 0.5, 2.0):
        for G in (1.0, 6.674e-3):
            a = orc.direct(pos, m, G=G, eps=eps)
            r = pos[1] - pos[0]
            d = (r @ r + eps * eps) ** 1.5
            np.testing.assert_allclose(a[0], G * m[1] * r / d, rtol=1e-15, atol=0)
            np.testing.assert_allclose(a[1], -G * m[0] * r / d, rtol=1e-15, atol=0)


def test_cube_corners_closed_form(orc):
    # 8 equal masses on the corners of a cube of side s: each corner feels
    # 3 edge, 3 face-diagonal and 1 body-diagonal neighbours; per axis
    # a = G m s [1/(s^2+e^2)^1.5 + 2/(2s^2+e^2)^1.5 + 1/(3s^2+e^2)^1.5]
    # pointing to the centre.
    s, m, eps = 2.0, 0.125, 0.3
    c = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], float) * s
    a = orc.direct(c, np.full(8, m), eps=eps)
    mag = m * s * ((s * s + eps * eps) ** -1.5 + 2 * (2 * s * s + eps * eps) ** -1.5
                   + (3 * s * s + eps * eps) ** -1.5)
    expect = mag * np.sign(c.mean(0) - c)
    np.testing.assert_allclose(a, expect, rtol=1e-14, atol=1e-16)


def test_equilateral_triangle(orc):
    # three equal masses at unit distance: |a| = 2 cos(30 deg) G m / (1+eps^2)^1.5,
    # directed to the centroid
    h = math.sqrt(3) / 2
    p = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, h, 0.0]])
    eps = 0.1
    a = orc.direct(p, np.ones(3), eps=eps)
    cen = p.mean(0)
    for i in range(3):
        u = (cen - p[i]) / np.linalg.norm(cen - p[i])
        np.testing.assert_allclose(a[i], u * 2 * h / (1 + eps * eps) ** 1.5, rtol=1e-14,
                                   atol=1e-15)


def test_newton_third_law(orc):
    p = I.plummer(4096, 11)
    a = orc.direct(p.pos, p.mass)
    tot = (p.mass[:, None] * a).sum(0)
    scale = (p.mass * np.linalg.norm(a, axis=1)).sum()
    assert np.linalg.norm(tot) <= 1e-13 * scale


def test_targets_subset_and_aabs(orc):
    p = I.plummer(2048, 5)
    tg = I.random_subset(2048, 100, 5)
    a_all, A_all = orc.direct(p.pos, p.mass, want_aabs=True)
    a_sub, A_sub = orc.direct(p.pos, p.mass, targets=tg, want_aabs=True)
    np.testing.assert_array_equal(a_sub, a_all[tg])
    np.testing.assert_array_equal(A_sub, A_all[tg])
    assert np.all(A_all >= np.linalg.norm(a_all, axis=1) * (1 - 1e-12))


def test_plummer_potential_energy_and_profile(orc):
    # Plummer (G = M = a = 1): W = -3 pi / 32; mean radial acceleration at r is
    # -M(<r)/r^2 = -r/(1+r^2)^1.5 (softening 2^-7 is small against a = 1).
    n = 16384
    p = I.plummer(n, 1, mfrac_max=0.999)
    a, phi = orc.direct(p.pos, p.mass, eps=2.0 ** -7, want_phi=True)
    W = 0.5 * (p.mass * phi).sum()
    assert abs(W / (-3 * math.pi / 32) - 1) < 0.03
    r = np.linalg.norm(p.pos, axis=1)
    ar = (a * p.pos).sum(1) / r
    edges = np.array([0.3, 0.5, 0.8, 1.2, 2.0, 3.0])
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (r > lo) & (r < hi)
        rm = r[sel]
        pred = -(rm / (1 + rm * rm) ** 1.5)
        resid = ar[sel] - pred
        sem = resid.std() / math.sqrt(sel.sum())
        assert abs(resid.mean()) < 3 * sem + 0.02 * abs(pred.mean()), (lo, hi)


def test_virial_ratio_plummer(orc):
    p = I.plummer(8192, 2)
    _, phi = orc.direct(p.pos, p.mass, eps=2.0 ** -7, want_phi=True)
    W = 0.5 * (p.mass * phi).sum()
    K = 0.5 * (p.mass * (p.vel ** 2).sum(1)).sum()
    assert abs(2 * K / abs(W) - 1) < 0.06
