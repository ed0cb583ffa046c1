"""Seeded synthetic initial conditions shared by the oracle and the HIP path.

This module draws particle sets and nothing else: it holds none of the
arithmetic of the tree method (no keys, no tree, no forces). Every generator
uses numpy's counter-based Philox bit generator (Salmon et al. 2011,
"Parallel random numbers: as easy as 1, 2, 3") seeded by the caller, works in
float64 in the centre-of-mass frame, and uses units G = 1, total mass M = 1.

Models
------
* ``plummer``: Plummer (1911) sphere, positions and velocities by the
  Aarseth, Henon & Wielen (1974) recipe.
* ``king``: King (1966) model with dimensionless central potential W0,
  isotropic lowered-Maxwellian velocities.
* ``galaxy``: three-component disc galaxy standing in for the paper's M31
  model (Sec. 2.2): an NFW dark halo, a Hernquist bulge and an exponential
  disc with a sech^2 vertical profile. Scale ratios follow the M31 model of
  Sec. 2.2 (halo scale 7.63 kpc is the length unit; bulge 0.61 kpc; disc
  scale length 5.4 kpc); mass fractions and the disc thickness are those of
  the benchmark configuration (80 % halo, 5 % bulge, 15 % disc, z_d = 0.1 R_d).
  Velocities are isotropic Gaussians whose dispersion solves the spherical
  isotropic Jeans equation of each component in the total enclosed mass; the
  model is a realistic mass distribution, not an exact equilibrium.
* ``cluster_batch``: a batch of independent Plummer/King clusters with
  log-uniform particle numbers.

All particles of one system have equal mass m = M / N, as in the paper's
M31 runs (Sec. 2.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Particles",
    "rng_for",
    "plummer",
    "king",
    "galaxy",
    "cluster_batch",
    "random_subset",
    "uniform_cube",
]


@dataclass
class Particles:
    """Particle set in float64, caller order."""

    pos: np.ndarray  # (n, 3) float64
    vel: np.ndarray  # (n, 3) float64
    mass: np.ndarray  # (n,) float64
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])

    def f32(self):
        """Positions, velocities and masses rounded to float32 SoA columns."""
        p = self.pos.astype(np.float32)
        v = self.vel.astype(np.float32)
        return (np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
                np.ascontiguousarray(p[:, 2]), np.ascontiguousarray(v[:, 0]),
                np.ascontiguousarray(v[:, 1]), np.ascontiguousarray(v[:, 2]),
                self.mass.astype(np.float32))


def rng_for(seed: int, stream: int = 0) -> np.random.Generator:
    """Philox generator for (seed, stream); streams are independent keys."""
    return np.random.Generator(np.random.Philox(key=[int(seed), int(stream)]))


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], axis=1)


def _to_com_frame(pos, vel, mass):
    mt = mass.sum()
    pos = pos - (mass[:, None] * pos).sum(0) / mt
    vel = vel - (mass[:, None] * vel).sum(0) / mt
    return pos, vel


def plummer(n: int, seed: int, *, mass: float = 1.0, a: float = 1.0,
            mfrac_max: float = 0.999, G: float = 1.0) -> Particles:
    """Plummer sphere by the Aarseth-Henon-Wielen (1974) method.

    Radius from the enclosed-mass fraction u: r = a (u^(-2/3) - 1)^(-1/2),
    u uniform in (0, mfrac_max]. Speed v = q v_esc with
    v_esc = sqrt(2 G M / a) (1 + r^2/a^2)^(-1/4) and q drawn by rejection from
    g(q) = q^2 (1 - q^2)^(7/2).
    """
    n = int(n)
    rng = rng_for(seed, 0)
    u = rng.uniform(0.0, 1.0, n)
    u = (1.0 - u) * mfrac_max  # (0, mfrac_max]
    u = np.maximum(u, 1e-300)
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    pos = r[:, None] * _unit_vectors(rng, n)
    q = np.empty(n)
    filled = 0
    while filled < n:
        k = max(2 * (n - filled), 64)
        xq = rng.uniform(0.0, 1.0, k)
        yq = rng.uniform(0.0, 0.1, k)
        ok = xq[yq < xq * xq * (1.0 - xq * xq) ** 3.5]
        take = min(ok.size, n - filled)
        q[filled:filled + take] = ok[:take]
        filled += take
    vesc = math.sqrt(2.0 * G * mass / a) * (1.0 + (r / a) ** 2) ** (-0.25)
    vel = (q * vesc)[:, None] * _unit_vectors(rng, n)
    m = np.full(n, mass / n)
    pos, vel = _to_com_frame(pos, vel, m)
    return Particles(pos, vel, m, {"model": "plummer", "seed": seed, "a": a})


# ---------------------------------------------------------------- King (1966)
def _king_profile(W0: float, npts: int = 20000):
    """Integrate the King (1966) model in units G = 1, r_c = 9 sigma^2/(4 pi G rho0) = 1.

    Returns radius grid, W(r), rho(r)/rho0 and M(<r) up to the tidal radius
    where W = 0. The density of the lowered isothermal distribution is
    rho(W) ∝ e^W erf(sqrt W) - sqrt(4W/pi) (1 + 2W/3).
    """
    from scipy.integrate import solve_ivp
    from scipy.special import erf

    def rho_w(w):
        w = np.maximum(w, 0.0)
        sw = np.sqrt(w)
        return np.exp(w) * erf(sw) - np.sqrt(4.0 * w / np.pi) * (1.0 + 2.0 * w / 3.0)

    rho0 = rho_w(W0)
    # Poisson in King units: (1/r^2) d/dr (r^2 dW/dr) = -9 rho/rho0
    def rhs(r, s):
        w, dw = s
        return [dw, -9.0 * rho_w(w) / rho0 - 2.0 * dw / r]

    r0 = 1e-6
    s0 = [W0 - 1.5 * r0 * r0, -3.0 * r0]

    def tidal(r, s):
        return s[0]
    tidal.terminal = True
    tidal.direction = -1
    sol = solve_ivp(rhs, (r0, 1e4), s0, events=tidal, rtol=1e-10, atol=1e-12,
                    dense_output=True, max_step=0.05)
    rt = sol.t_events[0][0]
    rr = np.concatenate([[0.0], np.geomspace(r0, rt, npts)])
    w = np.concatenate([[W0], sol.sol(rr[1:])[0]])
    w[-1] = 0.0
    rho = rho_w(w) / rho0
    dm = 4.0 * np.pi * 0.5 * (rho[1:] * rr[1:] ** 2 + rho[:-1] * rr[:-1] ** 2) * np.diff(rr)
    mass = np.concatenate([[0.0], np.cumsum(dm)])
    return rr, w, rho, mass


def king(n: int, seed: int, *, W0: float = 6.0, mass: float = 1.0,
         scale: float = 1.0) -> Particles:
    """King (1966) model with central potential W0, scaled to total mass
    ``mass`` and core radius ``scale``; speeds by rejection from the lowered
    Maxwellian f(E) ∝ exp(W - v^2/2sigma^2) - 1 (v below the local escape speed).
    """
    n = int(n)
    rr, w, rho, mencl = _king_profile(W0)
    rng = rng_for(seed, 1)
    u = rng.uniform(0.0, mencl[-1], n)
    r = np.interp(u, mencl, rr)
    wr = np.interp(r, rr, w)
    pos = r[:, None] * _unit_vectors(rng, n)
    # speed in units of sigma: s = v/sigma with s^2/2 <= W; pdf ∝ s^2 (e^{W - s^2/2} - 1)
    spd = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        wt = np.maximum(wr[todo], 1e-12)
        smax = np.sqrt(2.0 * wt)
        s = rng.uniform(0.0, 1.0, todo.size) * smax
        f = s * s * (np.exp(wt - 0.5 * s * s) - 1.0)
        fmax = smax * smax * (np.exp(wt) - 1.0) + 1e-300
        ok = rng.uniform(0.0, 1.0, todo.size) * fmax < f
        spd[todo[ok]] = s[ok]
        todo = todo[~ok]
    # King units: G = 1, r_c = 1, sigma^2 = 4 pi rho0 / 9 with rho0 = 1
    sigma = math.sqrt(4.0 * math.pi / 9.0)
    vel = (spd * sigma)[:, None] * _unit_vectors(rng, n)
    # rescale to total mass `mass`, core radius `scale` (G = 1): v ∝ sqrt(M/R)
    mt = mencl[-1]
    pos = pos * scale
    vel = vel * math.sqrt(mass / mt / scale)
    m = np.full(n, mass / n)
    pos, vel = _to_com_frame(pos, vel, m)
    return Particles(pos, vel, m, {"model": "king", "seed": seed, "W0": W0})


# ---------------------------------------------------------- galaxy stand-in
def _inverse_cdf(cdf_x: np.ndarray, cdf_y: np.ndarray, u: np.ndarray) -> np.ndarray:
    return np.interp(u, cdf_y, cdf_x)


def galaxy(n: int, seed: int, *, f_halo: float = 0.80, f_bulge: float = 0.05,
           f_disk: float = 0.15, c_halo: float = 30.0,
           a_bulge: float = 0.61 / 7.63, r_bulge_max: float = 30.0,
           R_d: float = 5.4 / 7.63, zd_over_Rd: float = 0.1,
           R_max_over_Rd: float = 10.0) -> Particles:
    """Three-component galaxy (NFW halo + Hernquist bulge + exponential disc).

    Length unit: NFW scale radius. Total mass 1, all particles of mass 1/n.
    Component counts are round(f * n) with the disc taking the remainder.
    """
    n = int(n)
    rng = rng_for(seed, 2)
    n_h = int(round(f_halo * n))
    n_b = int(round(f_bulge * n))
    n_d = n - n_h - n_b
    if min(n_h, n_b, n_d) < 0:
        raise ValueError("bad fractions")
    # --- NFW halo, M(<x) ∝ ln(1+x) - x/(1+x), truncated at c_halo
    xg = np.concatenate([[0.0], np.geomspace(1e-6, c_halo, 200001)])
    mg = np.log1p(xg) - xg / (1.0 + xg)
    mg /= mg[-1]
    r_h = _inverse_cdf(xg, mg, rng.uniform(0.0, 1.0, n_h))
    pos_h = r_h[:, None] * _unit_vectors(rng, n_h)
    # --- Hernquist bulge, M(<r) ∝ r^2/(r+a)^2, truncated at r_bulge_max
    mt = (r_bulge_max / (r_bulge_max + a_bulge)) ** 2
    su = np.sqrt(rng.uniform(0.0, 1.0, n_b) * mt)
    r_b = a_bulge * su / (1.0 - su)
    pos_b = r_b[:, None] * _unit_vectors(rng, n_b)
    # --- exponential disc: Sigma ∝ exp(-R/R_d), R <= R_max; z from sech^2(z/z_d)
    Rg = np.linspace(0.0, R_max_over_Rd, 200001)
    cg = 1.0 - (1.0 + Rg) * np.exp(-Rg)
    cg /= cg[-1]
    R = R_d * _inverse_cdf(Rg, cg, rng.uniform(0.0, 1.0, n_d))
    phi = rng.uniform(0.0, 2.0 * np.pi, n_d)
    z_d = zd_over_Rd * R_d
    uz = rng.uniform(-1.0, 1.0, n_d) * (1.0 - 1e-12)
    zz = z_d * np.arctanh(uz)
    pos_d = np.stack([R * np.cos(phi), R * np.sin(phi), zz], axis=1)

    pos = np.concatenate([pos_h, pos_b, pos_d])
    comp = np.concatenate([np.zeros(n_h, np.int8), np.ones(n_b, np.int8),
                           np.full(n_d, 2, np.int8)])
    m = np.full(n, 1.0 / n)
    r_all = np.sqrt((pos * pos).sum(1))

    # --- isotropic Jeans dispersion per component in the total M(<r)
    edges = np.concatenate([[0.0], np.geomspace(1e-4, r_all.max() * 1.0001, 401)])
    rc = 0.5 * (edges[1:] + edges[:-1])
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    m_tot_cum = np.cumsum(np.histogram(r_all, edges)[0]) / n
    sig2 = np.zeros(n)
    for c in range(3):
        sel = comp == c
        if not sel.any():
            continue
        rho = np.histogram(r_all[sel], edges)[0] / n / shell
        integrand = rho * m_tot_cum / np.maximum(rc, 1e-12) ** 2 * np.diff(edges)
        tail = np.cumsum(integrand[::-1])[::-1]  # ∫_r^∞ rho M / r^2 dr
        s2 = np.where(rho > 0, tail / np.maximum(rho, 1e-300), 0.0)
        sig2[sel] = np.interp(r_all[sel], rc, s2)
    vel = np.sqrt(np.maximum(sig2, 0.0))[:, None] * rng.standard_normal((n, 3))
    perm = rng.permutation(n)  # mix components in caller order
    pos, vel, comp = pos[perm], vel[perm], comp[perm]
    pos, vel = _to_com_frame(pos, vel, m)
    return Particles(pos, vel, m, {"model": "galaxy", "seed": seed, "component": comp})


def cluster_batch(n_sys: int, seed: int, *, log2_min: float = 10.0,
                  log2_max: float = 18.0, W0: float = 6.0):
    """Independent clusters, N_k = floor(2^(log2_min + (log2_max-log2_min) u_k)),
    each a Plummer or King(W0) model with probability 1/2, G = M = scale = 1.
    Returns a list of Particles."""
    rng = rng_for(seed, 3)
    u = rng.uniform(0.0, 1.0, n_sys)
    kinds = rng.uniform(0.0, 1.0, n_sys) < 0.5
    out = []
    for k in range(n_sys):
        nk = int(math.floor(2.0 ** (log2_min + (log2_max - log2_min) * u[k])))
        sk = int(seed) * 1000003 + k
        out.append(plummer(nk, sk) if kinds[k] else king(nk, sk, W0=W0))
    return out


def uniform_cube(n: int, seed: int, *, side: float = 1.0) -> Particles:
    """Uniform random points in [0, side)^3, zero velocities, equal masses."""
    rng = rng_for(seed, 4)
    pos = rng.uniform(0.0, side, (int(n), 3))
    return Particles(pos, np.zeros_like(pos), np.full(int(n), 1.0 / n), {"model": "cube"})


def random_subset(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices out of n: the first k entries of a seeded
    Fisher-Yates shuffle (numpy's permutation)."""
    return rng_for(seed, 5).permutation(int(n))[: int(k)].astype(np.int64)


def mlp_init(n_params: int, fan_in: np.ndarray, seed: int) -> np.ndarray:
    """Random initial weights for a small network: entry k uniform in
    [-1/sqrt(fan_in[k]), 1/sqrt(fan_in[k])) (fan_in gives, per entry, the
    number of inputs of the unit it feeds), float32."""
    rng = rng_for(seed, 6)
    fan = np.asarray(fan_in, np.float64)
    assert fan.shape == (n_params,)
    return (rng.uniform(-1.0, 1.0, n_params) / np.sqrt(fan)).astype(np.float32)
