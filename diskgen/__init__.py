"""Seeded synthetic planetesimal disks.

Input generation only: orbital elements are drawn from seeded distributions and converted to
heliocentric positions and barycentric ("democratic heliocentric") velocities. Nothing of the
integration method (kick, encounter test, drift, jump) lives here; both the CPU oracle and the
GPU library read the arrays this module writes.

Disk recipe (the workload of the paper's performance figure and its resolution study: a disk of
planetesimals between 0.5 and 4 AU with a few Earth masses around a solar-mass star):
  a ~ U[a_lo, a_hi] AU, e ~ Rayleigh(sigma_e), i ~ Rayleigh(sigma_i) rad,
  node, argument of pericentre, mean anomaly ~ U[0, 2 pi),
  masses equal (total mass given) or dN/dm ~ m^-slope on [m_lo, m_hi] by inverse CDF.
Units: G = 1, AU, solar masses, time unit 1/k days with k the Gaussian gravitational constant.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

K_GAUSS = 0.01720209895          # Gaussian gravitational constant (AU^1.5 Msun^-0.5 / day)
M_EARTH = 3.0034896e-6           # Earth mass in solar masses
AU_CM = 1.495978707e13
MSUN_G = 1.98847e33
DAY = K_GAUSS                    # one day in code time units
DT_6DAYS = 6.0 * DAY


@dataclasses.dataclass(frozen=True)
class Disk:
    n: int
    a_lo: float = 0.5
    a_hi: float = 4.0
    sigma_e: float = 0.01
    sigma_i: float = 0.005
    total_mass_earth: float | None = 2.0       # equal masses with this total
    powerlaw: tuple | None = None              # (slope, m_lo_earth, m_hi_earth), dN/dm ~ m^-slope
    density_cgs: float = 2.0
    seed: int | np.random.SeedSequence = 0
    m0: float = 1.0
    G: float = 1.0


def _solve_kepler_mean(M, e):
    """Eccentric anomaly from mean anomaly for 0 <= e < 1 (vectorised Newton)."""
    E = M + e * np.sin(M)
    for _ in range(50):
        f = E - e * np.sin(E) - M
        E = E - f / (1.0 - e * np.cos(E))
    return E


def elements_to_cartesian(a, e, inc, node, argp, M, mu):
    """Heliocentric position and velocity of elliptic orbits (vectorised)."""
    E = _solve_kepler_mean(M, e)
    cE, sE = np.cos(E), np.sin(E)
    b = a * np.sqrt(1.0 - e * e)
    # perifocal frame
    xp = a * (cE - e)
    yp = b * sE
    n = np.sqrt(mu / a ** 3)
    rdot = a * n / (1.0 - e * cE)
    vxp = -rdot * sE
    vyp = rdot * np.sqrt(1.0 - e * e) * cE
    cO, sO = np.cos(node), np.sin(node)
    cw, sw = np.cos(argp), np.sin(argp)
    ci, si = np.cos(inc), np.sin(inc)
    # rotation perifocal -> reference: Rz(node) Rx(inc) Rz(argp)
    r11 = cO * cw - sO * sw * ci
    r12 = -cO * sw - sO * cw * ci
    r21 = sO * cw + cO * sw * ci
    r22 = -sO * sw + cO * cw * ci
    r31 = sw * si
    r32 = cw * si
    x = np.stack([r11 * xp + r12 * yp, r21 * xp + r22 * yp, r31 * xp + r32 * yp], axis=1)
    v = np.stack([r11 * vxp + r12 * vyp, r21 * vxp + r22 * vyp, r31 * vxp + r32 * vyp], axis=1)
    return x, v


def make_disk(d: Disk):
    """Returns dict with x (n,3) heliocentric, v (n,3) barycentric, m (n,), radius (n,)."""
    rng = np.random.Generator(np.random.PCG64(d.seed))
    n = d.n
    a = rng.uniform(d.a_lo, d.a_hi, n)
    e = rng.rayleigh(d.sigma_e, n)
    e = np.minimum(e, 0.9)
    inc = rng.rayleigh(d.sigma_i, n)
    node = rng.uniform(0.0, 2 * math.pi, n)
    argp = rng.uniform(0.0, 2 * math.pi, n)
    M = rng.uniform(0.0, 2 * math.pi, n)
    if d.powerlaw is not None:
        slope, mlo, mhi = d.powerlaw
        u = rng.uniform(0.0, 1.0, n)
        k = 1.0 - slope
        m = ((mlo ** k) + u * ((mhi ** k) - (mlo ** k))) ** (1.0 / k) * M_EARTH
    else:
        m = np.full(n, d.total_mass_earth * M_EARTH / n)
    mu = d.G * (d.m0 + m)
    x, vh = elements_to_cartesian(a, e, inc, node, argp, M, mu)
    vbar = vh - (m[:, None] * vh).sum(axis=0) / (d.m0 + m.sum())
    rho = d.density_cgs * AU_CM ** 3 / MSUN_G
    radius = (3.0 * m / (4.0 * math.pi * rho)) ** (1.0 / 3.0)
    return {"x": np.ascontiguousarray(x), "v": np.ascontiguousarray(vbar), "m": m, "radius": radius}


def pack4(x, v, m):
    """(n,4) float64 layouts: xm = [x, y, z, m], v4 = [vx, vy, vz, 0]."""
    n = x.shape[0]
    xm = np.zeros((n, 4))
    xm[:, :3] = x
    xm[:, 3] = m
    v4 = np.zeros((n, 4))
    v4[:, :3] = v
    return xm, v4


# ---------------------------------------------------------------- the five workloads
PARAMS = dict(G=1.0, m0=1.0, dt=DT_6DAYS, n1=3.0, n2=0.4, f_in=0.1)

WORKLOADS = {
    "disk2048": dict(disk=Disk(2048, 0.5, 4.0, 0.01, 0.005, 2.0, seed=1000), steps=10),
    "disk32768": dict(disk=Disk(32768, 0.3, 4.0, 0.01, 0.005, 5.0, seed=1001), steps=1000),
    "ring131072": dict(disk=Disk(131072, 0.7, 1.0, 0.005, 0.005, None, (2.5, 1e-4, 1e-2), seed=1002),
                       steps=100),
    "ensemble4096": dict(systems=4096, n_lo=64, n_hi=2048, seed=1003, steps=100),
    "adjoint8192": dict(disk=Disk(8192, 0.5, 4.0, 0.01, 0.005, 2.0, seed=1004), steps=100, every=10),
}


def workload(name: str, n: int | None = None):
    """Disk of a named workload; n overrides the body count (a smaller case of the same recipe)."""
    d = WORKLOADS[name]["disk"]
    if n is not None:
        d = dataclasses.replace(d, n=n)
    return make_disk(d)


def ensemble(systems=4096, n_lo=64, n_hi=2048, seed=1003):
    """Independent disks of uneven size: N_s = round(exp U[ln n_lo, ln n_hi]); system s uses the
    s-th child of SeedSequence(seed). Returns (offsets (S+1,), x, v, m) concatenated."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.Generator(np.random.PCG64(ss))
    sizes = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), systems))).astype(np.int64)
    children = ss.spawn(systems)
    xs, vs, ms = [], [], []
    for s in range(systems):
        disk = make_disk(Disk(int(sizes[s]), 0.5, 4.0, 0.01, 0.005, 2.0, seed=children[s]))
        xs.append(disk["x"]); vs.append(disk["v"]); ms.append(disk["m"])
    offs = np.zeros(systems + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    return offs, np.concatenate(xs), np.concatenate(vs), np.concatenate(ms)


def loss_target(x_final, seed=1004, scale=1e-4):
    """Perturbed copy of final positions for the adjoint workload's loss."""
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    return x_final + scale * rng.standard_normal(x_final.shape)
