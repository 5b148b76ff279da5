"""Seeded synthetic planetesimal disks and fixtures.

This module only builds inputs.  It holds none of the integrator's arithmetic
(no changeover weight, no kick, no pair test, no drift): both the HIP path and
the CPU oracle consume the arrays it returns, so it must stay neutral.

Units are those of the Gaussian system: AU, day, solar mass, with
G = k^2 and k = 0.01720209895 (the paper states no units; this is the
customary choice for planetary N-body codes).

Disk recipe (stands in for the planetesimal disks of Sect. 6.2, Sect. 6.3 and
Sect. 9 of the paper, which are described only by their radial range, total
mass and particle count):
  * semi-major axis a ~ U[a_min, a_max]
  * eccentricity    e ~ Rayleigh(sigma_e)      (pdf x/s^2 exp(-x^2/2s^2))
  * inclination     i ~ Rayleigh(sigma_i) rad
  * Omega, omega, M ~ U[0, 2 pi)
  * equal masses m_i = M_total / N, physical radius from a bulk density
  * elements -> heliocentric Cartesian with mu_i = G (m_star + m_i)
  * heliocentric -> democratic coordinates (heliocentric positions,
    barycentric velocities), the coordinates of Sect. 2 of the paper.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAUSS_K = 0.01720209895
GAUSS_G = GAUSS_K * GAUSS_K              # AU^3 / (Msun day^2)
M_EARTH = 1.0 / 332946.0487              # in solar masses
MSUN_G = 1.98847e33                      # grams
AU_CM = 1.495978707e13                   # centimetres

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m")


@dataclass(frozen=True)
class DiskSpec:
    """A planetesimal disk: N bodies around a central star of mass m_star."""
    name: str
    n: int
    a_min: float
    a_max: float
    m_total_earth: float
    seed: int
    sigma_e: float = 0.01
    sigma_i: float = 0.005
    density_cgs: float = 2.0
    m_star: float = 1.0
    dt: float = 6.0
    n1: float = 3.0
    n2: float = 0.4


# The workloads of the build.  Names state what they are.
DISK_2048 = DiskSpec("disk_n2048_a0.5-1.5_2Mearth", 2048, 0.5, 1.5, 2.0, seed=0)
DISK_65536 = DiskSpec("disk_n65536_a0.5-4_5Mearth", 65536, 0.5, 4.0, 5.0, seed=1)
DISK_MIXED = {
    16384: DiskSpec("disk_n16384_a0.5-4_5Mearth", 16384, 0.5, 4.0, 5.0, seed=20),
    32768: DiskSpec("disk_n32768_a0.5-4_5Mearth", 32768, 0.5, 4.0, 5.0, seed=21),
    65536: DiskSpec("disk_n65536_a0.5-4_5Mearth_s22", 65536, 0.5, 4.0, 5.0, seed=22),
}
DISK_ADJOINT = DiskSpec("disk_n4096_a0.5-1.5_2Mearth", 4096, 0.5, 1.5, 2.0, seed=4)


def _rayleigh(rng: np.random.Generator, sigma: float, n: int) -> np.ndarray:
    # inverse-CDF draw; 1-U in (0, 1] keeps the log finite
    return sigma * np.sqrt(-2.0 * np.log1p(-rng.random(n)))


def _kepler_ecc_anomaly(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Eccentric anomaly for the initial conditions (bound orbits, e < 1)."""
    E = M + e * np.sin(M)
    for _ in range(60):
        f = E - e * np.sin(E) - M
        E_new = E - f / (1.0 - e * np.cos(E))
        if np.max(np.abs(E_new - E)) < 1e-15:
            E = E_new
            break
        E = E_new
    return E


def elements_to_state(a, e, inc, Omega, omega, M, mu):
    """Heliocentric position and velocity from Keplerian elements (e < 1)."""
    E = _kepler_ecc_anomaly(np.asarray(M, dtype=np.float64), np.asarray(e, dtype=np.float64))
    cE, sE = np.cos(E), np.sin(E)
    b = a * np.sqrt(1.0 - e * e)
    # position and velocity in the orbital plane (pericentre along +X)
    X = a * (cE - e)
    Y = b * sE
    r = a * (1.0 - e * cE)
    nmean = np.sqrt(mu / (a * a * a))
    VX = -a * nmean * a * sE / r
    VY = b * nmean * a * cE / r
    cO, sO = np.cos(Omega), np.sin(Omega)
    cw, sw = np.cos(omega), np.sin(omega)
    ci, si = np.cos(inc), np.sin(inc)
    # rotation R_z(Omega) R_x(i) R_z(omega)
    P = np.stack([cO * cw - sO * sw * ci, sO * cw + cO * sw * ci, sw * si])
    Q = np.stack([-cO * sw - sO * cw * ci, -sO * sw + cO * cw * ci, cw * si])
    pos = P * X + Q * Y
    vel = P * VX + Q * VY
    return pos, vel


def make_disk(spec: DiskSpec, masses=None) -> dict:
    """Return a dict of contiguous float64 arrays x,y,z,vx,vy,vz,m,R plus scalars
    (equal masses m_total/N unless `masses` [solar masses] is given)."""
    n = spec.n
    rng = np.random.default_rng(spec.seed)
    a = rng.uniform(spec.a_min, spec.a_max, n)
    e = _rayleigh(rng, spec.sigma_e, n)
    inc = _rayleigh(rng, spec.sigma_i, n)
    Omega = rng.uniform(0.0, 2.0 * math.pi, n)
    omega = rng.uniform(0.0, 2.0 * math.pi, n)
    M = rng.uniform(0.0, 2.0 * math.pi, n)
    if masses is None:
        m = np.full(n, spec.m_total_earth * M_EARTH / n)
    else:
        m = np.ascontiguousarray(masses, dtype=np.float64)
    mu = GAUSS_G * (spec.m_star + m)
    pos, vel = elements_to_state(a, e, inc, Omega, omega, M, mu)
    # democratic coordinates: heliocentric positions, barycentric velocities
    ptot = (m[None, :] * vel).sum(axis=1)
    vel = vel - (ptot / (spec.m_star + m.sum()))[:, None]
    R = np.cbrt(3.0 * m * MSUN_G / (4.0 * math.pi * spec.density_cgs)) / AU_CM
    out = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in
           zip(FIELDS, (pos[0], pos[1], pos[2], vel[0], vel[1], vel[2], m))}
    out["R"] = R
    out.update(n=n, G=GAUSS_G, m_star=spec.m_star, dt=spec.dt, n1=spec.n1, n2=spec.n2,
               name=spec.name)
    return out


def make_tp_disk(n: int = 65536, n_massive: int = 16, seed: int = 30,
                 m_massive_earth: float = 1.0, tp_total_earth: float = 5.0) -> dict:
    """The test-particle setup of Sect. 8: a disk between 0.5 and 4 AU with
    zero inclination, whose first `n_massive` bodies are massive (reading:
    m_massive_earth Earth masses each; the paper gives no value) and the rest
    test particles sharing tp_total_earth Earth masses (used by the
    semi-active mode)."""
    spec = DiskSpec(f"tpdisk_n{n}_m{n_massive}_a0.5-4_i0", n, 0.5, 4.0, tp_total_earth, seed=seed,
                    sigma_i=0.0)
    m = np.full(n, tp_total_earth * M_EARTH / max(n - n_massive, 1))
    m[:n_massive] = m_massive_earth * M_EARTH
    d = make_disk(spec, masses=m)
    d["n_massive"] = n_massive
    return d


def batch_sizes(n_systems: int = 512, n_lo: int = 16, n_hi: int = 4096, seed: int = 3) -> np.ndarray:
    """Per-system body counts, log-uniform in [n_lo, n_hi]."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(n_lo), math.log(n_hi), n_systems)
    return np.clip(np.rint(np.exp(u)).astype(np.int64), n_lo, n_hi)


def make_batch(n_systems: int = 512, n_lo: int = 16, n_hi: int = 4096, seed: int = 3,
               sizes=None) -> dict:
    """Many independent disks drawn from the 0.5-1.5 AU distribution.

    Every body has mass 2 M_earth / 2048, so a system's total mass scales with
    its size.  System s uses seed 1000 + s.  Arrays are concatenated; offsets
    has length S + 1.
    """
    if sizes is None:
        sizes = batch_sizes(n_systems, n_lo, n_hi, seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    parts = []
    for s, ns in enumerate(sizes):
        spec = DiskSpec(f"sys{s}", int(ns), 0.5, 1.5, 2.0 * int(ns) / 2048.0, seed=1000 + s)
        parts.append(make_disk(spec))
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    out = {k: np.ascontiguousarray(np.concatenate([p[k] for p in parts])) for k in FIELDS + ("R",)}
    out.update(offsets=offsets, sizes=sizes, S=len(sizes), G=GAUSS_G,
               m_star=np.ones(len(sizes)), dt=np.full(len(sizes), 6.0),
               n1=np.full(len(sizes), 3.0), n2=np.full(len(sizes), 0.4))
    return out


def make_ring(n: int, radius: float = 1.0, m_body: float = 1e-9, neighbours: int = 4):
    """N equal masses evenly spaced on a circle of given radius (Sect. 6.1).

    The critical radius is set midway between the chord to the k-th and the
    (k+1)-th neighbour, so that each body meets exactly `neighbours` bodies on
    each side (2*neighbours encounter partners, as in the paper's ring test).
    Velocities are zero: the fixture exercises positions only.
    """
    k = np.arange(n, dtype=np.float64)
    th = 2.0 * math.pi * k / n
    x = radius * np.cos(th)
    y = radius * np.sin(th)
    z = np.zeros(n)

    def chord(q):
        return 2.0 * radius * math.sin(math.pi * q / n)

    if n <= 2 * neighbours + 1:
        # every other body is a neighbour: take them all
        rc = np.full(n, 2.2 * radius)
    else:
        rc = np.full(n, 0.5 * (chord(neighbours) + chord(neighbours + 1)))
    zeros = np.zeros(n)
    return dict(x=x, y=y, z=z, vx=zeros.copy(), vy=zeros.copy(), vz=zeros.copy(),
                m=np.full(n, m_body), rc=rc, n=n)


def make_bs_ring(n: int, m_body: float | None = None, neighbours: int = 4,
                 G: float = GAUSS_G) -> dict:
    """The close-encounter performance test of Sect. 6.1: n equal masses
    evenly spaced on a circular orbit of radius 1 about a unit star
    (barycentric velocities, coplanar).  Returns the state and the n1 for
    which the critical radius n1 R_H (n2 = 0) lies midway between the chords
    to the k-th and (k+1)-th neighbour, k = `neighbours`: every body meets
    2k others and the encounter graph is one chain, a single group of n.
    Below 2k + 2 bodies every other body is a partner (rc = 2.2).

    The default mass, min(1e-9, 1e-4 (2 pi / n)^2), keeps a neighbour's pull
    below 1e-4 of the star's at every n, so that the ring stays a ring over a
    step (a heavier dense ring clumps and the group's steps shrink): the
    test then times the same Bulirsch-Stoer work per body at every n."""
    if m_body is None:
        m_body = min(1e-9, 1e-4 * (2.0 * math.pi / n) ** 2)
    th = 2.0 * math.pi * np.arange(n, dtype=np.float64) / n
    v = math.sqrt(G * (1.0 + m_body))
    m = np.full(n, m_body)
    vh = np.stack([-v * np.sin(th), v * np.cos(th), np.zeros(n)], 1)
    vb = vh - (m[:, None] * vh).sum(0) / (1.0 + m.sum())
    rh = (m_body / 3.0) ** (1.0 / 3.0)
    if n <= 2 * neighbours + 1:
        rc = 2.2
    else:
        def chord(q):
            return 2.0 * math.sin(math.pi * q / n)
        rc = 0.5 * (chord(neighbours) + chord(neighbours + 1))
    return {"x": np.cos(th), "y": np.sin(th), "z": np.zeros(n),
            "vx": vb[:, 0].copy(), "vy": vb[:, 1].copy(), "vz": vb[:, 2].copy(), "m": m,
            "n": n, "n1": rc / rh, "G": G, "m_star": 1.0, "dt": 6.0,
            "name": f"bs_ring_n{n}_k{neighbours}"}


def random_cloud(n: int, seed: int, spread: float = 1.0, rc_scale: float = 0.2,
                 m_scale: float = 1e-6) -> dict:
    """Uniform random bodies in a cube, random masses and critical radii.

    Used for parity tests that need many pairs inside the changeover band.
    """
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-spread, spread, (3, n))
    vel = rng.normal(0.0, 0.01, (3, n))
    m = m_scale * rng.uniform(0.5, 1.5, n)
    rc = rc_scale * spread * rng.uniform(0.25, 1.0, n)
    return dict(x=pos[0].copy(), y=pos[1].copy(), z=pos[2].copy(),
                vx=vel[0].copy(), vy=vel[1].copy(), vz=vel[2].copy(), m=m, rc=rc, n=n)
