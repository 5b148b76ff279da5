"""Pins of the oracle's post-Newtonian term (Sect. 3, eq. apn, applied by the
implicit midpoint rule of eq. implicit).

* perihelion precession per orbit = 6 pi G M / (c^2 a (1 - e^2)) for a test
  particle (closed form), with the real speed of light and with c / 10;
* the test-particle 1PN energy v^2/2 - mu/r + (3/8 v^4 + 3/2 mu v^2 / r +
  1/2 mu^2 / r^2) / c^2 is conserved 10^4 times better than the Newtonian one;
* a body of 0.3 star masses: the two-body 1PN energy with the symmetric mass
  ratio eta is conserved and converges at second order in dt, while the same
  energy without its eta terms is not (pins the eta terms of the force);
* the implicit midpoint update is time-symmetric: h then -h restores v.
"""
import numpy as np
import pytest

import oracle

G = 0.01720209895 ** 2
C = 173.1446326846693          # speed of light [AU/day]


def _orbit(m, a=0.387, e=0.2056):
    mu = G * (1.0 + m)
    rp = a * (1 - e)
    vp = np.sqrt(mu * (1 + e) / rp)
    # heliocentric relative velocity vp; barycentric planet velocity vp/(1+m)
    st = {"x": np.array([rp]), "y": np.array([0.0]), "z": np.array([0.0]),
          "vx": np.array([0.0]), "vy": np.array([vp / (1 + m)]), "vz": np.array([0.0]),
          "m": np.array([m])}
    return st, mu, 2 * np.pi * np.sqrt(a ** 3 / mu)


def _perihelion_angle(st, mu, m):
    r = np.array([st["x"][0], st["y"][0], st["z"][0]])
    u = np.array([st["vx"][0], st["vy"][0], st["vz"][0]]) * (1 + m)
    A = np.cross(u, np.cross(r, u)) - mu * r / np.linalg.norm(r)
    return np.arctan2(A[1], A[0])


@pytest.mark.parametrize("cfac,tol", [(1.0, 1e-4), (0.1, 1e-3)])
def test_perihelion_precession(cfac, tol):
    a, e, norb, spo = 0.387, 0.2056, 20, 400
    st, mu, T = _orbit(1e-12, a, e)
    c = C * cfac
    w0 = _perihelion_angle(st, mu, 1e-12)
    for _ in range(norb * spo):
        oracle.step_gr(st, G, 1.0, T / spo, 3.0, 0.4, c)
    dw = _perihelion_angle(st, mu, 1e-12) - w0
    pred = norb * 6 * np.pi * mu / (c * c * a * (1 - e * e))
    assert abs(dw / pred - 1.0) < tol
    # and without the term the orbit does not precess at this level
    st2, _, _ = _orbit(1e-12, a, e)
    for _ in range(spo):
        oracle.step(st2, G, 1.0, T / spo, 3.0, 0.4)
    assert abs(_perihelion_angle(st2, mu, 1e-12) - w0) < 1e-3 * pred / norb


def _energies(st, mu, m, c, eta):
    r = np.array([st["x"][0], st["y"][0], st["z"][0]])
    u = np.array([st["vx"][0], st["vy"][0], st["vz"][0]]) * (1 + m)
    rr = np.linalg.norm(r)
    v2 = u @ u
    rd = (r @ u) / rr
    en = v2 / 2 - mu / rr
    e1 = (3 / 8 * (1 - 3 * eta) * v2 * v2 + mu / (2 * rr) * ((3 + eta) * v2 + eta * rd * rd)
          + mu * mu / (2 * rr * rr)) / (c * c)
    return en, en + e1


def _energy_errors(m, spo, eta_in_energy, norb=2, c=C / 10):
    st, mu, T = _orbit(m)
    eta = m / (1 + m) ** 2 if eta_in_energy else 0.0
    e0 = _energies(st, mu, m, c, eta)
    dn = d1 = 0.0
    for _ in range(spo * norb):
        oracle.step_gr(st, G, 1.0, T / spo, 3.0, 0.4, c)
        en, e1 = _energies(st, mu, m, c, eta)
        dn = max(dn, abs(en - e0[0]) / abs(e0[0]))
        d1 = max(d1, abs(e1 - e0[1]) / abs(e0[1]))
    return dn, d1


def test_test_particle_1pn_energy_is_conserved():
    dn, d1 = _energy_errors(1e-12, 2000, True)
    assert dn > 1e-5 and d1 < 1e-4 * dn


def test_eta_terms_by_the_two_body_1pn_energy():
    _, d1a = _energy_errors(0.3, 2000, True)
    _, d1b = _energy_errors(0.3, 4000, True)
    _, d1w = _energy_errors(0.3, 4000, False)
    assert d1b < 0.4 * d1a          # second order in dt: the integrator's error
    assert d1w > 10 * d1b           # the eta-free energy is not conserved


def test_implicit_midpoint_is_symmetric():
    rng = np.random.default_rng(3)
    n = 5
    st = {"x": rng.uniform(0.3, 1, n), "y": rng.uniform(-1, 1, n), "z": rng.uniform(-0.1, 0.1, n),
          "vx": rng.uniform(-0.02, 0.02, n), "vy": rng.uniform(-0.02, 0.02, n),
          "vz": rng.uniform(-0.002, 0.002, n), "m": rng.uniform(1e-9, 1e-3, n)}
    v0 = {k: st[k].copy() for k in ("vx", "vy", "vz")}
    oracle.gr_kick(st, G, 1.0, C / 10, 3.0)
    moved = max(np.abs(st[k] - v0[k]).max() for k in v0)
    oracle.gr_kick(st, G, 1.0, C / 10, -3.0)
    back = max(np.abs(st[k] - v0[k]).max() for k in v0)
    assert moved > 1e-9 and back < 1e-16
