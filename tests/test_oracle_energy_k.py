"""Pins of the oracle's changeover potential and E_K (the energy that the
step map without the direct solver conserves for fixed critical radii; the
force reading of eq. Hb, Sect. 2).

* the integral int K(s)/s^2 ds against scipy's adaptive quadrature;
* the potential's derivative is the kick's K-weighted Newtonian force;
* limits: Newtonian beyond rho, flat below 0.1 rho;
* with rc held fixed, the kick-drift-kick map through a two-planet close
  pass conserves E_K to within its own O(dt^2) error, while E (the plain
  Newtonian energy) changes a hundred times more.
"""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from encounter_fixture import two_planets

G = 0.01720209895 ** 2


@pytest.mark.parametrize("r", [0.0005, 0.002, 0.005, 0.01, 0.0199])
def test_integral_matches_quad(r):
    rho = 0.02
    q = quad(lambda s: oracle.changeover(s, rho) / s ** 2, max(r, 0.1 * rho), rho,
             epsabs=0, epsrel=1e-13, limit=200)[0]
    assert abs(oracle.changeover_integral(r, rho) - q) <= 1e-12 * q


def _phi(r, rho, gmm=1.0):
    if r >= rho:
        return -gmm / r
    return -gmm * (1.0 / rho + oracle.changeover_integral(r, rho))


@pytest.mark.parametrize("r", [0.0035, 0.006, 0.012, 0.018])
def test_potential_derivative_is_the_weighted_force(r):
    rho, h = 0.02, 1e-6
    dphi = (_phi(r + h, rho) - _phi(r - h, rho)) / (2 * h)
    assert abs(dphi - oracle.changeover(r, rho) / r ** 2) <= 1e-6 * abs(dphi)


def test_potential_limits():
    rho = 0.02
    assert _phi(0.03, rho) == -1.0 / 0.03
    assert _phi(0.001, rho) == _phi(0.0015, rho)          # flat inside 0.1 rho
    assert abs(_phi(rho * (1 - 1e-9), rho) + 1.0 / rho) < 1e-6   # continuous at rho


def _kdk_errors(a2, dt, T=300.0):
    state, _ = two_planets(a2)
    rc = np.array([0.04, 0.04])
    st = {k: v.copy() for k, v in state.items()}
    e0, k0 = oracle.energy(st, G, 1.0), oracle.energy_k(st, rc, G, 1.0)
    de = dk = 0.0
    for _ in range(int(round(T / dt))):
        oracle.kick(st, rc, G, dt / 2)
        oracle.hc(st, 1.0, dt / 2)
        oracle.drift(st, G, dt)
        oracle.hc(st, 1.0, dt / 2)
        oracle.kick(st, rc, G, dt / 2)
        de = max(de, abs(oracle.energy(st, G, 1.0) - e0) / abs(e0))
        dk = max(dk, abs(oracle.energy_k(st, rc, G, 1.0) - k0) / abs(k0))
    return de, dk


def test_fixed_rc_map_conserves_e_k():
    de, dk = _kdk_errors(1.01, 6.0)
    assert dk < 0.01 * de
    _, dk2 = _kdk_errors(1.01, 3.0)
    assert dk2 < 0.35 * dk           # E_K's residual is the map's O(dt^2) error
