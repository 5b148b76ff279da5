"""Pins of the oracle's symplectic levels (Sect. 6.2, higher-level changeover
functions; Appendix A, the recursive encounter routine).

* one level is the base step, bit for bit;
* levels change nothing when no pair is inside the critical radius;
* the levels integrate the part of the pair force that the base step leaves to
  the direct solver: for a Sun + two-planet encounter whose closest approach
  stays outside the deepest level's critical radius (so nothing is left for
  the direct solver), the levelled step follows the Newtonian three-body
  solution (scipy's DOP853 at tight tolerance, in barycentric coordinates)
  orders of magnitude more closely than the base step, and converges as dt
  shrinks.  A dropped level weight, a wrong sign or a missing state restore
  before the sub-steps each leave errors of the base step's size;
* on the 2,048-body disk the energy error falls as levels are added.
"""
import numpy as np
import pytest
import oracle
from encounter_fixture import two_planets
from paper_2201_10058_amd import workload as W

G = W.GAUSS_G


def _two_planets(a2, m=3e-6, T=300.0):
    return two_planets(a2, m=m, T=T)


def _run(state, T, dt, n1, n2, levels, substeps):
    st = {k: v.copy() for k, v in state.items()}
    counts = np.zeros(levels, dtype=np.int64)
    for _ in range(int(round(T / dt))):
        r = oracle.step_levels(st, G, 1.0, dt, n1, n2, levels, substeps)
        assert r[5] == 0
        counts += r[4]
    return np.stack([st["x"], st["y"], st["z"]], 1), counts


def test_one_level_is_the_base_step():
    d = W.make_disk(W.DISK_2048)
    a, b = oracle.state_copy(d), oracle.state_copy(d)
    for _ in range(3):
        ra = oracle.step(a, G, 1.0, 6.0, 3.0, 0.4)
        rb = oracle.step_levels(b, G, 1.0, 6.0, 3.0, 0.4, 1, 7)
        assert ra[2] == rb[2] and np.array_equal(ra[0], rb[0]) and np.array_equal(ra[1], rb[1])
    for k in a:
        assert np.array_equal(a[k], b[k])


def test_levels_without_encounters_change_nothing():
    state, _ = _two_planets(1.5)
    a, ca = _run(state, 60.0, 6.0, 3.0, 0.4, 1, 1)
    b, cb = _run(state, 60.0, 6.0, 3.0, 0.4, 3, 4)
    assert ca[0] == 0 and cb.sum() == 0
    assert np.array_equal(a, b)


def test_two_levels_follow_the_newtonian_encounter():
    # closest approach 0.0225 AU: inside rho_0 = n2 v dt = 0.041 AU, outside
    # the level-1 radius (dt / 10: 0.0041 AU), so level 1 takes the whole
    # (1 - K_0) part and nothing is left for the direct solver
    T = 300.0
    state, ref = _two_planets(1.03, T=T)
    base, c1 = _run(state, T, 6.0, 0.5, 0.4, 1, 1)
    lev, c2 = _run(state, T, 6.0, 0.5, 0.4, 2, 10)
    e_base, e_lev = np.abs(base - ref).max(), np.abs(lev - ref).max()
    assert c1[0] > 0 and c2[1] == 0
    assert e_base > 1e-3
    assert e_lev < 1e-4
    # second-order convergence when dt is halved with rho_0 = n2 v dt kept
    # (n2 doubled), while the base step's error, the dropped (1 - K_0) part,
    # does not shrink
    lev2, _ = _run(state, T, 3.0, 0.5, 0.8, 2, 10)
    base2, _ = _run(state, T, 3.0, 0.5, 0.8, 1, 1)
    assert np.abs(lev2 - ref).max() < 0.3 * e_lev
    assert np.abs(base2 - ref).max() > 0.9 * e_base


def test_three_levels_reach_the_second_level():
    # n2 = 4: rho_0 = 0.41 AU, level 1 (dt / 5) 0.083 AU still holds the pair,
    # level 2 (dt / 25) 0.0165 AU does not: with three levels nothing is left
    # for the direct solver, with two the (1 - K_0)(1 - K_1) part is dropped
    T = 300.0
    state, ref = _two_planets(1.03, T=T)
    two, c2 = _run(state, T, 6.0, 0.5, 4.0, 2, 5)
    three, c3 = _run(state, T, 6.0, 0.5, 4.0, 3, 5)
    assert c2[1] > 0 and c3[1] > 0 and c3[2] == 0
    assert np.abs(two - ref).max() > 1e-3
    assert np.abs(three - ref).max() < 1e-5


def test_energy_error_falls_with_levels():
    d = W.make_disk(W.DISK_2048)
    E0 = oracle.energy(d, G, 1.0)
    errs = {}
    for L, s in ((1, 1), (3, 4)):
        st = oracle.state_copy(d)
        e = 0.0
        for _ in range(60):
            oracle.step_levels(st, G, 1.0, 6.0, 3.0, 0.4, L, s)
            e = max(e, abs(oracle.energy(st, G, 1.0) - E0) / abs(E0))
        errs[L] = e
    assert errs[3] < 0.7 * errs[1]


@pytest.mark.parametrize("levels,substeps", [(2, 2), (3, 2)])
def test_level_lists_shrink(levels, substeps):
    d = W.make_disk(W.DISK_2048)
    st = oracle.state_copy(d)
    r = oracle.step_levels(st, G, 1.0, 6.0, 3.0, 0.4, levels, substeps)
    counts = r[4]
    # each level's lists are subsets of the upper list, found once per sub-step
    assert counts[0] == r[2] > 0
    for l in range(1, levels):
        assert 0 < counts[l] <= counts[l - 1] * substeps


@pytest.mark.parametrize("L", [1, 2, 3, 5])
def test_level_weights_telescope(L):
    # sum_l W_l + remainder = 1 at every separation (Sect. 6.2: the levels
    # and the direct solver split each pair force without gap or overlap)
    rng = np.random.default_rng(L)
    for _ in range(200):
        rho = np.sort(rng.uniform(0.001, 0.05, L))[::-1]
        r = rng.uniform(0.0, 0.06)
        parts = [oracle.level_weight(r, rho, l) for l in range(L + 1)]
        assert all(p >= 0.0 for p in parts)
        assert abs(sum(parts) - 1.0) < 1e-15


def test_ten_substeps_keep_two_levels_active():
    # with the velocity term dominating, a level of dt / 10 has rho_1 =
    # rho_0 / 10, so K(r; rho_1) = 1 wherever 0 < K(r; rho_0) < 1: no more than
    # two levels act on a pair at once
    rho0 = 0.04
    rho1 = rho0 / 10
    for r in np.linspace(0.1 * rho0 * (1 + 1e-3), rho0 * (1 - 1e-3), 101):
        assert 0.0 < oracle.changeover(r, rho0) < 1.0
        assert oracle.changeover(r, rho1) == 1.0
        assert oracle.level_weight(r, [rho0, rho1], 2) == 0.0
