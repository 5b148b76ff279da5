"""Pins of the oracle's collisions in the direct solver (Sect. 7, collision
handling: perfect mergers, lost energy, survivor index).

* one base step through a contact against a reference built from scipy's
  DOP853 with event location of r = R_0 + R_1 and the paper's merger
  formulas (the collision fixture);
* survivor: the more massive body, the lower index for equal masses;
* E_after + sum of the lost energies equals E_before to the integrator's
  error, while E alone changes by the lost energy (1e-6 to 1e-5 of E here).
"""
import numpy as np
import pytest

import oracle
from collision_fixture import G, reference_step, two_bodies


@pytest.mark.parametrize("kw,survivor", [(dict(), 0), (dict(m1=3e-9), 1), (dict(m0=3e-9), 0)])
def test_merger_against_event_located_reference(kw, survivor):
    st = two_bodies(**kw)
    ref, tc, (s, g, dU) = reference_step(st, 6.0)
    assert 0.0 < tc < 6.0 and s == survivor
    o = {k: v.copy() for k, v in st.items()}
    r = oracle.step_coll(o, G, 1.0, 6.0, 3.0, 0.4, 1, 1, rk_steps=2000)
    assert r[-1] == 0
    assert len(r[3]) == 1
    cs, cg, cdu = r[3][0]
    assert (cs, cg) == (s, g)
    assert abs(cdu - dU) <= 1e-4 * abs(dU)
    for k in ("x", "y", "z"):
        assert abs(o[k][s] - ref[k][s]) < 1e-12
    for k in ("vx", "vy", "vz"):
        assert abs(o[k][s] - ref[k][s]) < 1e-14
    assert o["m"][s] == ref["m"][s] and o["m"][g] == 0.0
    assert abs(o["R"][s] - ref["R"][s]) <= 1e-15 * ref["R"][s] and o["R"][g] == 0.0
    assert abs(o["x"][g] - (1e6 + g)) < 1e-3          # the ghost is parked


@pytest.mark.parametrize("kw", [dict(), dict(m1=3e-9)])
def test_energy_plus_lost_energy_is_conserved(kw):
    st = two_bodies(**kw)
    e0 = oracle.energy(st, G, 1.0)
    o = {k: v.copy() for k, v in st.items()}
    r = oracle.step_coll(o, G, 1.0, 6.0, 3.0, 0.4, 1, 1, rk_steps=2000)
    e1 = oracle.energy(o, G, 1.0)
    lost = sum(c[2] for c in r[3])
    assert abs(e1 - e0) > 1e-6 * abs(e0)
    assert abs(e1 + lost - e0) < 1e-9 * abs(e0)


def test_no_radii_no_mergers():
    st = two_bodies(R=0.0)
    o = {k: v.copy() for k, v in st.items()}
    r = oracle.step_coll(o, G, 1.0, 6.0, 3.0, 0.4, 1, 1, rk_steps=2000)
    assert r[3] == [] and np.all(o["m"] == st["m"])
