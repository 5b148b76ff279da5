"""Energy bookkeeping (genga_energy) and the energy drift of the mixed path.

* genga_energy against the oracle's long-double energy (total, and the pair
  potential alone with v = 0 and a negligible central mass);
* the 10^4-step energy drift of the mixed-precision step on the 16,384-body
  disk against the same drift of the FP64 step, started from the same state.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2201_10058_amd import native as N
from paper_2201_10058_amd import workload as W

pytestmark = pytest.mark.gpu

G = W.GAUSS_G


def _say(*a):
    print(*a, flush=True)


def _energy(d, m_star=1.0):
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G, m_star=m_star)
    ws = N.Workspace(st.n, cfg)
    e = N.energy(st, cfg, ws).cpu().numpy()
    return e, N.read_status(ws)


@pytest.mark.parametrize("which", ["disk2048", "cloud700", "disk65536"])
def test_energy_matches_oracle(dev, which):
    if which == "disk2048":
        d = W.make_disk(W.DISK_2048)
    elif which == "cloud700":
        d = W.random_cloud(700, seed=31)
    else:
        d = W.make_disk(W.DISK_65536)
    e, code = _energy(d)
    assert code == N.OK
    ref = oracle.energy(d, G, 1.0)
    _say(which, "E", e[0], "oracle", ref, "rel", abs(e[0] - ref) / abs(ref))
    assert abs(e[0] - ref) <= 1e-13 * abs(ref)
    # single-body parts, summed plainly in binary64 here
    m = d["m"]
    T = 0.5 * np.sum(m * (d["vx"] ** 2 + d["vy"] ** 2 + d["vz"] ** 2))
    Us = -G * np.sum(m / np.sqrt(d["x"] ** 2 + d["y"] ** 2 + d["z"] ** 2))
    P = np.array([np.sum(m * d[k]) for k in ("vx", "vy", "vz")])
    C = P @ P / 2.0
    assert abs(e[1] - T) <= 1e-13 * abs(T)
    assert abs(e[2] - Us) <= 1e-13 * abs(Us)
    assert abs(e[4] - C) <= 1e-12 * abs(C)
    assert e[0] == pytest.approx(e[1] + e[2] + e[3] + e[4], rel=1e-15)


@pytest.mark.parametrize("which", ["disk2048", "cloud700"])
def test_pair_potential_matches_oracle(dev, which):
    # with v = 0 and m_star -> 1e-300 the oracle's energy is the pair sum alone
    d = W.make_disk(W.DISK_2048) if which == "disk2048" else W.random_cloud(700, seed=32)
    d = dict(d)
    for k in ("vx", "vy", "vz"):
        d[k] = np.zeros_like(d[k])
    e, code = _energy(d, m_star=1e-300)
    assert code == N.OK
    ref = oracle.energy(d, G, 1e-300)
    _say(which, "U", e[3], "oracle", ref, "rel", abs(e[3] - ref) / abs(ref))
    assert abs(e[3] - ref) <= 1e-13 * abs(ref)


def test_energy_coincident_bodies_status(dev):
    d = W.random_cloud(300, seed=33)
    d = dict(d)
    for k in ("x", "y", "z"):
        d[k] = d[k].copy()
        d[k][200] = d[k][17]
    _, code = _energy(d)
    assert code == N.E_NONFINITE


def test_energy_drift_mixed_vs_fp64_disk16384(dev):
    """10^4 base steps of 6 days on the 16,384-body disk in FP64 and in the
    mixed path from the same initial state; energy every 1000 steps."""
    d = W.make_disk(W.DISK_MIXED[16384])
    steps, every = 10_000, 1000
    E0_oracle = oracle.energy(d, G, d["m_star"])
    drift = {}
    for prec in (N.FP64, N.MIXED):
        st = N.State.from_numpy(d)
        cfg = N.Config(G=G, m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"], precision=prec,
                       flags=N.FLAG_NOSYNC)
        ws = N.Workspace(st.n, cfg)
        Es = [N.energy(st, cfg, ws).clone()]
        for k in range(steps):
            N.step(st, cfg, ws)
            if (k + 1) % every == 0:
                Es.append(N.energy(st, cfg, ws).clone())
        assert N.read_status(ws) == N.OK
        E = torch.stack(Es).cpu().numpy()[:, 0]
        if prec == N.FP64:
            assert abs(E[0] - E0_oracle) <= 1e-13 * abs(E0_oracle)
            Efinal_oracle = oracle.energy(st.numpy(), G, d["m_star"])
            assert abs(E[-1] - Efinal_oracle) <= 1e-13 * abs(Efinal_oracle)
        drift[prec] = (E - E[0]) / abs(E[0])
        _say("precision", prec, "relative energy drift every 1000 steps", drift[prec].tolist())
    diff = np.max(np.abs(drift[N.MIXED] - drift[N.FP64]))
    _say("max |drift_mixed - drift_fp64|", diff, "max |drift_fp64|", np.max(np.abs(drift[N.FP64])))
    assert np.all(np.isfinite(drift[N.MIXED]))
    assert diff <= 1e-9


def test_energy_k_matches_oracle(dev):
    # E_K of the 2,048-body disk after five steps, with the radii of the last
    # step, against the oracle's (Simpson) changeover potential
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G)
    ws = N.Workspace(st.n, cfg)
    for _ in range(5):
        assert N.step(st, cfg, ws) == N.OK
    pl = N.PairList(1 << 16)
    out = N.energy_k(st, cfg, ws, pl).cpu().numpy()
    assert N.read_status(ws) == N.OK
    s = st.numpy()
    ek = oracle.energy_k(s, s["rc"], G, 1.0)
    e = oracle.energy(s, G, 1.0)
    _say("E_K", out[5], ek, "E_K - E", out[5] - out[0], ek - e, "pairs", int(pl.count.item()))
    assert abs(out[5] - ek) <= 1e-13 * abs(ek)
    assert abs((out[5] - out[0]) - (ek - e)) <= 1e-9 * abs(ek - e)
    assert ek - e != 0.0


def test_fixed_rc_map_conserves_e_k_on_gpu(dev):
    # the oracle pin's close pass on the GPU operators with rc held fixed
    from encounter_fixture import two_planets
    state, _ = two_planets(1.01)
    st = N.State.from_numpy(state, rc=np.array([0.04, 0.04]))
    cfg = N.Config(G=G)
    ws = N.Workspace(st.n, cfg)
    pl = N.PairList(16)
    e0 = N.energy_k(st, cfg, ws, pl).cpu().numpy()
    de = dk = 0.0
    for _ in range(50):
        N.kick(st, cfg, ws, 3.0)
        N.hc(st, cfg, ws, 3.0)
        N.drift(st, cfg, ws, 6.0)
        N.hc(st, cfg, ws, 3.0)
        N.kick(st, cfg, ws, 3.0)
        e = N.energy_k(st, cfg, ws, pl).cpu().numpy()
        de = max(de, abs(e[0] - e0[0]) / abs(e0[0]))
        dk = max(dk, abs(e[5] - e0[5]) / abs(e0[5]))
    assert N.read_status(ws) == N.OK
    _say("fixed-rc close pass: max |dE|/E", de, "max |dE_K|/E_K", dk)
    assert dk < 0.01 * de
