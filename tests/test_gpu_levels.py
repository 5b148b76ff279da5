"""Symplectic levels (Sect. 6.2, higher-level changeover functions; Appendix A,
recursive encounter routine) of genga_step against the oracle's step_levels,
which test_oracle_levels.py pins to the Newtonian three-body problem."""
import numpy as np
import pytest
import torch

import oracle
from encounter_fixture import two_planets
from paper_2201_10058_amd import native as N
from paper_2201_10058_amd import workload as W

pytestmark = pytest.mark.gpu

G = W.GAUSS_G


def _say(*a):
    print(*a, flush=True)


def _cfg(L, s, cap=1 << 16, **kw):
    return N.Config(G=G, slevels=L, substeps=s, level_capacity=cap, **kw)


def _rel(out, ref, keys):
    g = np.stack([out[k] for k in keys])
    r = np.stack([ref[k] for k in keys])
    return np.max(np.abs(g - r)) / np.max(np.abs(r))


@pytest.mark.parametrize("L,s", [(2, 2), (3, 2), (2, 10), (3, 4), (4, 2)])
def test_levels_step_matches_oracle(dev, L, s):
    # 10 steps of the 2,048-body disk: every step's level-0 list against the
    # oracle's brute force on the GPU's own positions and radii, the list
    # sizes of every level against the oracle's trajectory, and the final
    # state against the oracle's trajectory
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = _cfg(L, s)
    ws = N.Workspace(st.n, cfg)
    pl = N.PairList(1 << 16)
    ref = oracle.state_copy(d)
    for k in range(10):
        x0 = {c: st.t[c].cpu().numpy().copy() for c in "xyz"}
        assert N.step(st, cfg, ws, pl) == N.OK
        pi, pj, cnt = pl.result()
        rc = st.t["rc"].cpu().numpy()
        opi, opj, ocnt = oracle.pairs(x0["x"], x0["y"], x0["z"], rc)
        assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)
        counts = N.level_counts(st.n, cfg, ws)
        r = oracle.step_levels(ref, G, 1.0, 6.0, 3.0, 0.4, L, s)
        assert r[5] == 0
        assert np.array_equal(counts, r[4]), (k, counts, r[4])
    out = st.numpy()
    ep, ev = _rel(out, ref, ("x", "y", "z")), _rel(out, ref, ("vx", "vy", "vz"))
    _say(f"levels {L}x{s}: 10 steps, last counts {counts}, position {ep:.2e} velocity {ev:.2e}")
    assert ep < 1e-12 and ev < 1e-12


def test_one_level_is_the_base_step(dev):
    d = W.make_disk(W.DISK_2048)
    a, b = N.State.from_numpy(d), N.State.from_numpy(d)
    ca, cb = N.Config(G=G), _cfg(1, 5, cap=0)
    wa, wb = N.Workspace(a.n, ca), N.Workspace(b.n, cb)
    for _ in range(3):
        assert N.step(a, ca, wa) == N.OK and N.step(b, cb, wb) == N.OK
    for k in a.t:
        assert torch.equal(a.t[k], b.t[k])


def _run_pair(state, L, s, n1, n2, dt=6.0, T=300.0):
    st = N.State.from_numpy(state)
    cfg = _cfg(L, s, cap=64, n1=n1, n2=n2, dt=dt)
    ws = N.Workspace(st.n, cfg)
    ref = oracle.state_copy(state)
    counts = np.zeros(max(L, 1), dtype=np.int64)
    for _ in range(int(round(T / dt))):
        assert N.step(st, cfg, ws) == N.OK
        counts += N.level_counts(st.n, cfg, ws)
        oracle.step_levels(ref, G, 1.0, dt, n1, n2, L, s)
    out = st.numpy()
    return np.stack([out["x"], out["y"], out["z"]], 1), ref, counts


@pytest.mark.parametrize("L,s,n2,bound", [(2, 10, 0.4, 1e-4), (3, 5, 4.0, 1e-5)])
def test_levels_follow_the_newtonian_encounter(dev, L, s, n2, bound):
    # the Sun + two-planet encounter of the oracle pins: the deepest level's
    # radius stays below the closest approach, so the levels integrate the
    # whole pair force and the step follows the Newtonian solution
    state, newton = two_planets(1.03)
    pos, ref, counts = _run_pair(state, L, s, 0.5, n2)
    rpos = np.stack([ref["x"], ref["y"], ref["z"]], 1)
    e_or = np.max(np.abs(pos - rpos))
    e_nw = np.max(np.abs(pos - newton))
    _say(f"encounter {L}x{s} n2={n2}: counts {counts}, vs oracle {e_or:.2e} AU, vs Newton {e_nw:.2e} AU")
    # every level above the deepest holds the pair at times; the deepest
    # (the direct solver's share) never does
    assert np.all(counts[:-1] > 0) and counts[-1] == 0
    # up to 1,250 sub-step drifts (two Kepler formulations that agree to a
    # few 1e-16) through a close encounter: 1e-11 AU against the oracle
    assert e_or < 1e-11
    assert e_nw < bound


def test_levels_overflow_is_reported(dev):
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = _cfg(2, 2, cap=100)
    ws = N.Workspace(st.n, cfg)
    pl = N.PairList(1 << 16)
    x0 = {c: st.t[c].cpu().numpy().copy() for c in "xyz"}
    assert N.step(st, cfg, ws, pl) == N.E_OVERFLOW
    pi, pj, cnt = pl.result()
    rc = st.t["rc"].cpu().numpy()
    opi, opj, ocnt = oracle.pairs(x0["x"], x0["y"], x0["z"], rc)
    # the true count, and the first level_capacity pairs (all the levels saw)
    assert cnt == ocnt > 100
    assert np.array_equal(pi[:100], opi[:100]) and np.array_equal(pj[:100], opj[:100])


def test_levels_graph_replay_bitwise(dev):
    # the levelled step captured once in a hipGraph and replayed, against the
    # same step issued eagerly (every list size lives on the device)
    d = W.make_disk(W.DISK_2048)
    cfg = _cfg(3, 2, flags=N.FLAG_NOSYNC)
    st_g, st_e = N.State.from_numpy(d), N.State.from_numpy(d)
    ws_g, ws_e = N.Workspace(st_g.n, cfg), N.Workspace(st_e.n, cfg)
    pl_g, pl_e = N.PairList(1 << 16), N.PairList(1 << 16)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tmp = N.State.from_numpy(d)
        N.step(tmp, cfg, N.Workspace(tmp.n, cfg), N.PairList(1 << 16))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        N.step(st_g, cfg, ws_g, pl_g)
    torch.cuda.synchronize()
    for k in st_g.t:
        st_g.t[k].copy_(st_e.t[k])
    for rep in range(4):
        g.replay()
        N.step(st_e, cfg, ws_e, pl_e)
        junk = torch.randn(1000, device="cuda").sum()     # unrelated eager work
        torch.cuda.synchronize()
        assert N.read_status(ws_g) == N.OK and N.read_status(ws_e) == N.OK
        for k in ("x", "y", "z", "vx", "vy", "vz", "rc"):
            assert torch.equal(st_g.t[k], st_e.t[k]), (rep, k)
        assert np.array_equal(N.level_counts(st_g.n, cfg, ws_g), N.level_counts(st_e.n, cfg, ws_e))
        del junk


def test_levels_disk65536_one_step(dev):
    # the benchmark's disk, two levels of two sub-steps, one step against the
    # oracle: level-0 list, level sizes and state
    d = W.make_disk(W.DISK_65536)
    st = N.State.from_numpy(d)
    cfg = _cfg(2, 2, cap=1 << 20, m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"])
    ws = N.Workspace(st.n, cfg)
    pl = N.PairList(1 << 20)
    assert N.step(st, cfg, ws, pl) == N.OK
    counts = N.level_counts(st.n, cfg, ws)
    ref = oracle.state_copy(d)
    r = oracle.step_levels(ref, G, d["m_star"], d["dt"], d["n1"], d["n2"], 2, 2, cap=1 << 20)
    pi, pj, cnt = pl.result()
    assert cnt == r[2] and np.array_equal(pi, r[0]) and np.array_equal(pj, r[1])
    assert np.array_equal(counts, r[4])
    out = st.numpy()
    ep, ev = _rel(out, ref, ("x", "y", "z")), _rel(out, ref, ("vx", "vy", "vz"))
    _say(f"disk65536 levels 2x2: counts {counts}, position {ep:.2e} velocity {ev:.2e}")
    assert ep < 1e-13 and ev < 1e-13


def test_tune_levels_picks_the_fastest_that_ran(dev):
    from paper_2201_10058_amd import autotune as AT
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    x0 = st.t["x"].clone()
    cfg = N.Config(G=G, level_capacity=1 << 16)
    cands = [(1, 1), (2, 2), (3, 2), (9, 2)]      # 9 levels: rejected, never runs
    r = AT.tune_levels(st, cfg, cands, steps=2)
    ms = r["ms"]
    _say("level tuner", r)
    assert ms["9x2"] == -1
    ran = {k: v for k, v in ms.items() if v >= 0}
    assert len(ran) == 3
    best = min(ran, key=ran.get)
    assert f"{r['slevels']}x{r['substeps']}" == best
    assert not torch.equal(st.t["x"], x0)        # the tuning steps are steps of the run
