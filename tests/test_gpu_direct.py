"""Direct solver of genga_step (close-encounter groups + Bulirsch-Stoer;
Sect. 2, Sect. 6.1, Appendix A) against the oracle's grouping and RK4 group
flow (pinned in test_oracle_direct.py) and the Newtonian three-body problem."""
import numpy as np
import pytest
import torch

import oracle
from encounter_fixture import ring_chain, two_planets
from paper_2201_10058_amd import native as N
from paper_2201_10058_amd import workload as W

pytestmark = pytest.mark.gpu

G = W.GAUSS_G


def _say(*a):
    print(*a, flush=True)


def _cfg(L, s, **kw):
    return N.Config(G=G, slevels=L, substeps=s, level_capacity=1 << 16, direct=1, **kw)


def _rel(out, ref, keys):
    g = np.stack([out[k] for k in keys])
    r = np.stack([ref[k] for k in keys])
    return np.max(np.abs(g - r)) / np.max(np.abs(r))


@pytest.mark.parametrize("L,s", [(3, 4), (2, 10), (4, 2)])
def test_direct_step_matches_oracle(dev, L, s):
    # 5 steps of the 2,048-body disk with the deepest level's groups
    # integrated: groups, largest group, level list sizes and the state
    # against the oracle (its RK4 flow in fine steps)
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = _cfg(L, s)
    ws = N.Workspace(st.n, cfg)
    ref = oracle.state_copy(d)
    for k in range(5):
        assert N.step(st, cfg, ws) == N.OK
        counts = N.level_counts(st.n, cfg, ws)
        gs = N.group_stats(st.n, cfg, ws)
        r = oracle.step_direct(ref, G, 1.0, 6.0, 3.0, 0.4, L, s, rk_steps=400)
        assert r[6] == 0
        assert np.array_equal(counts, r[4]), (k, counts, r[4])
        assert gs == r[5], (k, gs, r[5])
    out = st.numpy()
    ep, ev = _rel(out, ref, ("x", "y", "z")), _rel(out, ref, ("vx", "vy", "vz"))
    _say(f"direct {L}x{s}: groups {gs}, position {ep:.2e} velocity {ev:.2e}")
    assert gs[0] > 0
    assert ep < 1e-11 and ev < 1e-11


@pytest.mark.parametrize("L,s", [(1, 1), (2, 10)])
def test_direct_follows_a_close_encounter(dev, L, s):
    # closest approach at a third of the Hill radius (the oracle pin's case)
    state, newton = two_planets(1.004)
    st = N.State.from_numpy(state)
    cfg = N.Config(G=G, slevels=L, substeps=s, level_capacity=64, direct=1, n1=0.5, n2=0.4)
    ws = N.Workspace(st.n, cfg)
    ref = oracle.state_copy(state)
    groups = 0
    for _ in range(50):
        assert N.step(st, cfg, ws) == N.OK
        groups += N.group_stats(st.n, cfg, ws)[0]
        oracle.step_direct(ref, G, 1.0, 6.0, 0.5, 0.4, L, s, rk_steps=4000)
    out = st.numpy()
    pos = np.stack([out["x"], out["y"], out["z"]], 1)
    rpos = np.stack([ref["x"], ref["y"], ref["z"]], 1)
    e_or, e_nw = np.abs(pos - rpos).max(), np.abs(pos - newton).max()
    _say(f"direct encounter {L}x{s}: groups {groups}, vs oracle {e_or:.2e} AU, vs Newton {e_nw:.2e} AU")
    assert groups > 0
    assert e_nw < 1e-4
    assert e_or < 1e-8


@pytest.mark.parametrize("n", [230, 300, 500])
def test_direct_group_of_hundreds(dev, n):
    # one group of n bodies (a ring whose neighbours are inside each other's
    # critical radius): the 256- and 512-thread Bulirsch-Stoer classes
    # against the oracle's RK4 group flow
    ring = ring_chain(n)
    st = N.State.from_numpy(ring)
    cfg = N.Config(G=G, slevels=1, substeps=1, level_capacity=4 * n, direct=1, n1=3.0, n2=0.0)
    ws = N.Workspace(st.n, cfg)
    ref = oracle.state_copy(ring)
    for _ in range(2):
        assert N.step(st, cfg, ws) == N.OK
        gs = N.group_stats(st.n, cfg, ws)
        r = oracle.step_direct(ref, G, 1.0, 6.0, 3.0, 0.0, 1, 1, rk_steps=200)
        assert r[6] == 0 and gs == r[5] == (1, n), (gs, r[5])
    out = st.numpy()
    ep, ev = _rel(out, ref, ("x", "y", "z")), _rel(out, ref, ("vx", "vy", "vz"))
    _say(f"group of {n}: position {ep:.2e} velocity {ev:.2e}")
    assert ep < 1e-11 and ev < 1e-11


@pytest.mark.parametrize("n", [40, 100])
def test_direct_small_ring_members_over_several_waves(dev, n):
    # Sect. 6.1's ring of n bodies, each meeting its 8 nearest neighbours: one
    # group that the 512-thread class spreads over 8 waves per member (up to
    # 64 bodies) or 4 (up to 128), each wave summing a share of the partners;
    # against the oracle's RK4 group flow
    d = W.make_bs_ring(n)
    ring = {k: d[k] for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
    st = N.State.from_numpy(ring)
    cfg = N.Config(G=d["G"], m_star=1.0, dt=d["dt"], n1=d["n1"], n2=0.0, slevels=1, substeps=1,
                   direct=1, level_capacity=16 * n)
    ws = N.Workspace(st.n, cfg)
    ref = oracle.state_copy(ring)
    for _ in range(2):
        assert N.step(st, cfg, ws) == N.OK
        gs = N.group_stats(st.n, cfg, ws)
        r = oracle.step_direct(ref, d["G"], 1.0, d["dt"], d["n1"], 0.0, 1, 1, rk_steps=200)
        assert r[6] == 0 and gs == r[5] == (1, n), (gs, r[5])
    out = st.numpy()
    ep, ev = _rel(out, ref, ("x", "y", "z")), _rel(out, ref, ("vx", "vy", "vz"))
    _say(f"ring of {n}: position {ep:.2e} velocity {ev:.2e}")
    assert ep < 1e-11 and ev < 1e-11


def test_direct_disk2048_one_level(dev):
    # without levels the 2,048-body disk's level-0 list forms groups of up to
    # 337 bodies, all within the direct solver's reach
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = _cfg(1, 1)
    ws = N.Workspace(st.n, cfg)
    ref = oracle.state_copy(d)
    assert N.step(st, cfg, ws) == N.OK
    gs = N.group_stats(st.n, cfg, ws)
    r = oracle.step_direct(ref, G, 1.0, 6.0, 3.0, 0.4, 1, 1, rk_steps=200)
    assert r[6] == 0 and gs == r[5], (gs, r[5])
    out = st.numpy()
    ep, ev = _rel(out, ref, ("x", "y", "z")), _rel(out, ref, ("vx", "vy", "vz"))
    _say(f"disk2048 one level: groups {gs}, position {ep:.2e} velocity {ev:.2e}")
    assert gs[1] > 256
    assert ep < 1e-11 and ev < 1e-11


@pytest.mark.parametrize("L,s", [(1, 1), (2, 2)])
def test_direct_grid_group_ring1024(dev, L, s):
    # Sect. 6.1's ring test: 1,024 bodies, each inside the critical radius of
    # its nearest neighbours, form one group; more than one workgroup holds,
    # so all workgroups of the grid solver integrate it together (with two
    # levels, over each level-1 sub-step with both levels' weights)
    n = 1024
    ring = ring_chain(n)
    st = N.State.from_numpy(ring)
    cfg = N.Config(G=G, slevels=L, substeps=s, level_capacity=16 * n, direct=1, n1=3.0, n2=0.0)
    ws = N.Workspace(st.n, cfg)
    ref = oracle.state_copy(ring)
    _say(f"ring {n} {L}x{s}: grid solver step")
    assert N.step(st, cfg, ws) == N.OK
    gs = N.group_stats(st.n, cfg, ws)
    r = oracle.step_direct(ref, G, 1.0, 6.0, 3.0, 0.0, L, s, rk_steps=200)
    assert r[6] == 0 and gs == r[5] and gs[1] == n, (gs, r[5])
    out = st.numpy()
    ep, ev = _rel(out, ref, ("x", "y", "z")), _rel(out, ref, ("vx", "vy", "vz"))
    _say(f"ring {n} {L}x{s}: groups {gs}, position {ep:.2e} velocity {ev:.2e}")
    assert ep < 1e-11 and ev < 1e-11


def test_direct_disk4096_one_level_grid_group(dev):
    # without levels the 4,096-body disk's level-0 list links 1,916 bodies
    # into one group (379 groups in all): the grid solver with the members in
    # spatial order and tile culling, against the oracle's all-pairs flow
    d = W.make_disk(W.DISK_ADJOINT)
    st = N.State.from_numpy(d)
    cfg = _cfg(1, 1)
    ws = N.Workspace(st.n, cfg)
    ref = oracle.state_copy(d)
    _say("disk4096 one level: grid solver step")
    assert N.step(st, cfg, ws) == N.OK
    gs = N.group_stats(st.n, cfg, ws)
    r = oracle.step_direct(ref, G, 1.0, 6.0, 3.0, 0.4, 1, 1, rk_steps=200)
    assert r[6] == 0 and gs == r[5], (gs, r[5])
    out = st.numpy()
    ep, ev = _rel(out, ref, ("x", "y", "z")), _rel(out, ref, ("vx", "vy", "vz"))
    _say(f"disk4096 one level: groups {gs}, position {ep:.2e} velocity {ev:.2e}")
    assert gs[1] > 512
    assert ep < 1e-11 and ev < 1e-11


def test_oversized_group_is_reported(dev):
    # a ring of 70,000 bodies in one chain (m = 3e-12: 3 R_H = 3e-4 AU
    # against a spacing of 9.0e-5 AU): more than GENGA_GROUP_MAX = 65,536
    n = 70000
    ring = ring_chain(n, m=3e-12)
    st = N.State.from_numpy(ring)
    cfg = N.Config(G=G, slevels=1, substeps=1, level_capacity=1 << 19, direct=1, n1=3.0, n2=0.0)
    ws = N.Workspace(st.n, cfg)
    assert N.step(st, cfg, ws) == N.E_GROUP


def test_direct_graph_replay_bitwise(dev):
    d = W.make_disk(W.DISK_2048)
    cfg = _cfg(3, 4, flags=N.FLAG_NOSYNC)
    st_g, st_e = N.State.from_numpy(d), N.State.from_numpy(d)
    ws_g, ws_e = N.Workspace(st_g.n, cfg), N.Workspace(st_e.n, cfg)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tmp = N.State.from_numpy(d)
        N.step(tmp, cfg, N.Workspace(tmp.n, cfg))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        N.step(st_g, cfg, ws_g)
    torch.cuda.synchronize()
    for k in st_g.t:
        st_g.t[k].copy_(st_e.t[k])
    for rep in range(3):
        g.replay()
        N.step(st_e, cfg, ws_e)
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert N.read_status(ws_g) == N.OK and N.read_status(ws_e) == N.OK
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert torch.equal(st_g.t[k], st_e.t[k]), (rep, k)
        assert N.group_stats(st_g.n, cfg, ws_g) == N.group_stats(st_e.n, cfg, ws_e)
        del junk


def test_direct_cuts_the_energy_error(dev):
    d = W.make_disk(W.DISK_2048)
    err = {}
    for direct in (0, 1):
        st = N.State.from_numpy(d)
        cfg = N.Config(G=G, slevels=3, substeps=4, level_capacity=1 << 16, direct=direct)
        ws = N.Workspace(st.n, cfg)
        E0 = float(N.energy(st, cfg, ws)[0].item())
        e = 0.0
        for _ in range(40):
            assert N.step(st, cfg, ws) == N.OK
            e = max(e, abs(float(N.energy(st, cfg, ws)[0].item()) - E0) / abs(E0))
        err[direct] = e
    _say("energy error over 40 steps, 3 x 4 levels: without / with the direct solver", err)
    assert err[1] < 0.1 * err[0]


@pytest.mark.parametrize("n", [20000, 40000])
def test_grid_solver_keeps_the_ring_symmetric(dev, n):
    # Sect. 6.1's ring at sizes whose group the grid solver splits over 4
    # waves per tile (20,000 bodies) and over 2 (40,000) on the MI355X's 512
    # resident workgroups (one wave per tile needs more than 2,048 tiles of 64
    # there, beyond the 65,536-body limit): the ring is
    # invariant under rotation by 2 pi / n, so after a step every body must
    # have the same radius, radial and tangential velocity and angle advance
    # up to rounding.  A partner lost or counted twice at a tile or share
    # boundary moves the bodies there by ~1e-7 AU; the oracle cannot
    # integrate a group this large in seconds, the symmetry holds at any size.
    d = W.make_bs_ring(n)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=d["G"], m_star=1.0, dt=d["dt"], n1=d["n1"], n2=0.0, slevels=1, substeps=1,
                   direct=1, level_capacity=16 * n)
    ws = N.Workspace(st.n, cfg)
    _say(f"ring {n}: grid solver step")
    assert N.step(st, cfg, ws) == N.OK
    assert N.group_stats(st.n, cfg, ws) == (1, n)
    out = st.numpy()
    th0 = 2 * np.pi * np.arange(n) / n
    r = np.hypot(out["x"], out["y"])
    dth = np.angle(np.exp(1j * (np.arctan2(out["y"], out["x"]) - th0)))
    c, s = np.cos(th0 + dth), np.sin(th0 + dth)
    vr = out["vx"] * c + out["vy"] * s
    vt = -out["vx"] * s + out["vy"] * c
    spread = {k: float(np.ptp(v)) for k, v in (("r", r), ("angle", dth), ("v_r", vr), ("v_t", vt))}
    _say(f"ring {n}: spread over the bodies {spread}, mean angle advance {dth.mean():.6f}")
    assert dth.mean() > 0.05                         # the ring moved along its orbit
    assert spread["r"] < 1e-12 and spread["angle"] < 1e-12
    assert spread["v_t"] < 1e-11 * np.abs(vt).mean() and spread["v_r"] < 1e-13
    assert np.all(np.abs(out["z"]) == 0.0)


def test_grid_solver_two_groups_in_one_launch(dev):
    # two rings of 600 bodies at 1.0 and 1.6 AU (0.6 AU apart, far beyond
    # their 0.03 and 0.05 AU critical radii): two groups of more than 512
    # bodies, which the grid solver's one launch integrates one after the
    # other, reusing its scratch
    r1, r2 = ring_chain(600, a=1.0), ring_chain(600, a=1.6)
    d = {k: np.concatenate([r1[k], r2[k]]) for k in r1}
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G, slevels=1, substeps=1, level_capacity=1 << 14, direct=1, n1=3.0, n2=0.0)
    ws = N.Workspace(st.n, cfg)
    ref = oracle.state_copy(d)
    _say("two rings of 600: grid solver step")
    assert N.step(st, cfg, ws) == N.OK
    gs = N.group_stats(st.n, cfg, ws)
    r = oracle.step_direct(ref, G, 1.0, 6.0, 3.0, 0.0, 1, 1, rk_steps=200)
    assert r[6] == 0 and gs == r[5] == (2, 600), (gs, r[5])
    out = st.numpy()
    ep, ev = _rel(out, ref, ("x", "y", "z")), _rel(out, ref, ("vx", "vy", "vz"))
    _say(f"two rings of 600: position {ep:.2e} velocity {ev:.2e}")
    assert ep < 1e-11 and ev < 1e-11
