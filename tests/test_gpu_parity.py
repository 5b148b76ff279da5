"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: relative error per acceleration <= 1e-12 against the oracle's
compensated long-double sum (FP64 path); encounter lists bit-exact given the
same positions and critical radii; O(N) operators per body as stated at each
test.
"""
import numpy as np
import pytest
import torch

import oracle
import oracle_refs as R
from paper_2201_10058_amd import native as N
from paper_2201_10058_amd import workload as W

pytestmark = pytest.mark.gpu

G = W.GAUSS_G
ACC_TOL = 1e-12


def _say(*a):
    print(*a, flush=True)


def _rel_err(a_gpu, a_ref):
    return np.linalg.norm(a_gpu - a_ref, axis=0) / np.linalg.norm(a_ref, axis=0)


def _oracle_acc(d, rc, rows=None):
    ax, ay, az, st = oracle.kick_acc(d["x"], d["y"], d["z"], d["m"], rc, G, rows=rows, precise=True)
    assert st == 0
    return np.stack([ax, ay, az])


def _run_kick(d, rc, cfg, h=0.0, cap=None, pairs=True):
    st = N.State.from_numpy(d, rc=rc)
    ws = N.Workspace(st.n, cfg)
    pl = None
    if pairs:
        if cap is None:
            cap = max(16, oracle.pairs(d["x"], d["y"], d["z"], rc, cap=0)[2])
        pl = N.PairList(cap)
    a = N.kick(st, cfg, ws, h, acc=True, pairs=pl)
    torch.cuda.synchronize()
    code = N.read_status(ws)
    return a.cpu().numpy(), (pl.result() if pl else None), code, st


def _disk_rc(d, n2=0.4):
    return oracle.rcrit(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["m"], 1.0, 6.0, 3.0, n2)


@pytest.mark.parametrize("ipt,slices", [(1, 0), (2, 0), (1, 1), (2, 3)])
def test_kick_disk2048(dev, ipt, slices):
    d = W.make_disk(W.DISK_2048)
    rc = _disk_rc(d)
    _say("kick disk2048", ipt, slices)
    cfg = N.Config(G=G, ipt=ipt, slices=slices)
    a, (pi, pj, cnt), code, _ = _run_kick(d, rc, cfg)
    assert code == N.OK
    ref = _oracle_acc(d, rc)
    err = _rel_err(a, ref)
    _say("max rel err", err.max())
    assert err.max() <= ACC_TOL
    opi, opj, ocnt = oracle.pairs(d["x"], d["y"], d["z"], rc)
    assert cnt == ocnt
    assert np.array_equal(pi, opi) and np.array_equal(pj, opj)


@pytest.mark.parametrize("seed", range(12))
def test_kick_random_small(dev, seed):
    rng = np.random.default_rng(100 + seed)
    n = int([1, 2, 3, 63, 64, 65, 127, 200, 255, 256, 257, 300][seed])
    d = W.random_cloud(n, seed=seed, rc_scale=float(rng.uniform(0.05, 0.6)))
    rc = d["rc"]
    ipt = 1 + seed % 2
    slices = [0, 1, 2, 3][seed % 4]
    _say("random", n, ipt, slices)
    a, (pi, pj, cnt), code, _ = _run_kick(d, rc, N.Config(G=G, ipt=ipt, slices=slices))
    assert code == N.OK
    if n > 1:
        err = _rel_err(a, _oracle_acc(d, rc))
        assert err.max() <= ACC_TOL
    else:
        assert np.all(a == 0.0)
    opi, opj, ocnt = oracle.pairs(d["x"], d["y"], d["z"], rc)
    assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)


def test_kick_updates_velocity(dev):
    d = W.make_disk(W.DISK_2048)
    rc = _disk_rc(d)
    h = 3.0
    a, _, code, st = _run_kick(d, rc, N.Config(G=G), h=h, pairs=False)
    assert code == N.OK
    out = st.numpy()
    ref = _oracle_acc(d, rc)
    for c, k in enumerate(("vx", "vy", "vz")):
        dv = out[k] - d[k]
        assert np.max(np.abs(dv - h * ref[c])) <= 1e-12 * np.max(np.abs(h * ref[c])) + 4e-16 * np.max(np.abs(d[k]))


@pytest.mark.parametrize("n", [10, 1000, 10007])
def test_ring_fixture_pairs(dev, n):
    # the paper's ring test (Sect. 6.1): every body meets its 4 neighbours on
    # each side.  At 10007 rows a wave holds 256 pairs and overflows its
    # staging segment, which exercises the exact recompute path.
    ring = W.make_ring(n)
    _say("ring", n)
    a, (pi, pj, cnt), code, _ = _run_kick(ring, ring["rc"], N.Config(G=G), cap=4 * n + 8)
    assert code == N.OK
    assert cnt == 4 * n
    opi, opj, ocnt = oracle.pairs(ring["x"], ring["y"], ring["z"], ring["rc"])
    assert np.array_equal(pi, opi) and np.array_equal(pj, opj)
    err = _rel_err(a, _oracle_acc(ring, ring["rc"]))
    assert err.max() <= ACC_TOL


def test_pair_overflow_reports_true_count(dev):
    d = W.make_disk(W.DISK_2048)
    rc = _disk_rc(d)
    opi, opj, ocnt = oracle.pairs(d["x"], d["y"], d["z"], rc)
    cap = ocnt // 3
    _, (pi, pj, cnt), code, _ = _run_kick(d, rc, N.Config(G=G), cap=cap)
    assert code == N.E_OVERFLOW
    assert cnt == ocnt
    assert np.array_equal(pi, opi[:cap]) and np.array_equal(pj, opj[:cap])
    # zero capacity is legal: only the count is produced
    _, (pi0, pj0, cnt0), code0, _ = _run_kick(d, rc, N.Config(G=G), cap=0)
    assert cnt0 == ocnt and code0 == N.E_OVERFLOW


def test_coincident_and_invalid_rc(dev):
    d = W.random_cloud(100, seed=1, rc_scale=0.1)
    d["x"][7] = d["x"][3]; d["y"][7] = d["y"][3]; d["z"][7] = d["z"][3]
    _, _, code, _ = _run_kick(d, d["rc"], N.Config(G=G), cap=10000)
    assert code == N.E_NONFINITE
    d2 = W.random_cloud(100, seed=2, rc_scale=0.1)
    rc = d2["rc"].copy()
    rc[5] = -1.0
    _, _, code2, _ = _run_kick(d2, rc, N.Config(G=G), cap=10000)
    assert code2 == N.E_RCRIT


def test_encounter_pairs_standalone(dev):
    d = W.random_cloud(3000, seed=4, rc_scale=0.05)
    rc = d["rc"]
    st = N.State.from_numpy(d, rc=rc)
    cfg = N.Config(G=G)
    ws = N.Workspace(st.n, cfg)
    opi, opj, ocnt = oracle.pairs(d["x"], d["y"], d["z"], rc)
    pl = N.PairList(ocnt + 5)
    N.encounter_pairs(st, cfg, ws, pl)
    torch.cuda.synchronize()
    assert N.read_status(ws) == N.OK
    pi, pj, cnt = pl.result()
    assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)


def test_kick_deterministic(dev):
    d = W.make_disk(W.DISK_2048)
    rc = _disk_rc(d)
    a1, p1, _, _ = _run_kick(d, rc, N.Config(G=G))
    a2, p2, _, _ = _run_kick(d, rc, N.Config(G=G))
    assert np.array_equal(a1, a2)
    assert np.array_equal(p1[0], p2[0]) and np.array_equal(p1[1], p2[1])


# ---------------------------------------------------------------------------
# O(N) operators
# ---------------------------------------------------------------------------
def test_rcrit_matches_oracle(dev):
    d = W.make_disk(W.DISK_2048)
    for n2 in (0.4, 0.0):
        st = N.State.from_numpy(d)
        cfg = N.Config(G=G, n2=n2)
        ws = N.Workspace(st.n, cfg)
        N.rcrit(st, cfg, ws)
        torch.cuda.synchronize()
        assert N.read_status(ws) == N.OK
        rc = st.t["rc"].cpu().numpy()
        ref = _disk_rc(d, n2)
        assert np.max(np.abs(rc - ref) / ref) <= 4e-16


def test_hc_matches_oracle(dev):
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G)
    ws = N.Workspace(st.n, cfg)
    N.hc(st, cfg, ws, 3.0)
    out = st.numpy()
    ref = oracle.state_copy(d)
    oracle.hc(ref, 1.0, 3.0)
    for k in ("x", "y", "z"):
        assert np.max(np.abs(out[k] - ref[k])) <= 2.3e-16 * np.max(np.abs(ref[k]))


@pytest.mark.parametrize("dt", [6.0, -6.0, 250.0])
def test_drift_matches_oracle(dev, dt):
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G)
    ws = N.Workspace(st.n, cfg)
    N.drift(st, cfg, ws, dt)
    torch.cuda.synchronize()
    assert N.read_status(ws) == N.OK
    out = st.numpy()
    ref = oracle.state_copy(d)
    assert oracle.drift(ref, G * 1.0, dt) == 0
    pos = np.stack([out[k] for k in "xyz"]); rpos = np.stack([ref[k] for k in "xyz"])
    vel = np.stack([out[k] for k in ("vx", "vy", "vz")]); rvel = np.stack([ref[k] for k in ("vx", "vy", "vz")])
    ep = np.linalg.norm(pos - rpos, axis=0) / np.linalg.norm(rpos, axis=0)
    ev = np.linalg.norm(vel - rvel, axis=0) / np.linalg.norm(rvel, axis=0)
    _say("drift", dt, ep.max(), ev.max())
    assert ep.max() <= 1e-13 * max(1.0, abs(dt) / 6.0) and ev.max() <= 1e-13 * max(1.0, abs(dt) / 6.0)


def test_drift_hyperbolic_and_eccentric(dev):
    mu = G
    rng = np.random.default_rng(3)
    n = 500
    r = rng.uniform(0.3, 3.0, n)
    th = rng.uniform(0, 2 * np.pi, n)
    vcirc = np.sqrt(mu / r)
    fac = rng.uniform(0.2, 1.9, n)          # bound and unbound orbits
    d = dict(x=r * np.cos(th), y=r * np.sin(th), z=rng.normal(0, 0.01, n),
             vx=-fac * vcirc * np.sin(th) + rng.normal(0, 0.1, n) * vcirc,
             vy=fac * vcirc * np.cos(th), vz=rng.normal(0, 0.02, n) * vcirc, m=np.zeros(n))
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G)
    ws = N.Workspace(n, cfg)
    N.drift(st, cfg, ws, 20.0)
    torch.cuda.synchronize()
    assert N.read_status(ws) == N.OK
    out = st.numpy()
    ref = oracle.state_copy(d)
    assert oracle.drift(ref, mu, 20.0) == 0
    pos = np.stack([out[k] for k in "xyz"]); rpos = np.stack([ref[k] for k in "xyz"])
    ep = np.linalg.norm(pos - rpos, axis=0) / np.linalg.norm(rpos, axis=0)
    _say("drift mixed orbits", ep.max())
    assert ep.max() <= 1e-12


# ---------------------------------------------------------------------------
# Step
# ---------------------------------------------------------------------------
def test_step_matches_oracle_and_pairs_per_step(dev):
    # the 2,048-body disk for 100 base steps of 6 days: the encounter list of
    # every step is bit-exact against the oracle's brute force on the GPU's
    # own positions and r_crit, and the final state follows the oracle's own
    # 100-step trajectory (a 1e-15 perturbation grows to ~1e-13 in 100 steps)
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G)
    ws = N.Workspace(st.n, cfg)
    ref = oracle.state_copy(d)
    pl = N.PairList(20000)
    for k in range(100):
        x0 = {c: st.t[c].cpu().numpy().copy() for c in ("x", "y", "z")}
        code = N.step(st, cfg, ws, pl)
        assert code == N.OK
        pi, pj, cnt = pl.result()
        rc = st.t["rc"].cpu().numpy()
        opi, opj, ocnt = oracle.pairs(x0["x"], x0["y"], x0["z"], rc)
        assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)
        oracle.step(ref, G, 1.0, 6.0, 3.0, 0.4)
    out = st.numpy()
    pos = np.stack([out[c] for c in "xyz"]); rpos = np.stack([ref[c] for c in "xyz"])
    vel = np.stack([out[c] for c in ("vx", "vy", "vz")]); rvel = np.stack([ref[c] for c in ("vx", "vy", "vz")])
    ep = np.max(np.abs(pos - rpos)) / np.max(np.abs(rpos))
    ev = np.max(np.abs(vel - rvel)) / np.max(np.abs(rvel))
    _say("100 steps", ep, ev)
    assert ep < 1e-11 and ev < 1e-11


# ---------------------------------------------------------------------------
# Full size (65,536 bodies): every row against the oracle, full pair list
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ipt,flags", [(1, N.FLAG_DIRECTED), (2, N.FLAG_DIRECTED), (0, 0)])
def test_kick_disk65536_all_rows(dev, ipt, flags):
    # one-sided form with 1 and 2 rows per lane, and the default (symmetric);
    # the oracle's compensated kick of all 65,536 rows is computed once
    d, rc = R.disk(W.DISK_65536)
    _say("kick disk65536 ipt", ipt, "flags", flags)
    a, (pi, pj, cnt), code, _ = _run_kick(d, rc, N.Config(G=G, ipt=ipt, flags=flags),
                                          cap=1 << 21)
    assert code == N.OK
    err = R.rel_err(a, R.disk_acc(W.DISK_65536))
    _say(f"all rows: max rel err {err.max():.3e} p99 {np.quantile(err, 0.99):.3e} "
         f"worst row {int(np.argmax(err))}")
    assert err.max() <= ACC_TOL
    # Newton's third law holds for the whole system
    P = (d["m"] * a).sum(axis=1)
    assert np.max(np.abs(P)) <= 1e-13 * (d["m"] * np.abs(a)).sum()
    opi, opj, ocnt = R.disk_pairs(W.DISK_65536)
    assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)


def test_step_pairs_disk65536_every_100_steps(dev):
    # 1000 base steps of the 65,536-body disk; every 100 steps the encounter
    # list of the step (first half kick, positions the step starts from) is
    # compared with the oracle's brute force on the same positions and r_crit
    d = W.make_disk(W.DISK_65536)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G, m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"], flags=N.FLAG_NOSYNC)
    ws = N.Workspace(st.n, cfg)
    pl = N.PairList(1 << 20)
    checked = 0
    for k in range(1000):
        if k % 100 == 0:
            x0 = {c: st.t[c].cpu().numpy().copy() for c in "xyz"}
        N.step(st, cfg, ws, pl)
        if k % 100 == 0:
            assert N.read_status(ws) == N.OK
            pi, pj, cnt = pl.result()
            rc = st.t["rc"].cpu().numpy()
            opi, opj, ocnt = oracle.pairs(x0["x"], x0["y"], x0["z"], rc, cap=1 << 20)
            _say(f"step {k}: {cnt} pairs, oracle {ocnt}")
            assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)
            checked += 1
    assert N.read_status(ws) == N.OK
    assert checked == 10

