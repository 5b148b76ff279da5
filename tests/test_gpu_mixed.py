"""Mixed-precision kick (binary32 pair arithmetic on binary64 differences).

Bar: relative error per acceleration <= 1e-6 for every body against the
oracle's compensated binary64 kick; encounter lists identical to the
oracle's (the encounter test stays in binary64).
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
MIXED_TOL = 1e-6


def _say(*a):
    print(*a, flush=True)


def _kick(d, rc, precision, ipt=0, cap=None, h=0.0, flags=0):
    st = N.State.from_numpy(d, rc=rc)
    cfg = N.Config(G=G, precision=precision, ipt=ipt, flags=flags)
    ws = N.Workspace(st.n, cfg)
    if cap is None:
        cap = max(16, oracle.pairs(d["x"], d["y"], d["z"], rc, cap=0)[2])
    pl = N.PairList(cap)
    a = N.kick(st, cfg, ws, h, acc=True, pairs=pl)
    torch.cuda.synchronize()
    return a.cpu().numpy(), pl.result(), N.read_status(ws), st


def _rel(a, ref):
    return np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)


def _rc(d):
    return oracle.rcrit(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["m"], 1.0, 6.0, 3.0, 0.4)


@pytest.mark.parametrize("ipt,flags", [(1, 0), (2, 0), (0, N.FLAG_SYMMETRIC)])
def test_mixed_disk2048(dev, ipt, flags):
    # one-sided (the default at this size) and symmetric mixed kick
    d = W.make_disk(W.DISK_2048)
    rc = _rc(d)
    a, (pi, pj, cnt), code, _ = _kick(d, rc, N.MIXED, ipt, flags=flags)
    assert code == N.OK
    ax, ay, az, _ = oracle.kick_acc(d["x"], d["y"], d["z"], d["m"], rc, G, precise=True)
    err = _rel(a, np.stack([ax, ay, az]))
    _say("mixed 2048 ipt", ipt, "flags", flags, "max", err.max(), "p99", np.quantile(err, 0.99))
    assert err.max() <= MIXED_TOL
    opi, opj, ocnt = oracle.pairs(d["x"], d["y"], d["z"], rc)
    assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)


@pytest.mark.parametrize("seed", range(12))
def test_mixed_random_small(dev, seed):
    # seeds 0-5 one-sided, 6-11 symmetric (one and several row groups of 512)
    n = [1, 5, 64, 65, 257, 600, 1, 5, 65, 600, 1025, 2500][seed]
    flags = N.FLAG_SYMMETRIC if seed >= 6 else 0
    d = W.random_cloud(n, seed=50 + seed, rc_scale=0.3)
    a, (pi, pj, cnt), code, _ = _kick(d, d["rc"], N.MIXED, 1 + seed % 2, flags=flags)
    assert code == N.OK
    if n > 1:
        ax, ay, az, _ = oracle.kick_acc(d["x"], d["y"], d["z"], d["m"], d["rc"], G, precise=True)
        assert _rel(a, np.stack([ax, ay, az])).max() <= MIXED_TOL
    opi, opj, ocnt = oracle.pairs(d["x"], d["y"], d["z"], d["rc"])
    assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)


@pytest.mark.parametrize("n,flags", [(16384, 0), (32768, 0), (65536, 0), (16384, N.FLAG_DIRECTED)])
def test_mixed_full_disk_all_bodies(dev, n, flags):
    # every body against the oracle's compensated kick, per acceleration; the
    # default (symmetric) form at these sizes, and the one-sided one
    spec = W.DISK_MIXED[n]
    d, rc = R.disk(spec)
    a32, p32, c32, _ = _kick(d, rc, N.MIXED, flags=flags, cap=1 << 21)
    assert c32 == N.OK
    err = _rel(a32, R.disk_acc(spec))
    _say(f"mixed N={n}: max {err.max():.3e} p99 {np.quantile(err, 0.99):.3e} "
         f"p50 {np.median(err):.3e} worst body {int(np.argmax(err))}")
    assert err.max() <= MIXED_TOL
    opi, opj, ocnt = R.disk_pairs(spec)
    assert p32[2] == ocnt and np.array_equal(p32[0], opi) and np.array_equal(p32[1], opj)


def test_mixed_step_pairs_match_oracle(dev):
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G, precision=N.MIXED)
    ws = N.Workspace(st.n, cfg)
    pl = N.PairList(20000)
    for _ in range(5):
        x0 = {c: st.t[c].cpu().numpy().copy() for c in "xyz"}
        assert N.step(st, cfg, ws, pl) == N.OK
        pi, pj, cnt = pl.result()
        opi, opj, ocnt = oracle.pairs(x0["x"], x0["y"], x0["z"], st.t["rc"].cpu().numpy())
        assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)


def _refined_rows(ws) -> int:
    # the third int32 of the workspace: rows of the last mixed kick that were
    # evaluated again in binary64 (documented with genga_kick)
    return int(ws.buf[:12].view(torch.int32)[2].item())


@pytest.mark.parametrize("flags", [0, N.FLAG_SYMMETRIC])
def test_mixed_refines_cancelling_rows(dev, flags):
    # a body close to the centre of a ring of 4,096 equal masses: its terms
    # cancel almost completely (sum |a_ij| / |a_i| ~ 10^3), so the binary32
    # sum alone could not reach 1e-6; the kick must evaluate it in binary64
    ring = W.make_ring(4096)
    d = {k: np.append(ring[k], v) for k, v in
         (("x", 1e-3), ("y", 2e-3), ("z", 1e-4), ("vx", 0.0), ("vy", 0.0), ("vz", 0.0),
          ("m", 1e-9), ("rc", 1e-3))}
    n = d["x"].size
    st = N.State.from_numpy(d, rc=d["rc"])
    cfg = N.Config(G=G, precision=N.MIXED, flags=flags)
    ws = N.Workspace(n, cfg)
    a = N.kick(st, cfg, ws, 0.0, acc=True).cpu().numpy()
    assert N.read_status(ws) == N.OK
    refined = _refined_rows(ws)
    ax, ay, az, _ = oracle.kick_acc(d["x"], d["y"], d["z"], d["m"], d["rc"], G, precise=True)
    ref = np.stack([ax, ay, az])
    err = _rel(a, ref)
    mags = G * d["m"][:-1] / np.sum((np.stack([d[c][:-1] for c in "xyz"]) -
                                    np.array([[d[c][-1]] for c in "xyz"])) ** 2, axis=0)
    kappa = mags.sum() / np.linalg.norm(ref[:, -1])
    _say("ring + centre body: kappa", kappa, "centre error", err[-1], "max", err.max(),
         "refined rows", refined)
    assert kappa > 100
    assert refined >= 1
    assert err[-1] <= 1e-9
    assert err.max() <= MIXED_TOL


def test_mixed_evolved_disk16384(dev):
    # after 100 mixed-precision steps the disk holds bodies with stronger
    # cancellation than the initial state; every body against the oracle's
    # compensated kick on the same state
    d = W.make_disk(W.DISK_MIXED[16384])
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G, m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"], precision=N.MIXED,
                   flags=N.FLAG_NOSYNC)
    ws = N.Workspace(st.n, cfg)
    for _ in range(100):
        N.step(st, cfg, ws)
    assert N.read_status(ws) == N.OK
    N.rcrit(st, cfg, ws)
    a32 = N.kick(st, cfg, ws, 0.0, acc=True).cpu().numpy()
    refined = _refined_rows(ws)
    assert N.read_status(ws) == N.OK
    s = st.numpy()
    rc = st.t["rc"].cpu().numpy()
    ax, ay, az, code = oracle.kick_acc(s["x"], s["y"], s["z"], s["m"], rc, G, precise=True)
    assert code == 0
    err = _rel(a32, np.stack([ax, ay, az]))
    _say(f"evolved mixed: max {err.max():.3e} p99 {np.quantile(err, 0.99):.3e} refined rows {refined}")
    assert err.max() <= MIXED_TOL
    # the refinement is for the strongly cancelling few, not the bulk
    assert 0 < refined < st.n // 10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_step_graph_replay_bitwise(dev, precision):
    # the single-system step captured once in a hipGraph and replayed, against
    # the same step issued eagerly; the mixed step includes the refinement of
    # cancelling rows, whose count lives on the device
    prec = N.FP64 if precision == "fp64" else N.MIXED
    d = W.make_disk(W.DISK_MIXED[16384])
    cfg = N.Config(G=G, m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"], precision=prec,
                   flags=N.FLAG_NOSYNC)
    st_g, st_e = N.State.from_numpy(d), N.State.from_numpy(d)
    ws_g, ws_e = N.Workspace(st_g.n, cfg), N.Workspace(st_e.n, cfg)
    pl_g, pl_e = N.PairList(1 << 18), N.PairList(1 << 18)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tmp = N.State.from_numpy(d)
        N.step(tmp, cfg, N.Workspace(tmp.n, cfg), N.PairList(1 << 18))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        N.step(st_g, cfg, ws_g, pl_g)
    torch.cuda.synchronize()
    for k in st_g.t:
        st_g.t[k].copy_(st_e.t[k])
    refined = []
    for rep in range(4):
        g.replay()
        N.step(st_e, cfg, ws_e, pl_e)
        junk = torch.randn(1000, device="cuda").sum()     # unrelated eager work
        torch.cuda.synchronize()
        refined.append(_refined_rows(ws_e))
        assert N.read_status(ws_g) == N.OK and N.read_status(ws_e) == N.OK
        for k in ("x", "y", "z", "vx", "vy", "vz", "rc"):
            assert torch.equal(st_g.t[k], st_e.t[k]), (rep, k)
        assert int(pl_g.count.item()) == int(pl_e.count.item())
        c = min(int(pl_e.count.item()), pl_e.capacity)
        assert torch.equal(pl_g.i[:c], pl_e.i[:c]) and torch.equal(pl_g.j[:c], pl_e.j[:c])
        del junk
    _say(precision, "rows refined in binary64 per replayed step", refined)
    if prec == N.MIXED:
        assert min(refined) > 0
