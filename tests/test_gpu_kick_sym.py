"""The symmetric binary64 kick (each unordered pair evaluated once and applied
to both bodies, Newton's third law; the pair force of eq. Hb and its weight
K(r; max(rc_i, rc_j)) are symmetric in i and j, Sect. 2 and Sect. 6.2)
against the oracle: accelerations within 1e-12 relative per body, encounter
lists bit-exact (canonical order), on sizes that span one and several row
groups of 512 with ragged tails, and against the one-sided form."""
import numpy as np
import pytest
import torch

import oracle
from paper_2201_10058_amd import native as N
from paper_2201_10058_amd import workload as W

pytestmark = pytest.mark.gpu

G = W.GAUSS_G
ACC_TOL = 1e-12
SYM = N.FLAG_SYMMETRIC
DIR = N.FLAG_DIRECTED


def _say(*a):
    print(*a, flush=True)


def _rel_err(a_gpu, a_ref):
    return np.linalg.norm(a_gpu - a_ref, axis=0) / np.linalg.norm(a_ref, axis=0)


def _oracle_acc(d, rc, rows=None):
    ax, ay, az, st = oracle.kick_acc(d["x"], d["y"], d["z"], d["m"], rc, G, rows=rows, precise=True)
    assert st == 0
    return np.stack([ax, ay, az])


def _run_kick(d, rc, flags, h=0.0, cap=None):
    st = N.State.from_numpy(d, rc=rc)
    cfg = N.Config(G=G, flags=flags)
    ws = N.Workspace(st.n, cfg)
    if cap is None:
        cap = max(16, oracle.pairs(d["x"], d["y"], d["z"], rc, cap=0)[2])
    pl = N.PairList(cap)
    a = N.kick(st, cfg, ws, h, acc=True, pairs=pl)
    torch.cuda.synchronize()
    return a.cpu().numpy(), pl.result(), N.read_status(ws), st


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 200, 1000, 1023, 1024, 1025, 2500, 4097])
def test_sym_random_clouds(dev, n):
    d = W.random_cloud(n, seed=n, rc_scale=0.3)
    rc = d["rc"]
    _say("symmetric kick, random cloud", n)
    a, (pi, pj, cnt), code, _ = _run_kick(d, rc, SYM)
    assert code == N.OK
    if n > 1:
        err = _rel_err(a, _oracle_acc(d, rc))
        assert err.max() <= ACC_TOL, err.max()
    else:
        assert np.all(a == 0.0)
    opi, opj, ocnt = oracle.pairs(d["x"], d["y"], d["z"], rc)
    assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)


def test_sym_disk2048_and_one_sided(dev):
    d = W.make_disk(W.DISK_2048)
    rc = oracle.rcrit(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["m"], 1.0, 6.0, 3.0, 0.4)
    a_s, (pi, pj, cnt), code, _ = _run_kick(d, rc, SYM)
    assert code == N.OK
    ref = _oracle_acc(d, rc)
    err = _rel_err(a_s, ref)
    _say("disk2048 symmetric: max rel err", err.max(), "pairs", cnt)
    assert err.max() <= ACC_TOL
    opi, opj, ocnt = oracle.pairs(d["x"], d["y"], d["z"], rc)
    assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)
    a_d, (qi, qj, qc), code_d, _ = _run_kick(d, rc, DIR)
    assert code_d == N.OK and qc == cnt and np.array_equal(qi, pi) and np.array_equal(qj, pj)
    assert np.max(_rel_err(a_s, a_d)) <= 2 * ACC_TOL
    # Newton's third law: the symmetric form applies each pair force twice
    P = (d["m"] * a_s).sum(axis=1)
    assert np.max(np.abs(P)) <= 1e-14 * (d["m"] * np.abs(a_s)).sum()


def test_sym_outlier_radii_widen_the_wave_bound(dev):
    # The binary64 symmetric kick gates each pair by the largest rc^2 among the
    # wave's rows and the chunk's columns, and takes the exact test in the rare
    # path.  One body in 97 with a critical radius of 0.8 (a unit cloud, the
    # others 0.01) lifts that bound for its waves and chunks, so thousands of
    # pairs outside both of their radii enter the rare path: they must keep the
    # unweighted force and stay out of the list.
    d = W.random_cloud(3000, seed=5, rc_scale=0.01)
    rc = d["rc"].copy()
    rc[::97] = 0.8
    a, (pi, pj, cnt), code, _ = _run_kick(d, rc, SYM)
    assert code == N.OK
    err = _rel_err(a, _oracle_acc(d, rc))
    _say("outlier radii: max rel err", err.max(), "pairs", cnt)
    assert err.max() <= ACC_TOL
    opi, opj, ocnt = oracle.pairs(d["x"], d["y"], d["z"], rc)
    assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)
    a_d, (qi, qj, qc), code_d, _ = _run_kick(d, rc, DIR)
    assert code_d == N.OK and qc == cnt and np.array_equal(qi, pi) and np.array_equal(qj, pj)
    assert np.max(_rel_err(a, a_d)) <= 2 * ACC_TOL
    # the one-sided form with two rows per lane and the pairs-only call share
    # the wave-uniform gate
    st = N.State.from_numpy(d, rc=rc)
    cfg2 = N.Config(G=G, flags=DIR, ipt=2)
    ws2 = N.Workspace(st.n, cfg2)
    pl2 = N.PairList(max(16, ocnt))
    a2 = N.kick(st, cfg2, ws2, 0.0, acc=True, pairs=pl2).cpu().numpy()
    ri, rj, rcnt = pl2.result()
    assert N.read_status(ws2) == N.OK
    assert np.max(_rel_err(a2, _oracle_acc(d, rc))) <= ACC_TOL
    assert rcnt == ocnt and np.array_equal(ri, opi) and np.array_equal(rj, opj)
    for flags in (DIR, SYM):
        cfgp = N.Config(G=G, flags=flags)
        wsp = N.Workspace(st.n, cfgp)
        plp = N.PairList(max(16, ocnt))
        N.encounter_pairs(st, cfgp, wsp, plp)
        si, sj, scnt = plp.result()
        assert N.read_status(wsp) == N.OK
        assert scnt == ocnt and np.array_equal(si, opi) and np.array_equal(sj, opj), flags


def test_sym_ring_overflows_staging(dev):
    # the ring test of Sect. 6.1: every body meets its 4 neighbours on each
    # side; a wave's 128 rows then hold 512 pairs of one tile, more than its
    # staging segment, which takes the exact recompute path
    n = 10007
    ring = W.make_ring(n)
    a, (pi, pj, cnt), code, _ = _run_kick(ring, ring["rc"], SYM, cap=4 * n + 8)
    assert code == N.OK and cnt == 4 * n
    opi, opj, ocnt = oracle.pairs(ring["x"], ring["y"], ring["z"], ring["rc"])
    assert np.array_equal(pi, opi) and np.array_equal(pj, opj)
    assert _rel_err(a, _oracle_acc(ring, ring["rc"])).max() <= ACC_TOL


def test_sym_clump_of_encounters(dev):
    # 300 bodies inside each other's critical radii amid a sparse cloud: rows
    # with hundreds of pairs, many inside 0.1 rho (K = 0)
    d = W.random_cloud(3000, seed=11, rc_scale=0.05)
    rng = np.random.default_rng(5)
    idx = rng.choice(3000, 300, replace=False)
    for c in ("x", "y", "z"):
        d[c][idx] = 1.0 + 1e-3 * rng.standard_normal(300)
    d["rc"][idx] = 0.02
    a, (pi, pj, cnt), code, _ = _run_kick(d, d["rc"], SYM)
    assert code == N.OK
    opi, opj, ocnt = oracle.pairs(d["x"], d["y"], d["z"], d["rc"])
    _say("clump pairs", cnt)
    assert cnt == ocnt > 40000 and np.array_equal(pi, opi) and np.array_equal(pj, opj)
    assert _rel_err(a, _oracle_acc(d, d["rc"])).max() <= ACC_TOL


def test_sym_pair_overflow(dev):
    d = W.random_cloud(2500, seed=3, rc_scale=0.3)
    rc = d["rc"]
    opi, opj, ocnt = oracle.pairs(d["x"], d["y"], d["z"], rc)
    cap = ocnt // 3
    _, (pi, pj, cnt), code, _ = _run_kick(d, rc, SYM, cap=cap)
    assert code == N.E_OVERFLOW and cnt == ocnt
    assert np.array_equal(pi, opi[:cap]) and np.array_equal(pj, opj[:cap])


def test_sym_coincident_and_invalid_rc(dev):
    d = W.random_cloud(1500, seed=1, rc_scale=0.1)
    d["x"][1207] = d["x"][3]; d["y"][1207] = d["y"][3]; d["z"][1207] = d["z"][3]
    _, _, code, _ = _run_kick(d, d["rc"], SYM, cap=1 << 20)
    assert code == N.E_NONFINITE
    d2 = W.random_cloud(1500, seed=2, rc_scale=0.1)
    rc = d2["rc"].copy()
    rc[1100] = -1.0
    _, _, code2, _ = _run_kick(d2, rc, SYM, cap=1 << 20)
    assert code2 == N.E_RCRIT


def test_sym_kick_updates_velocity_and_is_deterministic(dev):
    d = W.random_cloud(3000, seed=9, rc_scale=0.2)
    rc = d["rc"]
    a1, p1, c1, st = _run_kick(d, rc, SYM, h=3.0)
    a2, p2, c2, _ = _run_kick(d, rc, SYM, h=3.0)
    assert c1 == N.OK and c2 == N.OK
    assert np.array_equal(a1, a2) and np.array_equal(p1[0], p2[0]) and np.array_equal(p1[1], p2[1])
    out = st.numpy()
    for c, k in enumerate(("vx", "vy", "vz")):
        assert np.array_equal(out[k], d[k] + 3.0 * a1[c]) or \
            np.max(np.abs(out[k] - d[k] - 3.0 * a1[c])) <= 4e-16 * np.max(np.abs(d[k]))


def test_sym_steps_match_oracle(dev):
    # five base steps of the 2,048-body disk with the symmetric kick (first
    # half kick with the encounter list, the second with the Sun kick fused
    # into its reduction) against the oracle's step
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G, flags=SYM)
    ws = N.Workspace(st.n, cfg)
    pl = N.PairList(1 << 16)
    ref = oracle.state_copy(d)
    for _ in range(5):
        x0 = {c: st.t[c].cpu().numpy().copy() for c in "xyz"}
        assert N.step(st, cfg, ws, pl) == N.OK
        pi, pj, cnt = pl.result()
        opi, opj, ocnt = oracle.pairs(x0["x"], x0["y"], x0["z"], st.t["rc"].cpu().numpy())
        assert cnt == ocnt and np.array_equal(pi, opi) and np.array_equal(pj, opj)
        oracle.step(ref, G, 1.0, 6.0, 3.0, 0.4)
    out = st.numpy()
    for keys in (("x", "y", "z"), ("vx", "vy", "vz")):
        g = np.stack([out[k] for k in keys])
        r = np.stack([ref[k] for k in keys])
        assert np.max(np.abs(g - r)) / np.max(np.abs(r)) < 1e-12


def test_sym_graph_replay_bitwise(dev):
    d = W.random_cloud(5000, seed=21, rc_scale=0.2)
    cfg = N.Config(G=G, flags=SYM | N.FLAG_NOSYNC)
    st_g, st_e = N.State.from_numpy(d), N.State.from_numpy(d)
    ws_g, ws_e = N.Workspace(st_g.n, cfg), N.Workspace(st_e.n, cfg)
    pl_g, pl_e = N.PairList(1 << 20), N.PairList(1 << 20)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tmp = N.State.from_numpy(d)
        N.step(tmp, cfg, N.Workspace(tmp.n, cfg), N.PairList(1 << 20))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        N.step(st_g, cfg, ws_g, pl_g)
    torch.cuda.synchronize()
    for k in st_g.t:
        st_g.t[k].copy_(st_e.t[k])
    for rep in range(3):
        g.replay()
        N.step(st_e, cfg, ws_e, pl_e)
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert N.read_status(ws_g) == N.OK and N.read_status(ws_e) == N.OK
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert torch.equal(st_g.t[k], st_e.t[k]), (rep, k)
        a, b = pl_g.result(), pl_e.result()
        assert a[2] == b[2] and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        del junk


def test_sym_disk16384_default_form(dev):
    # from 8,192 bodies the library picks the symmetric form by itself
    d = W.make_disk(W.DISK_MIXED[16384])
    rc = oracle.rcrit(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["m"], 1.0, 6.0, 3.0, 0.4)
    a, (pi, pj, cnt), code, _ = _run_kick(d, rc, 0)
    a_d, (qi, qj, qc), code_d, _ = _run_kick(d, rc, DIR)
    assert code == N.OK and code_d == N.OK
    assert cnt == qc and np.array_equal(pi, qi) and np.array_equal(pj, qj)
    rows = np.concatenate([np.arange(0, 16384, 131), [16383]])
    err = []
    for r in rows:
        ref = _oracle_acc(d, rc, rows=(int(r), int(r) + 1))[:, 0]
        err.append(np.linalg.norm(a[:, r] - ref) / np.linalg.norm(ref))
    _say("disk16384 symmetric sampled max rel err", max(err))
    assert max(err) <= ACC_TOL
    assert np.max(_rel_err(a, a_d)) <= 2 * ACC_TOL
