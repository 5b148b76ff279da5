"""Batched ensembles: many systems in one persistent kick launch.

Bar: every system's accelerations equal the oracle run on that system alone
(<= 1e-12 relative per acceleration in FP64, <= 1e-6 in mixed precision) and
its encounter pairs are bit-exact (with global
indices); a hipGraph replay of the batched step equals the eager step bit for
bit.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2201_10058_amd import autotune
from paper_2201_10058_amd import native as N
from paper_2201_10058_amd import workload as W

pytestmark = pytest.mark.gpu

G = W.GAUSS_G
MIXED_TOL = 1e-6
SMALL_SIZES = [16, 17, 63, 64, 65, 100, 255, 256, 257, 300, 700, 1500, 2048, 3001]


def _say(*a):
    print(*a, flush=True)


def _rc_batch(d):
    rc = np.empty(d["x"].size)
    for s in range(d["S"]):
        lo, hi = d["offsets"][s], d["offsets"][s + 1]
        rc[lo:hi] = oracle.rcrit(*(d[k][lo:hi] for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                                 d["m_star"][s], d["dt"][s], d["n1"][s], d["n2"][s])
    return rc


def _batch(d):
    return N.Batch(d["offsets"], d["m_star"], d["dt"], d["n1"], d["n2"])


def _oracle_system(d, rc, s, rows=None):
    lo, hi = d["offsets"][s], d["offsets"][s + 1]
    sl = {k: d[k][lo:hi] for k in ("x", "y", "z", "m")}
    ax, ay, az, st = oracle.kick_acc(sl["x"], sl["y"], sl["z"], sl["m"], rc[lo:hi], G, rows=rows)
    assert st == 0
    pi, pj, cnt = oracle.pairs(sl["x"], sl["y"], sl["z"], rc[lo:hi])
    return np.stack([ax, ay, az]), pi + lo, pj + lo, cnt


@pytest.mark.parametrize("block,ipt,cols,flags", [(256, 1, 1024, N.FLAG_DIRECTED), (64, 1, 256, N.FLAG_DIRECTED),
                                                  (64, 2, 512, N.FLAG_DIRECTED), (256, 2, 2048, N.FLAG_DIRECTED),
                                                  (0, 0, 0, 0)])
def test_batched_kick_matches_oracle(dev, block, ipt, cols, flags):
    # one-sided tile shapes, and the symmetric form (the binary64 default)
    d = W.make_batch(sizes=SMALL_SIZES)
    rc = _rc_batch(d)
    st = N.State.from_numpy(d, rc=rc)
    bt = _batch(d)
    cfg = N.Config(G=G, block=block, ipt=ipt, tile_cols=cols, flags=flags)
    ws = N.BatchWorkspace(bt, cfg)
    _say("plan", ws.info)
    pl = N.PairList(200000)
    a = N.kick_batched(st, ws, cfg, 0.0, acc=True, pairs=pl)
    torch.cuda.synchronize()
    assert N.read_status(ws) == N.OK
    a = a.cpu().numpy()
    pi, pj, cnt = pl.result()
    all_i, all_j = [], []
    worst = 0.0
    for s in range(d["S"]):
        lo, hi = d["offsets"][s], d["offsets"][s + 1]
        ref, opi, opj, ocnt = _oracle_system(d, rc, s)
        err = np.linalg.norm(a[:, lo:hi] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        worst = max(worst, err.max())
        all_i.append(opi); all_j.append(opj)
    _say("worst rel err", worst)
    assert worst <= 1e-12
    oi, oj = np.concatenate(all_i), np.concatenate(all_j)
    assert cnt == len(oi) and np.array_equal(pi, oi) and np.array_equal(pj, oj)


@pytest.mark.parametrize("slices", [1, 2, 4])
def test_batched_symmetric_widths_match_oracle(dev, slices):
    # the symmetric kick with 512-, 256- and 128-column slices (up to 24
    # tiles per 512-row group here, so the reduction adds up to 24 row sums
    # per row before the column sums); a second launch gives the same bits
    d = W.make_batch(sizes=SMALL_SIZES)
    rc = _rc_batch(d)
    st = N.State.from_numpy(d, rc=rc)
    bt = _batch(d)
    cfg = N.Config(G=G, slices=slices, flags=N.FLAG_SYMMETRIC)
    ws = N.BatchWorkspace(bt, cfg)
    _say("plan", ws.info)
    pl = N.PairList(200000)
    a = N.kick_batched(st, ws, cfg, 0.0, acc=True, pairs=pl).cpu().numpy()
    a2 = N.kick_batched(st, ws, cfg, 0.0, acc=True).cpu().numpy()
    torch.cuda.synchronize()
    assert N.read_status(ws) == N.OK
    assert np.array_equal(a, a2)
    pi, pj, cnt = pl.result()
    all_i, all_j = [], []
    for s in range(d["S"]):
        lo, hi = d["offsets"][s], d["offsets"][s + 1]
        ref, opi, opj, _ = _oracle_system(d, rc, s)
        err = np.linalg.norm(a[:, lo:hi] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        assert err.max() <= 1e-12, (s, err.max())
        all_i.append(opi); all_j.append(opj)
    oi, oj = np.concatenate(all_i), np.concatenate(all_j)
    assert cnt == len(oi) and np.array_equal(pi, oi) and np.array_equal(pj, oj)


def test_batched_step_matches_oracle_and_single(dev):
    d = W.make_batch(sizes=SMALL_SIZES)
    bt = _batch(d)
    cfg = N.Config(G=G, block=64, ipt=1, tile_cols=512)
    st = N.State.from_numpy(d)
    ws = N.BatchWorkspace(bt, cfg)
    pl = N.PairList(200000)
    x0 = {c: d[c].copy() for c in "xyz"}
    assert N.step_batched(st, ws, cfg, pl) == N.OK
    out = st.numpy()
    pi, pj, cnt = pl.result()
    rc_used = out["rc"]
    # pairs of the first half kick: oracle on the start positions and used radii
    all_i, all_j = [], []
    for s in range(d["S"]):
        lo, hi = d["offsets"][s], d["offsets"][s + 1]
        opi, opj, _ = oracle.pairs(x0["x"][lo:hi], x0["y"][lo:hi], x0["z"][lo:hi], rc_used[lo:hi])
        all_i.append(opi + lo); all_j.append(opj + lo)
    oi, oj = np.concatenate(all_i), np.concatenate(all_j)
    assert cnt == len(oi) and np.array_equal(pi, oi) and np.array_equal(pj, oj)
    # every system against the oracle step and against a single-system call
    st1 = N.State.from_numpy(d)
    for s in range(d["S"]):
        lo, hi = int(d["offsets"][s]), int(d["offsets"][s + 1])
        ref = {k: d[k][lo:hi].copy() for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
        oracle.step(ref, G, d["m_star"][s], d["dt"][s], d["n1"][s], d["n2"][s])
        sv = N.system_view(st1, lo, hi)
        c1 = N.Config(G=G, m_star=d["m_star"][s], dt=d["dt"][s], n1=d["n1"][s], n2=d["n2"][s])
        w1 = N.Workspace(hi - lo, c1)
        assert N.step(sv, c1, w1) == N.OK
        single = {k: v.cpu().numpy() for k, v in sv.t.items()}
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            scale = np.max(np.abs(ref[k]))
            assert np.max(np.abs(out[k][lo:hi] - ref[k])) <= 1e-12 * scale, (s, k)
            assert np.max(np.abs(out[k][lo:hi] - single[k])) <= 1e-12 * scale, (s, k)


@pytest.mark.parametrize("form", ["one-sided", "symmetric"])
def test_batched_graph_replay_bitwise(dev, form):
    if form == "one-sided":
        d = W.make_batch(sizes=SMALL_SIZES[:10])
        cfg = N.Config(G=G, flags=N.FLAG_NOSYNC, block=64, tile_cols=512)
    else:
        # 128-column slices, systems of 16 to 3,001 bodies
        d = W.make_batch(sizes=SMALL_SIZES)
        cfg = N.Config(G=G, flags=N.FLAG_NOSYNC | N.FLAG_SYMMETRIC, slices=4)
    bt = _batch(d)
    st_g = N.State.from_numpy(d)
    st_e = N.State.from_numpy(d)
    ws_g = N.BatchWorkspace(bt, cfg)
    ws_e = N.BatchWorkspace(bt, cfg)
    pl_g = N.PairList(100000)
    pl_e = N.PairList(100000)
    # warm up on a side stream before capture
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tmp = N.State.from_numpy(d)
        N.step_batched(tmp, N.BatchWorkspace(bt, cfg), cfg, N.PairList(100000))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        N.step_batched(st_g, ws_g, cfg, pl_g)
    torch.cuda.synchronize()
    # capture does not execute; reset the captured state to the start
    for k in st_g.t:
        st_g.t[k].copy_(st_e.t[k])
    for rep in range(5):
        g.replay()
        N.step_batched(st_e, ws_e, cfg, pl_e)
        junk = torch.randn(1000, device="cuda").sum()     # unrelated eager work
        torch.cuda.synchronize()
        assert N.read_status(ws_g) == N.OK and N.read_status(ws_e) == N.OK
        for k in ("x", "y", "z", "vx", "vy", "vz", "rc"):
            assert torch.equal(st_g.t[k], st_e.t[k]), (rep, k)
        assert int(pl_g.count.item()) == int(pl_e.count.item())
        c = min(int(pl_e.count.item()), pl_e.capacity)
        assert torch.equal(pl_g.i[:c], pl_e.i[:c]) and torch.equal(pl_g.j[:c], pl_e.j[:c])
        del junk


def test_batched_full_ensemble_sampled(dev):
    # the 512-system ensemble (log-uniform 16..4096 bodies): sampled systems
    d = W.make_batch()
    rc = _rc_batch(d)
    st = N.State.from_numpy(d, rc=rc)
    bt = _batch(d)
    cfg = N.Config(G=G)
    ws = N.BatchWorkspace(bt, cfg)
    pl = N.PairList(4_000_000)
    a = N.kick_batched(st, ws, cfg, 0.0, acc=True, pairs=pl)
    torch.cuda.synchronize()
    assert N.read_status(ws) == N.OK
    a = a.cpu().numpy()
    pi, pj, cnt = pl.result()
    _say("ensemble bodies", d["x"].size, "pairs", cnt, "plan", ws.info)
    rng = np.random.default_rng(0)
    sizes = np.diff(d["offsets"])
    pick = list(rng.choice(d["S"], 24, replace=False)) + [int(np.argmax(sizes)), int(np.argmin(sizes))]
    for s in pick:
        lo, hi = d["offsets"][s], d["offsets"][s + 1]
        ref, opi, opj, ocnt = _oracle_system(d, rc, s)
        err = np.linalg.norm(a[:, lo:hi] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        assert err.max() <= 1e-12, (s, err.max())
        sel = (pi >= lo) & (pi < hi)
        assert np.array_equal(pi[sel], opi) and np.array_equal(pj[sel], opj)
    # global list is sorted and stays inside systems
    assert np.all(np.diff(pi.astype(np.int64) * (1 << 32) + pj) > 0)
    sys_i = np.searchsorted(d["offsets"], pi, side="right") - 1
    sys_j = np.searchsorted(d["offsets"], pj, side="right") - 1
    assert np.array_equal(sys_i, sys_j)


def test_batched_mixed_precision(dev):
    # every body of every system against the oracle's compensated kick of
    # that system alone: relative error <= 1e-6 per acceleration; the encounter
    # list (binary64 test) equals the oracle's
    d = W.make_batch(sizes=SMALL_SIZES)
    rc = _rc_batch(d)
    st = N.State.from_numpy(d, rc=rc)
    bt = _batch(d)
    c32 = N.Config(G=G, precision=N.MIXED)
    w32 = N.BatchWorkspace(bt, c32)
    p32 = N.PairList(200000)
    a32 = N.kick_batched(st, w32, c32, 0.0, acc=True, pairs=p32)
    torch.cuda.synchronize()
    assert N.read_status(w32) == N.OK
    a32 = a32.cpu().numpy()
    pi, pj, cnt = p32.result()
    worst, all_i, all_j = 0.0, [], []
    for s in range(d["S"]):
        lo, hi = d["offsets"][s], d["offsets"][s + 1]
        ref, opi, opj, _ = _oracle_system(d, rc, s)
        err = np.linalg.norm(a32[:, lo:hi] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        _say(f"batched mixed system {s} ({hi - lo} bodies): max rel {err.max():.3e}")
        worst = max(worst, err.max())
        all_i.append(opi); all_j.append(opj)
    assert worst <= MIXED_TOL
    oi, oj = np.concatenate(all_i), np.concatenate(all_j)
    assert cnt == len(oi) and np.array_equal(pi, oi) and np.array_equal(pj, oj)


def test_batched_mixed_full_ensemble_sampled(dev):
    # the 512-system ensemble in mixed precision: 26 sampled systems (with the
    # largest and the smallest), every body against the oracle to 1e-6
    d = W.make_batch()
    rc = _rc_batch(d)
    st = N.State.from_numpy(d, rc=rc)
    bt = _batch(d)
    cfg = N.Config(G=G, precision=N.MIXED)
    ws = N.BatchWorkspace(bt, cfg)
    pl = N.PairList(4_000_000)
    a = N.kick_batched(st, ws, cfg, 0.0, acc=True, pairs=pl)
    torch.cuda.synchronize()
    assert N.read_status(ws) == N.OK
    a = a.cpu().numpy()
    pi, pj, cnt = pl.result()
    rng = np.random.default_rng(0)
    sizes = np.diff(d["offsets"])
    pick = list(rng.choice(d["S"], 24, replace=False)) + [int(np.argmax(sizes)), int(np.argmin(sizes))]
    worst = 0.0
    for s in pick:
        lo, hi = d["offsets"][s], d["offsets"][s + 1]
        ref, opi, opj, _ = _oracle_system(d, rc, s)
        err = np.linalg.norm(a[:, lo:hi] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        worst = max(worst, err.max())
        sel = (pi >= lo) & (pi < hi)
        assert np.array_equal(pi[sel], opi) and np.array_equal(pj[sel], opj)
    _say("ensemble mixed: worst rel err over the sampled systems", worst)
    assert worst <= MIXED_TOL


def test_autotune_batched_choice_is_valid(dev, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv(autotune.CACHE_ENV, str(cache))
    d = W.make_batch(sizes=SMALL_SIZES)
    st = N.State.from_numpy(d, rc=_rc_batch(d))
    x0 = st.t["x"].clone(), st.t["vx"].clone()
    bt = _batch(d)
    cfg = N.Config(G=G)
    choice = autotune.tune_batched(st, bt, cfg)
    _say("autotuned batched shape", choice)
    if choice["form"] == "one-sided":
        assert choice["block"] in (64, 256) and choice["ipt"] in (1, 2)
        assert choice["tile_cols"] in (256, 512, 1024, 2048) and choice["grid"] >= 0
    else:
        assert choice["flags"] & N.FLAG_SYMMETRIC and choice["slices"] in (0, 1, 2, 4)
    assert choice["ms"] > 0.0
    # the state is untouched (zero step factor)
    assert torch.equal(st.t["x"], x0[0]) and torch.equal(st.t["vx"], x0[1])
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("batch:")
    again = autotune.tune_batched(st, bt, cfg)                  # served from the cache
    shape = {k: choice[k] for k in ("block", "ipt", "tile_cols", "grid", "slices", "flags")}
    assert {k: again[k] for k in shape} == shape
    assert again["ms"] == pytest.approx(choice["ms"], rel=1e-5)
    assert len(cache.read_text().splitlines()) == 1
    c = N.Config(G=G, **shape)
    a = N.kick_batched(st, N.BatchWorkspace(bt, c), c, 0.0, acc=True).cpu().numpy()
    b = N.kick_batched(st, N.BatchWorkspace(bt, cfg), cfg, 0.0, acc=True).cpu().numpy()
    assert np.max(np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)) <= 1e-13


@pytest.mark.parametrize("n", [2048, 16384])
def test_autotune_single_choice_is_valid(dev, tmp_path, monkeypatch, n):
    # the tuner picks a form and its shape; the cached choice comes back, and
    # the chosen shape computes the default kick's accelerations
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv(autotune.CACHE_ENV, str(cache))
    d = W.make_disk(W.DISK_2048 if n == 2048 else W.DISK_MIXED[n])
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G)
    choice = autotune.tune_single(st, cfg)
    _say("autotuned single shape", n, choice)
    if choice["form"] == "one-sided":
        assert choice["flags"] & N.FLAG_DIRECTED
        assert choice["ipt"] in (1, 2) and choice["slices"] in (0, 8, 16, 32, 64)
    else:
        assert choice["flags"] & N.FLAG_SYMMETRIC and choice["slices"] in (0, 1, 2, 4, 8)
    again = autotune.tune_single(st, cfg)
    assert {k: again[k] for k in ("form", "ipt", "slices")} == \
        {k: choice[k] for k in ("form", "ipt", "slices")}
    assert cache.read_text().splitlines()[0].startswith("single:")
    tuned = N.Config(G=G, ipt=choice["ipt"], slices=choice["slices"], flags=choice["flags"])
    N.rcrit(st, cfg, N.Workspace(st.n, cfg))
    a0 = N.kick(st, cfg, N.Workspace(st.n, cfg), 0.0, acc=True).cpu().numpy()
    a1 = N.kick(st, tuned, N.Workspace(st.n, tuned), 0.0, acc=True).cpu().numpy()
    assert np.max(np.linalg.norm(a0 - a1, axis=0) / np.linalg.norm(a0, axis=0)) <= 1e-13
