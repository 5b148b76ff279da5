"""genga_kick_static (no workspace, the library's static scratch) against
genga_kick: the same accelerations, velocities, encounter list and status,
bit for bit, on consecutive calls of decreasing size (the scratch keeps the
previous call's contents) and in both precisions.
"""
import numpy as np
import pytest
import torch

from paper_2201_10058_amd import native as N
from paper_2201_10058_amd import workload as W

pytestmark = pytest.mark.gpu

G = W.GAUSS_G


def _say(*a):
    print(*a, flush=True)


def _rc(d):
    # critical radii written by the library itself (inputs for both calls)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G)
    N.rcrit(st, cfg, N.Workspace(st.n, cfg))
    return st.t["rc"].cpu().numpy()


def _pair(d, rc, cfg, h, cap):
    # the same inputs through genga_kick (caller's workspace) and
    # genga_kick_static; velocities are updated when h != 0
    st_w = N.State.from_numpy(d, rc=rc)
    st_s = N.State.from_numpy(d, rc=rc)
    ws = N.Workspace(st_w.n, cfg)
    pl_w, pl_s = N.PairList(cap), N.PairList(cap)
    a_w = N.kick(st_w, cfg, ws, h, acc=True, pairs=pl_w)
    a_s, status = N.kick_static(st_s, cfg, h, acc=True, pairs=pl_s)
    torch.cuda.synchronize()
    return (st_w, a_w, pl_w, N.read_status(ws)), (st_s, a_s, pl_s, int(status.item()))


def _same(w, s, what):
    st_w, a_w, pl_w, code_w = w
    st_s, a_s, pl_s, code_s = s
    _say(what, "status", code_w, code_s, "pairs", int(pl_w.count.item()), int(pl_s.count.item()))
    assert code_s == code_w
    assert torch.equal(a_s, a_w), what
    for k in ("vx", "vy", "vz"):
        assert torch.equal(st_s.t[k], st_w.t[k]), (what, k)
    assert int(pl_s.count.item()) == int(pl_w.count.item())
    c = min(int(pl_w.count.item()), pl_w.capacity)
    assert torch.equal(pl_s.i[:c], pl_w.i[:c]) and torch.equal(pl_s.j[:c], pl_w.j[:c])


def test_kick_static_matches_kick_on_consecutive_calls(dev):
    # 1: the 8,192-body disk (symmetric binary64 form), v += h a, full list
    d1 = W.make_disk(W.DiskSpec("disk_n8192_a0.5-4_5Mearth", 8192, 0.5, 4.0, 5.0, seed=40))
    rc1 = _rc(d1)
    w, s = _pair(d1, rc1, N.Config(G=G), 3.0, 1 << 16)
    assert w[3] == N.OK
    _same(w, s, "disk8192 fp64")
    # 2: a smaller system right after it (the scratch holds call 1's data),
    #    one-sided form, a list capacity below the count: overflow reported
    d2 = W.random_cloud(700, seed=41, rc_scale=0.2)
    w, s = _pair(d2, d2["rc"], N.Config(G=G), 0.0, 50)
    assert w[3] == N.E_OVERFLOW and int(w[2].count.item()) > 50
    _same(w, s, "cloud700 overflow")
    # 3: smaller again, mixed precision (binary64 refinement of cancelling rows)
    d3 = W.make_disk(W.DISK_2048)
    rc3 = _rc(d3)
    w, s = _pair(d3, rc3, N.Config(G=G, precision=N.MIXED), 3.0, 1 << 14)
    assert w[3] == N.OK
    _same(w, s, "disk2048 mixed")
    # 4: the first system again: nothing of calls 2-3 leaks into it
    w, s = _pair(d1, rc1, N.Config(G=G), 3.0, 1 << 16)
    _same(w, s, "disk8192 fp64 again")


def test_kick_static_rejects_oversize(dev):
    # beyond the static scratch: refused on the host, nothing enqueued
    d = W.random_cloud(20000, seed=42, rc_scale=0.01)
    st = N.State.from_numpy(d)
    with pytest.raises(N.GengaError) as e:
        N.kick_static(st, N.Config(G=G), 0.0, acc=True)
    assert e.value.code == N.E_SCRATCH
