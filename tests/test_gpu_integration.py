"""Integration checks of the step on the GPU: time reversibility of the
kick-drift-kick map with fixed critical radii, and bit-identical continuation
from a host checkpoint (the run is cut, its state copied to the host, every
device object rebuilt, and the run resumed)."""
import numpy as np
import pytest
import torch

from paper_2201_10058_amd import native as N
from paper_2201_10058_amd import workload as W

pytestmark = pytest.mark.gpu

G = W.GAUSS_G


def _say(*a):
    print(*a, flush=True)


def _kdk(st, cfg, ws, dt):
    N.kick(st, cfg, ws, 0.5 * dt)
    N.hc(st, cfg, ws, 0.5 * dt)
    N.drift(st, cfg, ws, dt)
    N.hc(st, cfg, ws, 0.5 * dt)
    N.kick(st, cfg, ws, 0.5 * dt)


def test_fixed_rc_map_is_reversible(dev):
    # 20 steps forward and 20 with -dt return the 2,048-body disk to its start
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=G)
    ws = N.Workspace(st.n, cfg)
    N.rcrit(st, cfg, ws)
    start = st.numpy()
    for _ in range(20):
        _kdk(st, cfg, ws, 6.0)
    mid = st.numpy()
    for _ in range(20):
        _kdk(st, cfg, ws, -6.0)
    assert N.read_status(ws) == N.OK
    end = st.numpy()
    moved = max(np.abs(mid[k] - start[k]).max() for k in ("x", "y", "z"))
    ex = max(np.abs(end[k] - start[k]).max() for k in ("x", "y", "z"))
    ev = max(np.abs(end[k] - start[k]).max() for k in ("vx", "vy", "vz"))
    _say(f"reversibility: moved {moved:.3e} AU, back to {ex:.2e} AU / {ev:.2e} AU/day")
    assert moved > 0.1
    assert ex < 1e-13 and ev < 1e-15


@pytest.mark.parametrize("kw", [dict(), dict(precision=N.MIXED),
                                dict(slevels=3, substeps=2, level_capacity=1 << 16, direct=1)])
def test_resume_from_host_checkpoint_is_bit_identical(dev, kw):
    d = W.make_disk(W.DISK_2048)
    cfg = N.Config(G=G, **kw)

    def run(state_np, steps):
        st = N.State.from_numpy(state_np)
        ws = N.Workspace(st.n, cfg)
        pl = N.PairList(1 << 16)
        for _ in range(steps):
            assert N.step(st, cfg, ws, pl) == N.OK
        out = st.numpy()
        del st, ws, pl
        torch.cuda.synchronize()
        return out

    straight = run(d, 20)
    half = run(d, 10)
    ckpt = {k: np.array(v, copy=True) for k, v in half.items()}   # the host checkpoint
    torch.cuda.empty_cache()
    resumed = run(ckpt, 10)
    for k in ("x", "y", "z", "vx", "vy", "vz", "rc"):
        assert np.array_equal(straight[k], resumed[k]), k
