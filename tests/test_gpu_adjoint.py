"""Hand-written adjoint (libgenga.so VJPs) against the autograd reference.

References: torch.autograd on oracle/torch_ref.py (float64, CPU), itself
pinned by finite differences in test_oracle_adjoint.py; plus central finite
differences of the GPU forward for the 4,096-body, 200-step trajectory.
"""
import numpy as np
import pytest
import torch

from oracle import torch_ref as T
from paper_2201_10058_amd import adjoint as A
from paper_2201_10058_amd import native as N
from paper_2201_10058_amd import workload as W

pytestmark = pytest.mark.gpu

G = W.GAUSS_G


def _say(*a):
    print(*a, flush=True)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _gpu_state(d, rc=None):
    return N.State.from_numpy(d, rc=rc)


def _small_disk(n, seed):
    return W.make_disk(W.DiskSpec(f"adj{n}", n, 0.5, 1.5, 2.0 * n / 64.0, seed=seed))


@pytest.mark.parametrize("flags", [0, N.FLAG_SYMMETRIC])
@pytest.mark.parametrize("n,scale", [(200, 0.4), (700, 0.15), (1100, 0.1)])
def test_kick_vjp_matches_autograd(dev, n, scale, flags):
    # the one-sided (gather) form and the symmetric form (each pair once,
    # applied to both bodies; the default from 8,192 bodies); 1,100 bodies
    # span three row groups of 512 and a ragged tail
    d = W.random_cloud(n, seed=21, rc_scale=scale)
    rng = np.random.default_rng(1)
    abar = rng.normal(size=(3, n))
    # reference
    x, v, m = T.state_tensors(d, requires_grad=True)
    rc = torch.tensor(d["rc"], dtype=T.TD, requires_grad=True)
    a = T.kick_acc(x, m, rc, G)
    L = (a * torch.tensor(abar.T) * 0.7).sum()
    gx, gm, grc = torch.autograd.grad(L, (x, m, rc))
    # GPU
    st = _gpu_state(d, rc=d["rc"])
    cfg = N.Config(G=G, flags=flags)
    ws = N.Workspace(n, cfg)
    adj = N.AdjointState(n)
    ab = [torch.tensor(abar[c], device="cuda") for c in range(3)]
    N.kick_vjp(st, cfg, ws, 0.7, ab, adj)
    torch.cuda.synchronize()
    assert N.read_status(ws) == N.OK
    out_x = np.stack([adj.t[k].cpu().numpy() for k in "xyz"]).T
    e = (_rel(out_x, gx.numpy()), _rel(adj.t["m"].cpu().numpy(), gm.numpy()),
         _rel(adj.t["rc"].cpu().numpy(), grc.numpy()))
    _say("kick vjp rel errors (x, m, rc)", e, "band rc grads", int((grc != 0).sum()))
    assert max(e) < 1e-10
    assert int((grc != 0).sum()) > 10


@pytest.mark.parametrize("n", [16384, 65536])
def test_kick_vjp_forms_agree_on_disks(dev, n):
    # at the benchmark sizes (beyond the autograd reference's reach) the
    # symmetric VJP against the one-sided gather form, which the autograd
    # test pins at small sizes: every body, relative to its own gradient
    d = W.make_disk(W.DISK_65536 if n == 65536 else W.DISK_MIXED[n])
    st = _gpu_state(d)
    c0 = N.Config(G=G)
    N.rcrit(st, c0, N.Workspace(n, c0))
    rng = np.random.default_rng(9)
    ab = [torch.tensor(rng.normal(size=n), device="cuda") for _ in range(3)]
    out = {}
    for name, fl in (("sym", N.FLAG_SYMMETRIC), ("one", N.FLAG_DIRECTED)):
        cfg = N.Config(G=G, flags=fl)
        ws = N.Workspace(n, cfg)
        adj = N.AdjointState(n)
        N.kick_vjp(st, cfg, ws, 1.3, ab, adj)
        torch.cuda.synchronize()
        assert N.read_status(ws) == N.OK
        out[name] = {k: adj.t[k].cpu().numpy() for k in ("x", "y", "z", "m", "rc")}
    xs = np.stack([out["sym"][k] for k in "xyz"]); xo = np.stack([out["one"][k] for k in "xyz"])
    ex = np.linalg.norm(xs - xo, axis=0) / np.linalg.norm(xo, axis=0)
    # scalar gradients (sums of terms of both signs, some near zero): against
    # the largest magnitude over the bodies
    em = np.abs(out["sym"]["m"] - out["one"]["m"]) / np.abs(out["one"]["m"]).max()
    band = out["one"]["rc"] != 0
    er = np.abs(out["sym"]["rc"] - out["one"]["rc"]) / np.abs(out["one"]["rc"]).max()
    _say(f"vjp forms n={n}: xbar {ex.max():.2e} mbar {em.max():.2e} rcbar {er.max():.2e} "
         f"({int(band.sum())} band rows)")
    assert ex.max() < 1e-10 and em.max() < 1e-12 and er.max() < 1e-12
    assert np.array_equal(out["sym"]["rc"] != 0, band)


def test_rcrit_hc_drift_vjp_match_autograd(dev):
    d = _small_disk(300, seed=9)
    n = 300
    rng = np.random.default_rng(2)
    cfg = N.Config(G=G)
    ws = N.Workspace(n, cfg)
    # rcrit
    x, v, m = T.state_tensors(d, requires_grad=True)
    rcb = rng.normal(size=n)
    L = (T.rcrit(x, v, m, 1.0, 6.0, 3.0, 0.4) * torch.tensor(rcb)).sum()
    gx, gv, gm = torch.autograd.grad(L, (x, v, m))
    adj = N.AdjointState(n)
    adj.t["rc"].copy_(torch.tensor(rcb))
    N.rcrit_vjp(_gpu_state(d), cfg, ws, adj)
    assert _rel(np.stack([adj.t[k].cpu().numpy() for k in "xyz"]).T, gx.numpy()) < 1e-13
    assert _rel(np.stack([adj.t[k].cpu().numpy() for k in ("vx", "vy", "vz")]).T, gv.numpy()) < 1e-13
    assert _rel(adj.t["m"].cpu().numpy(), gm.numpy()) < 1e-13
    # HC
    xb = rng.normal(size=(n, 3))
    x, v, m = T.state_tensors(d, requires_grad=True)
    L = (T.hc(x, v, m, 1.0, 3.0) * torch.tensor(xb)).sum()
    gx, gv, gm = torch.autograd.grad(L, (x, v, m))
    adj = N.AdjointState(n)
    for c, k in enumerate("xyz"):
        adj.t[k].copy_(torch.tensor(xb[:, c]))
    N.hc_vjp(_gpu_state(d), cfg, ws, 3.0, adj)
    assert _rel(np.stack([adj.t[k].cpu().numpy() for k in "xyz"]).T, gx.numpy()) < 1e-15
    assert _rel(np.stack([adj.t[k].cpu().numpy() for k in ("vx", "vy", "vz")]).T, gv.numpy()) < 1e-13
    assert _rel(adj.t["m"].cpu().numpy(), gm.numpy()) < 1e-13
    # drift
    b6 = rng.normal(size=(n, 6))
    x, v, m = T.state_tensors(d, requires_grad=True)
    x1, v1 = T.drift(x, v, G, 6.0)
    L = (x1 * torch.tensor(b6[:, :3])).sum() + (v1 * torch.tensor(b6[:, 3:])).sum()
    gx, gv = torch.autograd.grad(L, (x, v))
    adj = N.AdjointState(n)
    for c, k in enumerate(("x", "y", "z", "vx", "vy", "vz")):
        adj.t[k].copy_(torch.tensor(b6[:, c]))
    N.drift_vjp(_gpu_state(d), cfg, ws, 6.0, adj)
    torch.cuda.synchronize()
    assert N.read_status(ws) == N.OK
    ex = _rel(np.stack([adj.t[k].cpu().numpy() for k in "xyz"]).T, gx.numpy())
    ev = _rel(np.stack([adj.t[k].cpu().numpy() for k in ("vx", "vy", "vz")]).T, gv.numpy())
    _say("drift vjp rel errors", ex, ev)
    assert ex < 1e-11 and ev < 1e-11


def test_drift_vjp_bound_and_unbound_match_autograd(dev):
    # bound and unbound orbits in one call: the hyperbolic branch of the
    # drift VJP against autograd of the reference's hyperbolic-anomaly drift
    rng = np.random.default_rng(33)
    n = 400
    r = rng.uniform(0.3, 3.0, n)
    th = rng.uniform(0, 2 * np.pi, n)
    vc = np.sqrt(G / r)
    fac = rng.uniform(0.2, 1.9, n)
    d = dict(x=r * np.cos(th), y=r * np.sin(th), z=rng.normal(0, 0.01, n),
             vx=-fac * vc * np.sin(th) + rng.normal(0, 0.1, n) * vc,
             vy=fac * vc * np.cos(th), vz=rng.normal(0, 0.02, n) * vc, m=np.zeros(n))
    cfg = N.Config(G=G)
    ws = N.Workspace(n, cfg)
    for dt in (20.0, -35.0):
        b6 = rng.normal(size=(n, 6))
        x, v, _ = T.state_tensors(d, requires_grad=True)
        alpha = 2.0 / torch.linalg.norm(x, dim=1) - (v * v).sum(1) / G
        assert int((alpha < 0).sum()) > 80 and int((alpha > 0).sum()) > 80
        x1, v1 = T.drift(x, v, G, dt)
        L = (x1 * torch.tensor(b6[:, :3])).sum() + (v1 * torch.tensor(b6[:, 3:])).sum()
        gx, gv = torch.autograd.grad(L, (x, v))
        adj = N.AdjointState(n)
        for c, k in enumerate(("x", "y", "z", "vx", "vy", "vz")):
            adj.t[k].copy_(torch.tensor(b6[:, c]))
        N.drift_vjp(_gpu_state(d), cfg, ws, dt, adj)
        torch.cuda.synchronize()
        assert N.read_status(ws) == N.OK
        gxs = np.stack([adj.t[k].cpu().numpy() for k in "xyz"]).T
        gvs = np.stack([adj.t[k].cpu().numpy() for k in ("vx", "vy", "vz")]).T
        # per body, relative to the body's own gradient
        ex = np.linalg.norm(gxs - gx.numpy(), axis=1) / np.linalg.norm(gx.numpy(), axis=1)
        ev = np.linalg.norm(gvs - gv.numpy(), axis=1) / np.linalg.norm(gv.numpy(), axis=1)
        _say("drift vjp, bound + unbound, dt", dt, "max rel errors", ex.max(), ev.max())
        assert ex.max() < 1e-10 and ev.max() < 1e-10


def _torch_dev(d):
    X = torch.tensor(np.stack([d["x"], d["y"], d["z"]]), device="cuda")
    V = torch.tensor(np.stack([d["vx"], d["vy"], d["vz"]]), device="cuda")
    m = torch.tensor(d["m"], device="cuda")
    return X, V, m


def test_trajectory_gradient_matches_autograd(dev):
    d = _small_disk(48, seed=13)
    steps = 12
    cfg = N.Config(G=G)
    rng = np.random.default_rng(3)
    wX = rng.normal(size=(3, 48))
    wV = rng.normal(size=(3, 48))
    X, V, m = _torch_dev(d)
    X.requires_grad_(True); V.requires_grad_(True); m.requires_grad_(True)
    XT, VT = A.simulate(X, V, m, steps, cfg, checkpoint_every=5)
    L = (XT * torch.tensor(wX, device="cuda")).sum() + (VT * torch.tensor(wV, device="cuda")).sum()
    gX, gV, gm = torch.autograd.grad(L, (X, V, m))
    x, v, mm = T.state_tensors(d, requires_grad=True)
    xT, vT = T.simulate(x, v, mm, steps, G, 1.0, 6.0, 3.0, 0.4)
    Lr = (xT * torch.tensor(wX.T)).sum() + (vT * torch.tensor(wV.T)).sum()
    rx, rv, rm = torch.autograd.grad(Lr, (x, v, mm))
    e = (_rel(gX.cpu().numpy().T, rx.numpy()), _rel(gV.cpu().numpy().T, rv.numpy()),
         _rel(gm.cpu().numpy(), rm.numpy()))
    _say("trajectory gradient rel errors (x, v, m)", e)
    assert max(e) < 1e-9


def test_checkpointing_is_bitwise_neutral(dev):
    d = _small_disk(256, seed=14)
    cfg = N.Config(G=G)
    grads = []
    for ce in (3, 7, 100):
        X, V, m = _torch_dev(d)
        X.requires_grad_(True); V.requires_grad_(True); m.requires_grad_(True)
        XT, VT = A.simulate(X, V, m, 20, cfg, checkpoint_every=ce)
        L = (XT ** 2).sum() + (VT ** 2).sum()
        grads.append([t.cpu() for t in torch.autograd.grad(L, (X, V, m))])
    for g in grads[1:]:
        for a, b in zip(grads[0], g):
            assert torch.equal(a, b)


def test_fd_directions_disk4096_200_steps(dev):
    # The adjoint workload: 4,096-body disk (0.5-1.5 AU, 2 Earth masses), 200
    # steps of 6 days, loss = sum |x_T - target|^2 with target = nominal x_T +
    # 1e-3 AU N(0, 1) (seed 4); 32 central differences, h = 1e-7 on
    # theta + h (s * u), u ~ N(0, I) (seed 5), s = (1 AU, 0.0172 AU/day, m_i).
    d = W.make_disk(W.DISK_ADJOINT)
    cfg = N.Config(G=G)
    steps = 200
    X0, V0, m0 = _torch_dev(d)
    with torch.no_grad():
        XT, _ = A.simulate(X0, V0, m0, steps, cfg)
    rng = np.random.default_rng(4)
    target = XT + torch.tensor(1e-3 * rng.normal(size=XT.shape), device="cuda")

    def loss(X, V, m):
        XT_, _ = A.simulate(X, V, m, steps, cfg, checkpoint_every=20)
        return ((XT_ - target) ** 2).sum()

    X, V, m = X0.clone().requires_grad_(True), V0.clone().requires_grad_(True), m0.clone().requires_grad_(True)
    gX, gV, gm = torch.autograd.grad(loss(X, V, m), (X, V, m))
    rng = np.random.default_rng(5)
    h = 1e-7
    worst = 0.0
    for k in range(32):
        uX = torch.tensor(rng.normal(size=X0.shape), device="cuda") * 1.0
        uV = torch.tensor(rng.normal(size=V0.shape), device="cuda") * 0.0172
        um = torch.tensor(rng.normal(size=m0.shape), device="cuda") * m0
        ad = float((gX * uX).sum() + (gV * uV).sum() + (gm * um).sum())
        with torch.no_grad():
            lp = float(loss(X0 + h * uX, V0 + h * uV, m0 + h * um))
            lm = float(loss(X0 - h * uX, V0 - h * uV, m0 - h * um))
        fd = (lp - lm) / (2 * h)
        rel = abs(ad - fd) / max(abs(fd), 1e-300)
        worst = max(worst, rel)
        _say(f"dir {k}: adjoint {ad:.10e} fd {fd:.10e} rel {rel:.2e}")
    assert worst <= 1e-5
