"""Pins of the PyTorch reference used for gradients (CPU, float64).

* its forward maps agree with the C oracle (itself pinned in test_oracle_pins);
* its autograd gradients agree with central finite differences of the same
  forward, for the kick, the drift, rcrit, HC and short trajectories.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import torch_ref as T
from paper_2201_10058_amd import workload as W

G = W.GAUSS_G


def _small_disk(n, seed, a0=0.5, a1=1.5):
    spec = W.DiskSpec(f"t{n}", n, a0, a1, 2.0 * n / 64.0, seed=seed)
    return W.make_disk(spec)


def test_torch_kick_matches_c_oracle():
    d = W.random_cloud(60, seed=8, rc_scale=0.4)
    x, v, m = T.state_tensors(d)
    rc = torch.tensor(d["rc"], dtype=T.TD)
    a = T.kick_acc(x, m, rc, G).numpy().T
    ax, ay, az, st = oracle.kick_acc(d["x"], d["y"], d["z"], d["m"], d["rc"], G)
    ref = np.stack([ax, ay, az])
    assert np.max(np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)) < 1e-13


def test_torch_step_matches_c_oracle():
    d = _small_disk(48, seed=3)
    x, v, m = T.state_tensors(d)
    for _ in range(5):
        x, v = T.step(x, v, m, G, 1.0, 6.0, 3.0, 0.4)
    ref = oracle.state_copy(d)
    for _ in range(5):
        oracle.step(ref, G, 1.0, 6.0, 3.0, 0.4)
    X = np.stack([ref["x"], ref["y"], ref["z"]]).T
    V = np.stack([ref["vx"], ref["vy"], ref["vz"]]).T
    assert np.max(np.abs(x.numpy() - X)) < 1e-13 * np.max(np.abs(X))
    assert np.max(np.abs(v.numpy() - V)) < 1e-12 * np.max(np.abs(V))


def _fd_check(fn, inputs, seed, h=1e-6, tol=1e-6, ndir=6):
    """Directional derivatives: autograd <g, u> vs central differences."""
    torch.manual_seed(seed)
    ins = [t.detach().clone().requires_grad_(True) for t in inputs]
    out = fn(*ins)
    outs = out if isinstance(out, tuple) else (out,)
    wts = [torch.randn_like(o) for o in outs]
    L = sum((w * o).sum() for w, o in zip(wts, outs))
    grads = torch.autograd.grad(L, ins)
    for _ in range(ndir):
        dirs = [torch.randn_like(t) * (t.detach().abs() + 1e-30) for t in inputs]
        ad = sum((g * u).sum() for g, u in zip(grads, dirs)).item()

        def Lof(s):
            with torch.no_grad():
                o = fn(*[t + s * u for t, u in zip(inputs, dirs)])
                o = o if isinstance(o, tuple) else (o,)
                return sum((w * oo).sum() for w, oo in zip(wts, o)).item()

        fd = (Lof(h) - Lof(-h)) / (2 * h)
        assert abs(ad - fd) <= tol * max(abs(fd), abs(ad), 1e-300), (ad, fd)


def test_kick_gradient_fd_with_band_pairs():
    d = W.random_cloud(24, seed=12, rc_scale=0.8)
    x, v, m = T.state_tensors(d)
    rc = torch.tensor(d["rc"], dtype=T.TD)
    # many pairs inside the changeover band: K' terms and rc gradients active
    r = torch.cdist(x, x)
    rho = T.pair_rho(rc)
    yb = (r - 0.1 * rho) / (0.9 * rho)
    assert int(((yb > 0) & (yb < 1)).sum()) > 20
    _fd_check(lambda x_, m_, rc_: T.kick_acc(x_, m_, rc_, G), [x, m, rc], seed=1)


def test_drift_gradient_fd():
    d = _small_disk(30, seed=5)
    x, v, m = T.state_tensors(d)
    _fd_check(lambda x_, v_: T.drift(x_, v_, G, 37.0), [x, v], seed=2)


def test_rcrit_and_hc_gradient_fd():
    d = _small_disk(30, seed=6)
    x, v, m = T.state_tensors(d)
    _fd_check(lambda x_, v_, m_: T.rcrit(x_, v_, m_, 1.0, 6.0, 3.0, 0.4), [x, v, m], seed=3)
    _fd_check(lambda x_, v_, m_: T.hc(x_, v_, m_, 1.0, 3.0), [x, v, m], seed=4)


def test_trajectory_gradient_fd():
    d = _small_disk(20, seed=7)
    x, v, m = T.state_tensors(d)
    _fd_check(lambda x_, v_, m_: T.simulate(x_, v_, m_, 8, G, 1.0, 6.0, 3.0, 0.4), [x, v, m],
              seed=5, h=1e-7, tol=1e-5)


def test_rho_tie_routes_to_lower_index():
    rc = torch.tensor([0.3, 0.3, 0.1], dtype=T.TD, requires_grad=True)
    rho = T.pair_rho(rc)
    g = torch.autograd.grad(rho[0, 1] + rho[1, 0], rc)[0]
    assert g.tolist() == [2.0, 0.0, 0.0]


def _mixed_orbits(n, seed):
    """Bound and unbound heliocentric orbits (speed 0.2-1.9 times circular)."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.3, 3.0, n)
    th = rng.uniform(0, 2 * np.pi, n)
    vc = np.sqrt(G / r)
    fac = rng.uniform(0.2, 1.9, n)
    return dict(x=r * np.cos(th), y=r * np.sin(th), z=rng.normal(0, 0.01, n),
                vx=-fac * vc * np.sin(th) + rng.normal(0, 0.1, n) * vc,
                vy=fac * vc * np.cos(th), vz=rng.normal(0, 0.02, n) * vc, m=np.zeros(n))


def test_torch_drift_unbound_matches_c_oracle():
    # the hyperbolic branch against the C oracle's drift (itself pinned by
    # brentq on Kepler's hyperbolic equation and by energy conservation)
    d = _mixed_orbits(200, seed=31)
    x, v, _ = T.state_tensors(d)
    alpha = 2.0 / torch.linalg.norm(x, dim=1) - (v * v).sum(1) / G
    assert int((alpha < 0).sum()) > 40 and int((alpha > 0).sum()) > 40
    for dt in (20.0, -35.0, 300.0):
        x1, v1 = T.drift(x, v, G, dt)
        ref = oracle.state_copy(d)
        assert oracle.drift(ref, G, dt) == 0
        X = np.stack([ref["x"], ref["y"], ref["z"]]).T
        V = np.stack([ref["vx"], ref["vy"], ref["vz"]]).T
        ex = np.linalg.norm(x1.numpy() - X, axis=1) / np.linalg.norm(X, axis=1)
        ev = np.linalg.norm(v1.numpy() - V, axis=1) / np.linalg.norm(V, axis=1)
        assert ex.max() < 1e-12 and ev.max() < 1e-12, (dt, ex.max(), ev.max())


def test_drift_gradient_fd_unbound():
    # autograd through both branches against central differences
    d = _mixed_orbits(40, seed=32)
    x, v, _ = T.state_tensors(d)
    _fd_check(lambda x_, v_: T.drift(x_, v_, G, 25.0), [x, v], seed=6)
