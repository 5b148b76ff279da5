"""Host build of the drift's Kepler solver (csrc/kepler.h) against the oracle.

The HIP drift kernel calls a header-only __host__ __device__ solver; here the
same header is compiled for the CPU with g++ and compared body by body with
the oracle's independent f-and-g formulation (eccentric/hyperbolic anomaly).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2201_10058_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2201_10058_amd", "csrc")
G = W.GAUSS_G

SHIM = r'''
#define GENGA_HD
#include "kepler.h"
extern "C" int kepler_host(double mu, double dt, long n, double *x, double *y, double *z,
                           double *vx, double *vy, double *vz) {
    int st = 0;
    for (long i = 0; i < n; ++i) st |= genga::kepler_uv(mu, dt, x[i], y[i], z[i], vx[i], vy[i], vz[i]);
    return st;
}
// in: states s (n x 6) and adjoints b (n x 6) of the drifted states; out: b <- adjoints of s
extern "C" int kepler_vjp_host(double mu, double dt, long n, const double *s, double *b) {
    int st = 0;
    for (long i = 0; i < n; ++i) st |= genga::kepler_uv_vjp(mu, dt, s + 6 * i, s + 6 * i + 3, b + 6 * i, b + 6 * i + 3);
    return st;
}
'''


@pytest.fixture(scope="module")
def kep(tmp_path_factory):
    d = tmp_path_factory.mktemp("kep")
    src = d / "shim.cpp"
    src.write_text(SHIM)
    lib = d / "libkep.so"
    subprocess.run(["g++", "-O2", "-ffp-contract=off", "-std=c++17", "-shared", "-fPIC",
                    f"-I{CSRC}", str(src), "-o", str(lib)], check=True)
    L = ctypes.CDLL(str(lib))
    L.kepler_host.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_long] + [ctypes.c_void_p] * 6
    L.kepler_vjp_host.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_long] + [ctypes.c_void_p] * 2
    return L


def _run(L, d, mu, dt):
    s = oracle.state_copy(d)
    st = L.kepler_host(mu, dt, len(s["x"]), *(s[k].ctypes.data for k in ("x", "y", "z", "vx", "vy", "vz")))
    return s, st


def _err(a, b, keys):
    A = np.stack([a[k] for k in keys]); B = np.stack([b[k] for k in keys])
    return (np.linalg.norm(A - B, axis=0) / np.linalg.norm(B, axis=0)).max()


@pytest.mark.parametrize("dt", [6.0, -6.0, 250.0])
def test_kepler_host_disk(kep, dt):
    d = W.make_disk(W.DISK_2048)
    out, st = _run(kep, d, G, dt)
    assert st == 0
    ref = oracle.state_copy(d)
    assert oracle.drift(ref, G, dt) == 0
    tol = 2e-15 * max(1.0, abs(dt) / 6.0) * 10
    assert _err(out, ref, "xyz") < tol
    assert _err(out, ref, ("vx", "vy", "vz")) < tol


def test_kepler_host_bound_and_unbound(kep):
    rng = np.random.default_rng(3)
    n = 500
    r = rng.uniform(0.3, 3.0, n)
    th = rng.uniform(0, 2 * np.pi, n)
    vc = np.sqrt(G / r)
    fac = rng.uniform(0.2, 1.9, n)
    d = dict(x=r * np.cos(th), y=r * np.sin(th), z=rng.normal(0, 0.01, n),
             vx=-fac * vc * np.sin(th) + rng.normal(0, 0.1, n) * vc, vy=fac * vc * np.cos(th),
             vz=rng.normal(0, 0.02, n) * vc, m=np.zeros(n))
    out, st = _run(kep, d, G, 20.0)
    assert st == 0
    ref = oracle.state_copy(d)
    assert oracle.drift(ref, G, 20.0) == 0
    assert _err(out, ref, "xyz") < 1e-12


def test_kepler_host_exact_root_terminates(kep):
    # a body whose Newton iteration hits a zero residual exactly: the solver
    # must stop there instead of leaving the bracket
    d = W.make_disk(W.DISK_2048)
    one = {k: d[k][48:49].copy() for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
    out, st = _run(kep, one, G, 6.0)
    ref = oracle.state_copy(one)
    oracle.drift(ref, G, 6.0)
    assert st == 0 and _err(out, ref, "xyz") < 1e-15


def _vjp(L, S, B, mu, dt):
    S = np.ascontiguousarray(S, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64).copy()
    st = L.kepler_vjp_host(mu, dt, S.shape[0], S.ctypes.data, B.ctypes.data)
    return B, st


@pytest.mark.parametrize("dt", [6.0, 130.0, -40.0])
def test_kepler_vjp_matches_autograd(kep, dt):
    import torch
    from oracle import torch_ref as T
    d = W.make_disk(W.DISK_2048)
    n = 300
    S = np.stack([d[k][:n] for k in ("x", "y", "z", "vx", "vy", "vz")], axis=1)
    rng = np.random.default_rng(11)
    B = rng.normal(size=(n, 6))
    got, st = _vjp(kep, S, B, G, dt)
    assert st == 0
    x = torch.tensor(S[:, :3], requires_grad=True)
    v = torch.tensor(S[:, 3:], requires_grad=True)
    x1, v1 = T.drift(x, v, G, dt)
    L = (x1 * torch.tensor(B[:, :3])).sum() + (v1 * torch.tensor(B[:, 3:])).sum()
    gx, gv = torch.autograd.grad(L, (x, v))
    ref = np.concatenate([gx.numpy(), gv.numpy()], axis=1)
    err = np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)
    assert err.max() < 1e-10, err.max()


def test_kepler_vjp_unbound_orbits_fd(kep):
    # hyperbolic and near-parabolic orbits: central differences of the host solver
    rng = np.random.default_rng(4)
    n = 60
    r = rng.uniform(0.4, 2.0, n)
    th = rng.uniform(0, 2 * np.pi, n)
    vesc = np.sqrt(2 * G / r)
    fac = rng.uniform(1.05, 2.5, n)
    S = np.stack([r * np.cos(th), r * np.sin(th), rng.normal(0, 0.02, n),
                  -fac * vesc * np.sin(th) * 0.8, fac * vesc * np.cos(th) * 0.6 + 0.1 * vesc,
                  rng.normal(0, 0.05, n) * vesc], axis=1)
    B = rng.normal(size=(n, 6))
    dt = 25.0
    got, st = _vjp(kep, S, B, G, dt)
    assert st == 0
    scale = np.concatenate([np.full(3, 1.0), np.full(3, 0.02)])
    for k in range(6):
        h = 1e-6 * scale[k]
        Sp, Sm = S.copy(), S.copy()
        Sp[:, k] += h
        Sm[:, k] -= h
        outp = {c: Sp[:, i].copy() for i, c in enumerate(("x", "y", "z", "vx", "vy", "vz"))}
        outm = {c: Sm[:, i].copy() for i, c in enumerate(("x", "y", "z", "vx", "vy", "vz"))}
        assert kep.kepler_host(G, dt, n, *(outp[c].ctypes.data for c in ("x", "y", "z", "vx", "vy", "vz"))) == 0
        assert kep.kepler_host(G, dt, n, *(outm[c].ctypes.data for c in ("x", "y", "z", "vx", "vy", "vz"))) == 0
        P = np.stack([outp[c] for c in ("x", "y", "z", "vx", "vy", "vz")], axis=1)
        M = np.stack([outm[c] for c in ("x", "y", "z", "vx", "vy", "vz")], axis=1)
        fd = ((P - M) * B).sum(1) / (2 * h)
        assert np.max(np.abs(got[:, k] - fd) / (np.abs(fd) + 1e-3 * np.abs(got).max())) < 1e-5
