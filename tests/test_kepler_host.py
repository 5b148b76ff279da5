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
