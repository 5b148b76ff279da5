"""Oracle accelerations of whole benchmark disks, computed once per process.

The compensated (long double, Neumaier) oracle kick of a 65,536-body disk
takes 15-40 s of host time; several GPU tests compare all of its rows, so
the result is kept for the life of the test process.  Only oracle/ and the
input generators are used here.
"""
from __future__ import annotations

import functools

import numpy as np

import oracle
from paper_2201_10058_amd import workload as W

G = W.GAUSS_G


def disk_rc(d, n2=0.4):
    """Critical radii of eq. (rcrit) for a disk state (n1 = 3, dt = 6 d)."""
    return oracle.rcrit(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["m"], 1.0, 6.0, 3.0,
                        n2)


@functools.lru_cache(maxsize=None)
def disk(spec: W.DiskSpec):
    """(state, rc) of a disk; the arrays must not be modified by callers."""
    d = W.make_disk(spec)
    return d, disk_rc(d, spec.n2)


@functools.lru_cache(maxsize=None)
def disk_acc(spec: W.DiskSpec):
    """Compensated oracle accelerations (3, N) of every body of the disk."""
    d, rc = disk(spec)
    ax, ay, az, st = oracle.kick_acc(d["x"], d["y"], d["z"], d["m"], rc, G, precise=True)
    assert st == 0
    return np.stack([ax, ay, az])


@functools.lru_cache(maxsize=None)
def disk_pairs(spec: W.DiskSpec):
    """Brute-force encounter list (i, j, count) of the disk at its rc."""
    d, rc = disk(spec)
    return oracle.pairs(d["x"], d["y"], d["z"], rc, cap=1 << 21)


def rel_err(a, ref):
    """Relative error per acceleration, ||a_i - ref_i|| / ||ref_i||."""
    return np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)
