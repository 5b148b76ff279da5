"""CPU oracle: slow, plain FP64 reference implementation of the method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; only the tests, the smoke check and the benchmark's CPU-baseline leg
use it.  It shares no code with the HIP library (paper_2201_10058_amd).

Contents:
  genga_oracle.c  - C implementation (kick, pairs, rcrit, HC, drift, step,
                    energy), loaded here through ctypes.
  torch_ref.py    - plain PyTorch float64 CPU re-statement of the same maps,
                    used with torch.autograd as the reference for the adjoint.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgenga_oracle.so")
_lib = None

OK = 0
E_NONFINITE = -3
E_NOCONV = -6

_d = ctypes.c_double
_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.or_changeover_y.restype = _d
    lib.or_changeover_y.argtypes = [_d]
    lib.or_changeover_dy.restype = _d
    lib.or_changeover_dy.argtypes = [_d]
    lib.or_changeover.restype = _d
    lib.or_changeover.argtypes = [_d, _d]
    lib.or_rcrit.restype = None
    lib.or_rcrit.argtypes = [_i64] + [_p] * 7 + [_d] * 4 + [_p]
    lib.or_kick_acc.restype = ctypes.c_int
    lib.or_kick_acc.argtypes = [_i64] + [_p] * 5 + [_d, _i64, _i64, ctypes.c_int] + [_p] * 3
    lib.or_kick_acc_tp.restype = ctypes.c_int
    lib.or_kick_acc_tp.argtypes = ([_i64] + [_p] * 5 + [_d, _i64, ctypes.c_int, _i64, _i64, ctypes.c_int]
                                   + [_p] * 3)
    lib.or_pairs_tp.restype = _i64
    lib.or_pairs_tp.argtypes = [_i64] + [_p] * 4 + [_i64, ctypes.c_int, _i64, _p, _p]
    lib.or_step_tp.restype = _i64
    lib.or_step_tp.argtypes = [_i64] + [_p] * 8 + [_d] * 5 + [_i64, ctypes.c_int, _i64, _p, _p, _p]
    lib.or_step_levels.restype = _i64
    lib.or_step_levels.argtypes = ([_i64] + [_p] * 8 + [_d] * 5
                                   + [ctypes.c_int, ctypes.c_int, _i64, _p, _p, _p, _p])
    lib.or_step_direct.restype = _i64
    lib.or_step_direct.argtypes = ([_i64] + [_p] * 8 + [_d] * 5
                                   + [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64, _i64]
                                   + [_p] * 5)
    lib.or_step_coll.restype = _i64
    lib.or_step_coll.argtypes = ([_i64] + [_p] * 9 + [_d] * 5
                                 + [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64, _d, _i64]
                                 + [_p] * 4 + [_i64] + [_p] * 5)
    lib.or_groups.restype = None
    lib.or_groups.argtypes = [_i64, _p, _p, _i64, _p]
    lib.or_direct_group.restype = None
    lib.or_direct_group.argtypes = ([_i64] + [_p] * 8 + [ctypes.c_int, _d, _d, _p, _i64, _d, _i64])
    lib.or_gr_kick.restype = None
    lib.or_gr_kick.argtypes = [_i64] + [_p] * 7 + [_d] * 4
    lib.or_step_gr.restype = _i64
    lib.or_step_gr.argtypes = [_i64] + [_p] * 8 + [_d] * 6 + [_i64, _p, _p, _p]
    lib.or_kick.restype = ctypes.c_int
    lib.or_kick.argtypes = [_i64] + [_p] * 8 + [_d, _d]
    lib.or_pairs.restype = _i64
    lib.or_pairs.argtypes = [_i64] + [_p] * 4 + [_i64, _p, _p]
    lib.or_hc.restype = None
    lib.or_hc.argtypes = [_i64] + [_p] * 7 + [_d, _d]
    lib.or_drift.restype = ctypes.c_int
    lib.or_drift.argtypes = [_i64] + [_p] * 6 + [_d, _d]
    lib.or_step.restype = _i64
    lib.or_step.argtypes = [_i64] + [_p] * 8 + [_d] * 5 + [_i64, _p, _p, _p]
    lib.or_energy.restype = _d
    lib.or_energy.argtypes = [_i64] + [_p] * 7 + [_d, _d]
    lib.or_changeover_integral.restype = _d
    lib.or_changeover_integral.argtypes = [_d, _d]
    lib.or_energy_k.restype = _d
    lib.or_energy_k.argtypes = [_i64] + [_p] * 8 + [_d, _d]
    lib.or_level_weight.restype = _d
    lib.or_level_weight.argtypes = [_d, _p, ctypes.c_int, ctypes.c_int]
    lib.or_num_threads.restype = ctypes.c_int
    lib.or_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def changeover_y(y: float) -> float:
    return _load().or_changeover_y(float(y))


def changeover_dy(y: float) -> float:
    return _load().or_changeover_dy(float(y))


def changeover(r: float, rho: float) -> float:
    return _load().or_changeover(float(r), float(rho))


def rcrit(x, y, z, vx, vy, vz, m, m_star, dt, n1, n2):
    arrs = [_f64(a) for a in (x, y, z, vx, vy, vz, m)]
    n = arrs[0].size
    rc = np.empty(n)
    _load().or_rcrit(n, *map(_ptr, arrs), float(m_star), float(dt), float(n1), float(n2), _ptr(rc))
    return rc


def kick_acc(x, y, z, m, rc, G, rows=None, precise=True):
    """Accelerations for rows [i0, i1) (all rows by default).

    Returns (ax, ay, az, status).
    """
    arrs = [_f64(a) for a in (x, y, z, m, rc)]
    n = arrs[0].size
    i0, i1 = (0, n) if rows is None else rows
    k = max(i1 - i0, 0)
    ax, ay, az = np.zeros(k), np.zeros(k), np.zeros(k)
    st = _load().or_kick_acc(n, *map(_ptr, arrs), float(G), int(i0), int(i1), int(bool(precise)),
                             _ptr(ax), _ptr(ay), _ptr(az))
    return ax, ay, az, st


def kick_acc_tp(x, y, z, m, rc, G, nm, mode, rows=None, precise=True):
    """Accelerations in test-particle mode `mode` (bodies [0, nm) massive)."""
    arrs = [_f64(a) for a in (x, y, z, m, rc)]
    n = arrs[0].size
    i0, i1 = (0, n) if rows is None else rows
    k = max(i1 - i0, 0)
    ax, ay, az = np.zeros(k), np.zeros(k), np.zeros(k)
    st = _load().or_kick_acc_tp(n, *map(_ptr, arrs), float(G), int(nm), int(mode), int(i0), int(i1),
                                int(bool(precise)), _ptr(ax), _ptr(ay), _ptr(az))
    return ax, ay, az, st


def pairs_tp(x, y, z, rc, nm, mode, cap=None):
    """Canonical close-encounter list in test-particle mode `mode`."""
    arrs = [_f64(a) for a in (x, y, z, rc)]
    n = arrs[0].size
    lib = _load()
    if cap is None:
        cap = lib.or_pairs_tp(n, *map(_ptr, arrs), int(nm), int(mode), 0, None, None)
    pi = np.zeros(max(cap, 1), dtype=np.int32)
    pj = np.zeros(max(cap, 1), dtype=np.int32)
    cnt = lib.or_pairs_tp(n, *map(_ptr, arrs), int(nm), int(mode), int(cap), _ptr(pi), _ptr(pj))
    k = min(cnt, cap)
    return pi[:k].copy(), pj[:k].copy(), int(cnt)


def step_tp(state, G, m_star, dt, n1, n2, nm, mode, cap=1 << 20):
    """One base step in place in test-particle mode `mode`.
    Returns (pi, pj, count, rc, status)."""
    n = state["x"].size
    rc = np.empty(n)
    pi = np.zeros(max(cap, 1), dtype=np.int32)
    pj = np.zeros(max(cap, 1), dtype=np.int32)
    st = ctypes.c_int(0)
    cnt = _load().or_step_tp(n, *(_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                             _ptr(rc), float(G), float(m_star), float(dt), float(n1), float(n2),
                             int(nm), int(mode), int(cap), _ptr(pi), _ptr(pj), ctypes.byref(st))
    k = min(cnt, cap)
    return pi[:k].copy(), pj[:k].copy(), int(cnt), rc, st.value


def step_levels(state, G, m_star, dt, n1, n2, levels, substeps, cap=1 << 20):
    """One base step in place with `levels` symplectic levels of `substeps`
    sub-steps (levels = 1 is `step`).  Returns (pi, pj, count, rc, counts,
    status): the level-0 list, its count, the level-0 radii and the summed
    list sizes found at each level."""
    n = state["x"].size
    rc = np.empty(n)
    pi = np.zeros(max(cap, 1), dtype=np.int32)
    pj = np.zeros(max(cap, 1), dtype=np.int32)
    counts = np.zeros(max(int(levels), 1), dtype=np.int64)
    st = ctypes.c_int(0)
    cnt = _load().or_step_levels(n, *(_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                                 _ptr(rc), float(G), float(m_star), float(dt), float(n1), float(n2),
                                 int(levels), int(substeps), int(cap), _ptr(pi), _ptr(pj),
                                 _ptr(counts), ctypes.byref(st))
    k = min(cnt, cap)
    return pi[:k].copy(), pj[:k].copy(), int(cnt), rc, counts, st.value


def step_direct(state, G, m_star, dt, n1, n2, levels, substeps, rk_steps=2000, cap=1 << 20):
    """One step with levels and the direct solver for the deepest level's
    groups.  Returns (pi, pj, count, rc, counts, (groups, largest), status)."""
    n = state["x"].size
    rc = np.empty(n)
    pi = np.zeros(max(cap, 1), dtype=np.int32)
    pj = np.zeros(max(cap, 1), dtype=np.int32)
    counts = np.zeros(max(int(levels), 1), dtype=np.int64)
    gstats = np.zeros(2, dtype=np.int64)
    st = ctypes.c_int(0)
    cnt = _load().or_step_direct(n, *(_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                                 _ptr(rc), float(G), float(m_star), float(dt), float(n1), float(n2),
                                 int(levels), int(substeps), 1, int(rk_steps), int(cap), _ptr(pi),
                                 _ptr(pj), _ptr(counts), _ptr(gstats), ctypes.byref(st))
    k = min(cnt, cap)
    return pi[:k].copy(), pj[:k].copy(), int(cnt), rc, counts, (int(gstats[0]), int(gstats[1])), st.value


def step_coll(state, G, m_star, dt, n1, n2, levels, substeps, rk_steps=2000, coll_tol=1e-6,
              capcoll=1024, cap=1 << 20):
    """One step with levels, the direct solver and collisions (state["R"]:
    radii; m and R are updated by mergers).  Returns (pairs count, counts,
    (groups, largest), [(survivor, absorbed, lost energy), ...], status)."""
    n = state["x"].size
    rc = np.empty(n)
    pi = np.zeros(max(cap, 1), dtype=np.int32)
    pj = np.zeros(max(cap, 1), dtype=np.int32)
    counts = np.zeros(max(int(levels), 1), dtype=np.int64)
    gstats = np.zeros(2, dtype=np.int64)
    ci = np.zeros(max(capcoll, 1), dtype=np.int32)
    cj = np.zeros(max(capcoll, 1), dtype=np.int32)
    cdu = np.zeros(max(capcoll, 1), dtype=np.float64)
    nc = np.zeros(1, dtype=np.int64)
    st = ctypes.c_int(0)
    cnt = _load().or_step_coll(n, *(_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "R")),
                               _ptr(rc), float(G), float(m_star), float(dt), float(n1), float(n2),
                               int(levels), int(substeps), 1, int(rk_steps), float(coll_tol),
                               int(capcoll), _ptr(ci), _ptr(cj), _ptr(cdu), _ptr(nc), int(cap),
                               _ptr(pi), _ptr(pj), _ptr(counts), _ptr(gstats), ctypes.byref(st))
    k = int(min(nc[0], capcoll))
    coll = [(int(ci[q]), int(cj[q]), float(cdu[q])) for q in range(k)]
    return int(cnt), counts, (int(gstats[0]), int(gstats[1])), coll, st.value


def groups(n, pi, pj):
    """Connected components of the pair graph: label = smallest body of the
    group for the list's bodies, -1 elsewhere."""
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    label = np.zeros(max(int(n), 1), dtype=np.int32)
    _load().or_groups(int(n), _ptr(pi), _ptr(pj), int(pi.size), _ptr(label))
    return label[:n]


def direct_group(state, rc_levels, G, m_star, members, dt, steps=2000):
    """Advance the members of one group in place by the direct solver's
    flow (RK4); rc_levels: (levels used, n) radii."""
    n = state["x"].size
    rcl = np.ascontiguousarray(rc_levels, dtype=np.float64).reshape(-1, n)
    mem = np.ascontiguousarray(members, dtype=np.int64)
    _load().or_direct_group(n, *(_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                            _ptr(rcl), rcl.shape[0] - 1, float(G), float(m_star), _ptr(mem),
                            int(mem.size), float(dt), int(steps))


def gr_kick(state, G, m_star, c, h):
    """In-place post-Newtonian velocity update over h (implicit midpoint)."""
    n = state["x"].size
    _load().or_gr_kick(n, *(_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                       float(G), float(m_star), float(c), float(h))


def step_gr(state, G, m_star, dt, n1, n2, c, cap=1 << 20):
    """One base step with the post-Newtonian term; (pi, pj, count, rc, status)."""
    n = state["x"].size
    rc = np.empty(n)
    pi = np.zeros(max(cap, 1), dtype=np.int32)
    pj = np.zeros(max(cap, 1), dtype=np.int32)
    st = ctypes.c_int(0)
    cnt = _load().or_step_gr(n, *(_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                             _ptr(rc), float(G), float(m_star), float(dt), float(n1), float(n2),
                             float(c), int(cap), _ptr(pi), _ptr(pj), ctypes.byref(st))
    k = min(cnt, cap)
    return pi[:k].copy(), pj[:k].copy(), int(cnt), rc, st.value


def kick(state, rc, G, h):
    """In-place v += h a (plain binary64 sums)."""
    n = state["x"].size
    return _load().or_kick(n, *(_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                           _ptr(_f64(rc)), float(G), float(h))


def pairs(x, y, z, rc, cap=None):
    """Canonical close-encounter list (i < j, i asc, j asc) and true count."""
    arrs = [_f64(a) for a in (x, y, z, rc)]
    n = arrs[0].size
    lib = _load()
    if cap is None:
        cnt = lib.or_pairs(n, *map(_ptr, arrs), 0, None, None)
        cap = cnt
    pi = np.zeros(max(cap, 1), dtype=np.int32)
    pj = np.zeros(max(cap, 1), dtype=np.int32)
    cnt = lib.or_pairs(n, *map(_ptr, arrs), int(cap), _ptr(pi), _ptr(pj))
    k = min(cnt, cap)
    return pi[:k].copy(), pj[:k].copy(), int(cnt)


def hc(state, m_star, h):
    n = state["x"].size
    _load().or_hc(n, *(_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                  float(m_star), float(h))


def drift(state, mu, dt):
    n = state["x"].size
    return _load().or_drift(n, *(_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz")),
                            float(mu), float(dt))


def step(state, G, m_star, dt, n1, n2, cap=None):
    """One base step in place.  Returns (pi, pj, count, rc, status)."""
    n = state["x"].size
    lib = _load()
    rc = np.empty(n)
    if cap is None:
        rc0 = rcrit(state["x"], state["y"], state["z"], state["vx"], state["vy"], state["vz"],
                    state["m"], m_star, dt, n1, n2)
        cap = pairs(state["x"], state["y"], state["z"], rc0, cap=0)[2]
    pi = np.zeros(max(cap, 1), dtype=np.int32)
    pj = np.zeros(max(cap, 1), dtype=np.int32)
    st = ctypes.c_int(0)
    cnt = lib.or_step(n, *(_ptr(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                      _ptr(rc), float(G), float(m_star), float(dt), float(n1), float(n2),
                      int(cap), _ptr(pi), _ptr(pj), ctypes.byref(st))
    k = min(cnt, cap)
    return pi[:k].copy(), pj[:k].copy(), int(cnt), rc, st.value


def energy(state, G, m_star):
    n = state["x"].size
    return _load().or_energy(n, *(_ptr(_f64(state[k])) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                             float(G), float(m_star))


def level_weight(r: float, rho, l: int) -> float:
    """W_l(r) for the level radii rho (l < len(rho)); l = len(rho): the
    remainder no level takes."""
    rr = np.ascontiguousarray(rho, dtype=np.float64)
    return _load().or_level_weight(float(r), _ptr(rr), int(rr.size), int(l))


def changeover_integral(r: float, rho: float) -> float:
    """int_{max(r, 0.1 rho)}^{rho} K(s)/s^2 ds (0 for r >= rho)."""
    return _load().or_changeover_integral(float(r), float(rho))


def energy_k(state, rc, G, m_star):
    """E with the changeover potential for the pairs inside rho_ij."""
    n = state["x"].size
    return _load().or_energy_k(n, *(_ptr(_f64(state[k])) for k in ("x", "y", "z", "vx", "vy", "vz", "m")),
                               _ptr(_f64(rc)), float(G), float(m_star))


def num_threads() -> int:
    return _load().or_num_threads()


def set_num_threads(t: int) -> None:
    _load().or_set_num_threads(int(t))


def state_copy(d):
    """Contiguous float64 copies of the state arrays of a workload dict."""
    return {k: np.array(d[k], dtype=np.float64, copy=True) for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
