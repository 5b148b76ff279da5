"""Thin ctypes binding of libgenga.so (include/genga.h).

Only argument marshalling happens here: torch tensors provide device memory
and the current HIP stream; every step of the computation runs in the HIP
kernels of libgenga.so.  The binding fails loudly if the library or a GPU is
missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgenga.so")

OK = 0
E_INVAL = -1
E_OVERFLOW = -2
E_NONFINITE = -3
E_HIP = -4
E_UNSUPPORTED = -5
E_NOCONV = -6
E_RCRIT = -7
E_GROUP = -8
E_SCRATCH = -9

FP64 = 0
MIXED = 1
FLAG_NOSYNC = 1
FLAG_DIRECTED = 2     # binary64 kick: one-sided form at any n
FLAG_SYMMETRIC = 4    # binary64 kick: symmetric form at any n

_c_double_p = ctypes.c_void_p


class Bodies(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in
                                           ("x", "y", "z", "vx", "vy", "vz", "m", "rc", "R")]


class Params(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("m_star", ctypes.c_double), ("dt", ctypes.c_double),
                ("n1", ctypes.c_double), ("n2", ctypes.c_double), ("precision", ctypes.c_int),
                ("flags", ctypes.c_int), ("ipt", ctypes.c_int), ("slices", ctypes.c_int),
                ("block", ctypes.c_int), ("tile_cols", ctypes.c_int), ("grid", ctypes.c_int),
                ("prof_events", ctypes.c_void_p * 4), ("tp_mode", ctypes.c_int),
                ("slevels", ctypes.c_int), ("n_massive", ctypes.c_int64),
                ("substeps", ctypes.c_int), ("direct", ctypes.c_int),
                ("level_capacity", ctypes.c_int64), ("bs_eps", ctypes.c_double),
                ("c_light", ctypes.c_double), ("coll_tol", ctypes.c_double)]


class BatchC(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int64), ("offsets", ctypes.c_void_p), ("m_star", ctypes.c_void_p),
                ("dt", ctypes.c_void_p), ("n1", ctypes.c_void_p), ("n2", ctypes.c_void_p)]


class Adjoint(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "rc")]


class Pairs(ctypes.Structure):
    _fields_ = [("i", ctypes.c_void_p), ("j", ctypes.c_void_p), ("capacity", ctypes.c_int64),
                ("count", ctypes.c_void_p)]


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "genga_version": (ctypes.c_int, []),
    "genga_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "genga_last_hip_error": (ctypes.c_int, []),
    "genga_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.POINTER(Params)]),
    "genga_read_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "genga_clear_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "genga_rcrit": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params), ctypes.c_void_p,
                                   ctypes.c_void_p]),
    "genga_kick": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params), ctypes.c_double,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.POINTER(Pairs), ctypes.c_void_p, ctypes.c_void_p]),
    "genga_kick_static": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params),
                                         ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.POINTER(Pairs), ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "genga_encounter_pairs": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params),
                                             ctypes.POINTER(Pairs), ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "genga_hc": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params), ctypes.c_double,
                                ctypes.c_void_p, ctypes.c_void_p]),
    "genga_drift": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params), ctypes.c_double,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "genga_step": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params),
                                  ctypes.POINTER(Pairs), ctypes.c_void_p, ctypes.c_void_p]),
    "genga_tune_levels": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params),
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "genga_energy_k": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params),
                                      ctypes.POINTER(Pairs), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "genga_gr_kick": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params), ctypes.c_double,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "genga_collisions": (ctypes.c_int, [ctypes.c_int64, ctypes.POINTER(Params), ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "genga_group_stats": (ctypes.c_int, [ctypes.c_int64, ctypes.POINTER(Params), ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "genga_level_counts": (ctypes.c_int, [ctypes.c_int64, ctypes.POINTER(Params), ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "genga_energy": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params),
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "genga_kick_vjp": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params), ctypes.c_double,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(Adjoint), ctypes.c_void_p, ctypes.c_void_p]),
    "genga_rcrit_vjp": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params),
                                       ctypes.POINTER(Adjoint), ctypes.c_void_p, ctypes.c_void_p]),
    "genga_hc_vjp": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params), ctypes.c_double,
                                    ctypes.POINTER(Adjoint), ctypes.c_void_p, ctypes.c_void_p]),
    "genga_drift_vjp": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params), ctypes.c_double,
                                       ctypes.POINTER(Adjoint), ctypes.c_void_p, ctypes.c_void_p]),
    "genga_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(BatchC), ctypes.POINTER(Params)]),
    "genga_batch_plan": (ctypes.c_int, [ctypes.POINTER(BatchC), ctypes.POINTER(Params),
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "genga_batch_info": (ctypes.c_int, [ctypes.POINTER(BatchC), ctypes.POINTER(Params),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "genga_kick_batched": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(BatchC),
                                          ctypes.POINTER(Params), ctypes.c_double, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Pairs),
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "genga_autotune_batched_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(BatchC),
                                                                 ctypes.POINTER(Params)]),
    "genga_autotune_batched": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(BatchC),
                                              ctypes.POINTER(Params), ctypes.c_void_p,
                                              ctypes.c_size_t, ctypes.c_char_p,
                                              ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "genga_autotune_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.POINTER(Params)]),
    "genga_autotune": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(Params), ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.c_char_p,
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "genga_step_batched": (ctypes.c_int, [ctypes.POINTER(Bodies), ctypes.POINTER(BatchC),
                                          ctypes.POINTER(Params), ctypes.POINTER(Pairs),
                                          ctypes.c_void_p, ctypes.c_void_p]),
}

_lib = None


class GengaError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = load().genga_strerror(code).decode() if _lib is not None else str(code)
        if code == E_HIP:
            msg += f" (hipError {load().genga_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{code}]" if what else f"{msg} [{code}]")


def load(path: str = LIB_PATH):
    """Load libgenga.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libgenga.so not found at {path}; build it with "
                           "`python -m paper_2201_10058_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code: int, what: str):
    if code != OK:
        raise GengaError(code, what)


def _require_gpu(t: torch.Tensor, dtype=torch.float64):
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return t.data_ptr()


def _stream_ptr() -> int:
    return torch.cuda.current_stream().cuda_stream


@dataclass
class Config:
    G: float
    m_star: float = 1.0
    dt: float = 6.0
    n1: float = 3.0
    n2: float = 0.4
    precision: int = FP64
    flags: int = 0
    ipt: int = 0
    slices: int = 0
    block: int = 0
    tile_cols: int = 0
    grid: int = 0
    events: tuple = field(default=(None, None, None, None))
    tp_mode: int = 0
    n_massive: int = 0
    slevels: int = 0
    substeps: int = 0
    level_capacity: int = 0
    direct: int = 0
    bs_eps: float = 0.0
    c_light: float = 0.0
    coll_tol: float = 0.0

    def params(self) -> Params:
        p = Params(self.G, self.m_star, self.dt, self.n1, self.n2, self.precision, self.flags,
                   self.ipt, self.slices, self.block, self.tile_cols, self.grid)
        for k, e in enumerate(tuple(self.events)[:4]):
            p.prof_events[k] = e
        p.tp_mode = self.tp_mode
        p.n_massive = self.n_massive
        p.slevels = self.slevels
        p.substeps = self.substeps
        p.level_capacity = self.level_capacity
        p.direct = self.direct
        p.bs_eps = self.bs_eps
        p.c_light = self.c_light
        p.coll_tol = self.coll_tol
        return p


class State:
    """Device SoA state of one system (float64 tensors on the GPU)."""

    KEYS = ("x", "y", "z", "vx", "vy", "vz", "m", "rc")

    def __init__(self, tensors: dict):
        self.t = tensors
        self.n = int(tensors["x"].numel())
        for k in self.KEYS:
            _require_gpu(tensors[k])
            if tensors[k].numel() != self.n:
                raise ValueError(f"{k} has {tensors[k].numel()} elements, expected {self.n}")

    @classmethod
    def from_numpy(cls, d: dict, device="cuda:0", rc=None, radius=None):
        """radius: physical radii (enables collisions in the direct solver)."""
        t = {}
        for k in ("x", "y", "z", "vx", "vy", "vz", "m"):
            t[k] = torch.as_tensor(d[k], dtype=torch.float64).to(device).contiguous()
        src = rc if rc is not None else d.get("rc")
        if src is None:
            t["rc"] = torch.zeros_like(t["x"])
        else:
            t["rc"] = torch.as_tensor(src, dtype=torch.float64).to(device).contiguous()
        if radius is not None:
            t["R"] = torch.as_tensor(radius, dtype=torch.float64).to(device).contiguous()
        return cls(t)

    def bodies(self) -> Bodies:
        b = Bodies()
        b.n = self.n
        for k in self.KEYS:
            setattr(b, k, self.t[k].data_ptr())
        b.R = self.t["R"].data_ptr() if "R" in self.t else None
        return b

    def numpy(self) -> dict:
        return {k: v.detach().cpu().numpy().copy() for k, v in self.t.items()}


class PairList:
    """Device encounter list with a given capacity."""

    def __init__(self, capacity: int, device="cuda:0"):
        self.capacity = int(capacity)
        self.i = torch.zeros(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.j = torch.zeros(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)

    def struct(self) -> Pairs:
        return Pairs(self.i.data_ptr(), self.j.data_ptr(), self.capacity, self.count.data_ptr())

    def result(self):
        c = int(self.count.item())
        k = min(c, self.capacity)
        return self.i[:k].cpu().numpy(), self.j[:k].cpu().numpy(), c


class Workspace:
    """Caller-owned scratch for a system size and configuration."""

    def __init__(self, n: int, cfg: Config, device="cuda:0"):
        lib = load()
        p = cfg.params()
        nbytes = lib.genga_workspace_bytes(int(n), ctypes.byref(p))
        if nbytes == 0:
            raise GengaError(E_INVAL, "workspace size")
        self.buf = torch.zeros(int(nbytes), dtype=torch.uint8, device=device)
        self.nbytes = int(nbytes)

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()


def read_status(ws: Workspace) -> int:
    return load().genga_read_status(ctypes.c_void_p(ws.ptr), ctypes.c_void_p(_stream_ptr()))


def kick_static(state: State, cfg: Config, h: float, acc: bool = False,
                pairs: PairList | None = None):
    """genga_kick_static: the kick with the library's static scratch (no
    workspace).  Returns (a or None, status) where status is a device int32
    tensor that receives the call's status code."""
    b, p = state.bodies(), cfg.params()
    a = None
    ptrs = (None, None, None)
    if acc:
        a = torch.empty((3, state.n), dtype=torch.float64, device=state.t["x"].device)
        ptrs = (a[0].data_ptr(), a[1].data_ptr(), a[2].data_ptr())
    status = torch.full((1,), -100, dtype=torch.int32, device=state.t["x"].device)
    ps = pairs.struct() if pairs is not None else None
    _check(load().genga_kick_static(ctypes.byref(b), ctypes.byref(p), float(h), ptrs[0], ptrs[1],
                                    ptrs[2], ctypes.byref(ps) if ps is not None else None,
                                    ctypes.c_void_p(status.data_ptr()),
                                    ctypes.c_void_p(_stream_ptr())), "genga_kick_static")
    return a, status


def rcrit(state: State, cfg: Config, ws: Workspace):
    b, p = state.bodies(), cfg.params()
    _check(load().genga_rcrit(ctypes.byref(b), ctypes.byref(p), ctypes.c_void_p(ws.ptr),
                              ctypes.c_void_p(_stream_ptr())), "genga_rcrit")


def kick(state: State, cfg: Config, ws: Workspace, h: float, acc: bool = False,
         pairs: PairList | None = None):
    """v += h a (h may be 0); optionally return a (3, n) and fill pairs."""
    b, p = state.bodies(), cfg.params()
    a = None
    ptrs = (None, None, None)
    if acc:
        a = torch.empty((3, state.n), dtype=torch.float64, device=state.t["x"].device)
        ptrs = (a[0].data_ptr(), a[1].data_ptr(), a[2].data_ptr())
    ps = pairs.struct() if pairs is not None else None
    _check(load().genga_kick(ctypes.byref(b), ctypes.byref(p), float(h), ptrs[0], ptrs[1], ptrs[2],
                             ctypes.byref(ps) if ps is not None else None, ctypes.c_void_p(ws.ptr),
                             ctypes.c_void_p(_stream_ptr())), "genga_kick")
    return a


def encounter_pairs(state: State, cfg: Config, ws: Workspace, pairs: PairList):
    b, p, ps = state.bodies(), cfg.params(), pairs.struct()
    _check(load().genga_encounter_pairs(ctypes.byref(b), ctypes.byref(p), ctypes.byref(ps),
                                        ctypes.c_void_p(ws.ptr), ctypes.c_void_p(_stream_ptr())),
           "genga_encounter_pairs")


def hc(state: State, cfg: Config, ws: Workspace, h: float):
    b, p = state.bodies(), cfg.params()
    _check(load().genga_hc(ctypes.byref(b), ctypes.byref(p), float(h), ctypes.c_void_p(ws.ptr),
                           ctypes.c_void_p(_stream_ptr())), "genga_hc")


def drift(state: State, cfg: Config, ws: Workspace, dt: float):
    b, p = state.bodies(), cfg.params()
    _check(load().genga_drift(ctypes.byref(b), ctypes.byref(p), float(dt), ctypes.c_void_p(ws.ptr),
                              ctypes.c_void_p(_stream_ptr())), "genga_drift")


def step(state: State, cfg: Config, ws: Workspace, pairs: PairList | None = None) -> int:
    """One base step; returns the status code (raises on argument/HIP errors)."""
    b, p = state.bodies(), cfg.params()
    ps = pairs.struct() if pairs is not None else None
    code = load().genga_step(ctypes.byref(b), ctypes.byref(p),
                             ctypes.byref(ps) if ps is not None else None, ctypes.c_void_p(ws.ptr),
                             ctypes.c_void_p(_stream_ptr()))
    if code in (E_INVAL, E_HIP, E_UNSUPPORTED):
        raise GengaError(code, "genga_step")
    return code


def level_counts(n: int, cfg: Config, ws: Workspace):
    """Sizes of the symplectic levels' lists in the last step (numpy int64
    array of cfg.slevels entries; synchronises the stream)."""
    import numpy as np
    out = np.zeros(max(cfg.slevels, 1), dtype=np.int64)
    p = cfg.params()
    _check(load().genga_level_counts(n, ctypes.byref(p), ctypes.c_void_p(ws.ptr),
                                     out.ctypes.data_as(ctypes.c_void_p),
                                     ctypes.c_void_p(_stream_ptr())), "genga_level_counts")
    return out


def energy_k(state: State, cfg: Config, ws: Workspace, pairs: PairList, out=None):
    """Energy parts and E_K: float64 device tensor (E, T, U_*, U, C, E_K);
    `pairs` receives the encounter list of the current positions."""
    if out is None:
        out = torch.empty(6, dtype=torch.float64, device=state.t["x"].device)
    b, p, ps = state.bodies(), cfg.params(), pairs.struct()
    _check(load().genga_energy_k(ctypes.byref(b), ctypes.byref(p), ctypes.byref(ps),
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.ptr),
                                 ctypes.c_void_p(_stream_ptr())), "genga_energy_k")
    return out


def gr_kick(state: State, cfg: Config, ws: Workspace, h: float) -> None:
    """Post-Newtonian velocity update over h (asynchronous)."""
    b, p = state.bodies(), cfg.params()
    _check(load().genga_gr_kick(ctypes.byref(b), ctypes.byref(p), ctypes.c_double(h),
                                ctypes.c_void_p(ws.ptr), ctypes.c_void_p(_stream_ptr())),
           "genga_gr_kick")


def collisions(n: int, cfg: Config, ws: Workspace, cap: int = 4096):
    """Mergers of the last step: (count, [(survivor, absorbed, lost energy), ...])
    sorted by (survivor, absorbed)."""
    import numpy as np
    c = np.zeros(1, dtype=np.int64)
    i = np.zeros(max(cap, 1), dtype=np.int32)
    j = np.zeros(max(cap, 1), dtype=np.int32)
    du = np.zeros(max(cap, 1), dtype=np.float64)
    p = cfg.params()
    _check(load().genga_collisions(n, ctypes.byref(p), ctypes.c_void_p(ws.ptr),
                                   c.ctypes.data_as(ctypes.c_void_p), i.ctypes.data_as(ctypes.c_void_p),
                                   j.ctypes.data_as(ctypes.c_void_p), du.ctypes.data_as(ctypes.c_void_p),
                                   int(cap), ctypes.c_void_p(_stream_ptr())), "genga_collisions")
    k = int(min(c[0], cap, 4096))
    return int(c[0]), [(int(i[q]), int(j[q]), float(du[q])) for q in range(k)]


def group_stats(n: int, cfg: Config, ws: Workspace):
    """(groups integrated, largest group) of the last step's direct solver."""
    import numpy as np
    out = np.zeros(2, dtype=np.int64)
    p = cfg.params()
    _check(load().genga_group_stats(n, ctypes.byref(p), ctypes.c_void_p(ws.ptr),
                                    out.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.c_void_p(_stream_ptr())), "genga_group_stats")
    return int(out[0]), int(out[1])


def energy(state: State, cfg: Config, ws: Workspace, out=None):
    """Energy parts (E, T, U_*, U, C) as a float64 device tensor of 5
    (asynchronous; read the status afterwards for coincident bodies)."""
    if out is None:
        out = torch.empty(5, dtype=torch.float64, device=state.t["x"].device)
    b, p = state.bodies(), cfg.params()
    _check(load().genga_energy(ctypes.byref(b), ctypes.byref(p), ctypes.c_void_p(out.data_ptr()),
                               ctypes.c_void_p(ws.ptr), ctypes.c_void_p(_stream_ptr())),
           "genga_energy")
    return out


# ---------------------------------------------------------------------------
# Batched ensembles
# ---------------------------------------------------------------------------
class Batch:
    """S systems stored back to back; per-system parameters live on the GPU."""

    def __init__(self, offsets, m_star, dt, n1, n2, device="cuda:0"):
        import numpy as np
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)   # host
        self.S = len(self.offsets) - 1
        self.t = {k: torch.as_tensor(np.asarray(v, dtype=np.float64)).to(device).contiguous()
                  for k, v in (("m_star", m_star), ("dt", dt), ("n1", n1), ("n2", n2))}
        for v in self.t.values():
            if v.numel() != self.S:
                raise ValueError("per-system arrays must have S entries")

    def struct(self) -> BatchC:
        return BatchC(self.S, self.offsets.ctypes.data, self.t["m_star"].data_ptr(),
                      self.t["dt"].data_ptr(), self.t["n1"].data_ptr(), self.t["n2"].data_ptr())

    @property
    def n(self) -> int:
        return int(self.offsets[-1])


class BatchWorkspace:
    """Workspace holding a batch plan (built at construction)."""

    def __init__(self, batch: Batch, cfg: Config, device="cuda:0"):
        lib = load()
        self.bt = batch.struct()           # keeps the host offsets referenced
        self._batch = batch
        p = cfg.params()
        nbytes = lib.genga_batch_workspace_bytes(ctypes.byref(self.bt), ctypes.byref(p))
        if nbytes == 0:
            raise GengaError(E_INVAL, "batch workspace size")
        self.buf = torch.zeros(int(nbytes), dtype=torch.uint8, device=device)
        self.nbytes = int(nbytes)
        _check(lib.genga_batch_plan(ctypes.byref(self.bt), ctypes.byref(p), ctypes.c_void_p(self.ptr),
                                    ctypes.c_void_p(_stream_ptr())), "genga_batch_plan")
        info = (ctypes.c_int64 * 5)()
        _check(lib.genga_batch_info(ctypes.byref(self.bt), ctypes.byref(p), info), "genga_batch_info")
        self.info = dict(tiles=info[0], grid=info[1], block=info[2], ipt=info[3], tile_cols=info[4])

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()


def kick_batched(state: State, ws: BatchWorkspace, cfg: Config, hfac: float, acc: bool = False,
                 pairs: PairList | None = None):
    b, p = state.bodies(), cfg.params()
    a = None
    ptrs = (None, None, None)
    if acc:
        a = torch.empty((3, state.n), dtype=torch.float64, device=state.t["x"].device)
        ptrs = (a[0].data_ptr(), a[1].data_ptr(), a[2].data_ptr())
    ps = pairs.struct() if pairs is not None else None
    _check(load().genga_kick_batched(ctypes.byref(b), ctypes.byref(ws.bt), ctypes.byref(p), float(hfac),
                                     ptrs[0], ptrs[1], ptrs[2],
                                     ctypes.byref(ps) if ps is not None else None,
                                     ctypes.c_void_p(ws.ptr), ctypes.c_void_p(_stream_ptr())),
           "genga_kick_batched")
    return a


def step_batched(state: State, ws: BatchWorkspace, cfg: Config, pairs: PairList | None = None) -> int:
    b, p = state.bodies(), cfg.params()
    ps = pairs.struct() if pairs is not None else None
    code = load().genga_step_batched(ctypes.byref(b), ctypes.byref(ws.bt), ctypes.byref(p),
                                     ctypes.byref(ps) if ps is not None else None,
                                     ctypes.c_void_p(ws.ptr), ctypes.c_void_p(_stream_ptr()))
    if code in (E_INVAL, E_HIP, E_UNSUPPORTED):
        raise GengaError(code, "genga_step_batched")
    return code


def system_view(state: State, lo: int, hi: int) -> State:
    """State of bodies [lo, hi) (views into the same device memory)."""
    return State({k: v[lo:hi] for k, v in state.t.items()})


# ---------------------------------------------------------------------------
# Adjoint
# ---------------------------------------------------------------------------
class AdjointState:
    """Device adjoint arrays (float64, length n): x, y, z, vx, vy, vz, m, rc."""

    KEYS = ("x", "y", "z", "vx", "vy", "vz", "m", "rc")

    def __init__(self, n: int, device="cuda:0", tensors: dict | None = None):
        if tensors is None:
            tensors = {k: torch.zeros(n, dtype=torch.float64, device=device) for k in self.KEYS}
        self.t = tensors
        for k in self.KEYS:
            _require_gpu(self.t[k])

    def struct(self) -> Adjoint:
        return Adjoint(*(self.t[k].data_ptr() for k in self.KEYS))


def kick_vjp(state: State, cfg: Config, ws: Workspace, scale: float, abar, adj: AdjointState):
    """adj += VJP of the accelerations at `state` for abar (3 tensors)."""
    b, p, a = state.bodies(), cfg.params(), adj.struct()
    ptrs = [_require_gpu(t) for t in abar]
    _check(load().genga_kick_vjp(ctypes.byref(b), ctypes.byref(p), float(scale), ptrs[0], ptrs[1],
                                 ptrs[2], ctypes.byref(a), ctypes.c_void_p(ws.ptr),
                                 ctypes.c_void_p(_stream_ptr())), "genga_kick_vjp")


def rcrit_vjp(state: State, cfg: Config, ws: Workspace, adj: AdjointState):
    b, p, a = state.bodies(), cfg.params(), adj.struct()
    _check(load().genga_rcrit_vjp(ctypes.byref(b), ctypes.byref(p), ctypes.byref(a),
                                  ctypes.c_void_p(ws.ptr), ctypes.c_void_p(_stream_ptr())),
           "genga_rcrit_vjp")


def hc_vjp(state: State, cfg: Config, ws: Workspace, h: float, adj: AdjointState):
    b, p, a = state.bodies(), cfg.params(), adj.struct()
    _check(load().genga_hc_vjp(ctypes.byref(b), ctypes.byref(p), float(h), ctypes.byref(a),
                               ctypes.c_void_p(ws.ptr), ctypes.c_void_p(_stream_ptr())),
           "genga_hc_vjp")


def drift_vjp(state: State, cfg: Config, ws: Workspace, dt: float, adj: AdjointState):
    b, p, a = state.bodies(), cfg.params(), adj.struct()
    _check(load().genga_drift_vjp(ctypes.byref(b), ctypes.byref(p), float(dt), ctypes.byref(a),
                                  ctypes.c_void_p(ws.ptr), ctypes.c_void_p(_stream_ptr())),
           "genga_drift_vjp")
