"""Self-tuning of kick launch shapes (cf. the start-up self-tuning of kernel
parameters in GENGA II, Sect. 8): a thin binding of the native autotuner of
libgenga.so (genga_autotune_batched, genga_autotune).  Candidate shapes are
timed on the caller's own inputs with a zero step factor, so the state is not
modified; the choice is cached in a plain-text file keyed by device
architecture, precision and problem signature.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import native as N

CACHE_ENV = "GENGA_TUNE_CACHE"


def cache_path() -> str:
    """$GENGA_TUNE_CACHE, else ~/.cache/genga_mi355x/autotune.txt."""
    p = os.environ.get(CACHE_ENV)
    if not p:
        p = os.path.join(os.path.expanduser("~"), ".cache", "genga_mi355x", "autotune.txt")
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
    except OSError:
        pass
    return p


def tune_batched(state: N.State, batch: N.Batch, cfg: N.Config, use_cache: bool = True) -> dict:
    """Pick the batched kick's form and its shape: (block, ipt, tile_cols,
    grid) for the one-sided form, the column slices per 512-row group for the
    symmetric one; returns the choice (with the time of a step's two kicks,
    one without and one with the encounter list, in "ms")."""
    lib = N.load()
    bt = batch.struct()
    p = cfg.params()
    nbytes = lib.genga_autotune_batched_workspace_bytes(ctypes.byref(bt), ctypes.byref(p))
    if nbytes == 0:
        raise N.GengaError(N.E_INVAL, "genga_autotune_batched_workspace_bytes")
    ws = torch.zeros(int(nbytes), dtype=torch.uint8, device=state.t["x"].device)
    ms = ctypes.c_double(0.0)
    path = cache_path().encode() if use_cache else None
    b = state.bodies()
    N._check(lib.genga_autotune_batched(ctypes.byref(b), ctypes.byref(bt), ctypes.byref(p),
                                        ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(int(nbytes)),
                                        path, ctypes.byref(ms), ctypes.c_void_p(N._stream_ptr())),
             "genga_autotune_batched")
    form = "symmetric" if p.flags & N.FLAG_SYMMETRIC else "one-sided"
    return dict(form=form, block=p.block, ipt=p.ipt, tile_cols=p.tile_cols, grid=p.grid,
                slices=p.slices, flags=p.flags, ms=ms.value)


def tune_single(state: N.State, cfg: N.Config, use_cache: bool = True) -> dict:
    """Pick the kick form (one-sided or symmetric) and its (ipt, slices) for
    the single-system kick of this size; `flags` is cfg.flags with the chosen
    form flag."""
    lib = N.load()
    p = cfg.params()
    nbytes = lib.genga_autotune_workspace_bytes(state.n, ctypes.byref(p))
    if nbytes == 0:
        raise N.GengaError(N.E_INVAL, "genga_autotune_workspace_bytes")
    ws = torch.zeros(int(nbytes), dtype=torch.uint8, device=state.t["x"].device)
    ms = ctypes.c_double(0.0)
    path = cache_path().encode() if use_cache else None
    b = state.bodies()
    N._check(lib.genga_autotune(ctypes.byref(b), ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()),
                                ctypes.c_size_t(int(nbytes)), path, ctypes.byref(ms),
                                ctypes.c_void_p(N._stream_ptr())),
             "genga_autotune")
    form = "symmetric" if p.flags & N.FLAG_SYMMETRIC else "one-sided"
    return dict(form=form, ipt=p.ipt, slices=p.slices, flags=p.flags, ms=ms.value)


def tune_levels(state: N.State, cfg: N.Config, candidates, steps: int = 10) -> dict:
    """Pick (slevels, substeps) of the levelled step by running each candidate
    for `steps` steps on `state` (which advances: these are steps of the
    integration).  Returns the choice and every candidate's ms per step (-1
    where it could not run)."""
    lib = N.load()
    cands = [(int(L), int(s)) for L, s in candidates]
    most = 0
    for L, s in cands:
        q = N.Config(**{**cfg.__dict__, "slevels": L, "substeps": s}).params()
        most = max(most, int(lib.genga_workspace_bytes(state.n, ctypes.byref(q))))
    if most == 0:
        raise N.GengaError(N.E_INVAL, "genga_workspace_bytes")
    ws = torch.zeros(most, dtype=torch.uint8, device=state.t["x"].device)
    lev = (ctypes.c_int * len(cands))(*[c[0] for c in cands])
    sub = (ctypes.c_int * len(cands))(*[c[1] for c in cands])
    ms = (ctypes.c_double * len(cands))()
    p = cfg.params()
    b = state.bodies()
    N._check(lib.genga_tune_levels(ctypes.byref(b), ctypes.byref(p), lev, sub, len(cands), int(steps),
                                   ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(most), ms,
                                   ctypes.c_void_p(N._stream_ptr())),
             "genga_tune_levels")
    return dict(slevels=p.slevels, substeps=p.substeps,
                ms={f"{L}x{s}": ms[k] for k, (L, s) in enumerate(cands)})
