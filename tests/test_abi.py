"""The C-ABI library loads on the CPU and exports every declared entry point.

No compute call is made here (there is no GPU in the CPU test run); argument
checks that return before any HIP call are exercised instead.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "genga.h")
LIB = os.path.join(ROOT, "paper_2201_10058_amd", "libgenga.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(genga_[a-z0-9_]+)\s*\(", text)))


def _lib():
    if not os.path.exists(LIB):
        from paper_2201_10058_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("genga_kick", "genga_drift", "genga_encounter_pairs", "genga_step",
                     "genga_rcrit", "genga_hc", "genga_workspace_bytes", "genga_read_status"):
        assert required in names


def test_every_declared_symbol_is_exported():
    lib = _lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_signatures_cover_header():
    from paper_2201_10058_amd import native
    assert set(declared_functions()) <= set(native.SIGNATURES)


def test_host_side_argument_errors():
    from paper_2201_10058_amd import native
    lib = native.load()
    assert lib.genga_version() >= 100
    assert lib.genga_strerror(native.E_OVERFLOW).decode().startswith("encounter list")
    p = native.Config(G=2.959e-4).params()
    assert lib.genga_workspace_bytes(0, ctypes.byref(p)) == 0
    assert lib.genga_workspace_bytes(65536, ctypes.byref(p)) > 65536 * 8 * 3
    # null bodies / workspace and invalid scalars fail before any device work
    assert lib.genga_kick(None, ctypes.byref(p), 0.0, None, None, None, None, None, None) == native.E_INVAL
    b = native.Bodies()
    b.n = 0
    assert lib.genga_rcrit(ctypes.byref(b), ctypes.byref(p), None, None) == native.E_INVAL
    b.n = 10
    assert lib.genga_step(ctypes.byref(b), ctypes.byref(p), None, None, None) == native.E_INVAL
    bad = native.Config(G=float("nan")).params()
    assert lib.genga_hc(ctypes.byref(b), ctypes.byref(bad), 1.0, None, None) == native.E_INVAL
    assert lib.genga_read_status(None, None) == native.E_INVAL
    assert lib.genga_energy(ctypes.byref(b), ctypes.byref(p), None, None, None) == native.E_INVAL
    # test-particle modes: checked on the host before any device work
    fake = ctypes.c_void_p(256)     # never dereferenced by the host-side checks
    for k in ("x", "y", "z", "vx", "vy", "vz", "m", "rc"):
        setattr(b, k, fake)
    b.n = 10
    bad_tp = native.Config(G=2.959e-4, tp_mode=3).params()
    assert lib.genga_kick(ctypes.byref(b), ctypes.byref(bad_tp), 0.0, None, None, None, None, fake,
                          None) == native.E_INVAL
    too_many = native.Config(G=2.959e-4, tp_mode=1, n_massive=11).params()
    assert lib.genga_kick(ctypes.byref(b), ctypes.byref(too_many), 0.0, None, None, None, None, fake,
                          None) == native.E_INVAL
    mixed_tp = native.Config(G=2.959e-4, tp_mode=2, n_massive=5, precision=native.MIXED).params()
    assert lib.genga_kick(ctypes.byref(b), ctypes.byref(mixed_tp), 0.0, None, None, None, None, fake,
                          None) == native.E_UNSUPPORTED
    tp = native.Config(G=2.959e-4, tp_mode=2, n_massive=5).params()
    assert lib.genga_kick_vjp(ctypes.byref(b), ctypes.byref(tp), 1.0, fake, fake, fake, None, fake,
                              None) in (native.E_INVAL, native.E_UNSUPPORTED)
    # the two kick forms exclude each other
    both = native.Config(G=2.959e-4, flags=native.FLAG_SYMMETRIC | native.FLAG_DIRECTED).params()
    assert lib.genga_kick(ctypes.byref(b), ctypes.byref(both), 0.0, None, None, None, None, fake,
                          None) == native.E_INVAL


@pytest.mark.parametrize("n", [1, 1000, 16383, 16384, 65536, 100003])
def test_symmetric_kick_workspace_on_host(n):
    # the workspace holds either form: the symmetric kick's row and column
    # sums (4 values each in mixed precision) and its per-tile counts
    from paper_2201_10058_amd import native
    lib = native.load()
    rg, tiles = 512, 0
    w = 512
    while w > 64:
        G = -(-n // rg)
        S0 = -(-n // w)
        d = rg // w
        tiles = G * S0 - d * (G * (G - 1) // 2)
        if tiles >= 4096:
            break
        w //= 2
    if w == 64:
        G = -(-n // rg)
        S0 = -(-n // w)
        d = rg // w
        tiles = G * S0 - d * (G * (G - 1) // 2)
    G = -(-n // rg)
    colsums = G * n - rg * (G * (G - 1) // 2)
    need = 8 * 4 * (tiles * rg + colsums) + 4 * tiles * rg
    for flags in (0, native.FLAG_SYMMETRIC, native.FLAG_DIRECTED):
        for prec in (native.FP64, native.MIXED):
            p = native.Config(G=2.959e-4, flags=flags, precision=prec).params()
            ws = lib.genga_workspace_bytes(n, ctypes.byref(p))
            sym = flags == native.FLAG_SYMMETRIC or (flags == 0 and n >= 8192)
            if sym:
                assert ws >= need, (n, flags, prec, ws, need)
            assert ws > 0


def test_level_params_on_host():
    from paper_2201_10058_amd import native
    lib = native.load()
    out = (ctypes.c_int64 * 4)()
    fake = ctypes.c_void_p(256)     # never dereferenced by the host-side checks
    b = native.Bodies()
    b.n = 10
    for k in ("x", "y", "z", "vx", "vy", "vz", "m", "rc"):
        setattr(b, k, fake)
    for kw in (dict(slevels=9, substeps=2, level_capacity=100),
               dict(slevels=2, substeps=0, level_capacity=100),
               dict(slevels=2, substeps=2, level_capacity=0),
               dict(slevels=3, substeps=2, level_capacity=(1 << 30) + 1),
               dict(slevels=-1)):
        p = native.Config(G=2.959e-4, **kw).params()
        assert lib.genga_step(ctypes.byref(b), ctypes.byref(p), None, fake, None) == native.E_INVAL
    for kw in (dict(direct=2, level_capacity=64), dict(direct=1, level_capacity=0),
               dict(direct=1, level_capacity=64, bs_eps=-1.0),
               dict(direct=1, level_capacity=64, bs_eps=float("nan"))):
        p = native.Config(G=2.959e-4, **kw).params()
        assert lib.genga_step(ctypes.byref(b), ctypes.byref(p), None, fake, None) == native.E_INVAL
    assert lib.genga_strerror(native.E_GROUP).decode().startswith("close-encounter group")
    bad_tol = native.Config(G=2.959e-4, coll_tol=1.5).params()
    assert lib.genga_step(ctypes.byref(b), ctypes.byref(bad_tol), None, fake, None) == native.E_INVAL
    cnt = (ctypes.c_int64 * 1)()
    plain = native.Config(G=2.959e-4, slevels=2, substeps=2, level_capacity=64).params()
    assert lib.genga_collisions(10, ctypes.byref(plain), fake, cnt, None, None, None, 0,
                                None) == native.E_INVAL
    neg_c = native.Config(G=2.959e-4, c_light=-1.0).params()
    assert lib.genga_step(ctypes.byref(b), ctypes.byref(neg_c), None, fake, None) == native.E_INVAL
    no_c = native.Config(G=2.959e-4).params()
    assert lib.genga_gr_kick(ctypes.byref(b), ctypes.byref(no_c), 1.0, fake, None) == native.E_INVAL
    no_direct = native.Config(G=2.959e-4, slevels=2, substeps=2, level_capacity=64).params()
    assert lib.genga_group_stats(10, ctypes.byref(no_direct), fake, out, None) == native.E_INVAL
    tp = native.Config(G=2.959e-4, tp_mode=1, n_massive=4, slevels=2, substeps=2,
                       level_capacity=64).params()
    assert lib.genga_step(ctypes.byref(b), ctypes.byref(tp), None, fake, None) == native.E_UNSUPPORTED
    one = native.Config(G=2.959e-4, slevels=1).params()
    assert lib.genga_level_counts(10, ctypes.byref(one), fake, out, None) == native.E_INVAL
    # the workspace grows with the levels and their capacity (two lists and
    # one adjacency of 2 int32 each per pair at L = 2); a larger L
    # contains the layout of a smaller one
    sizes = []
    for L in (1, 2, 3, 4):
        p = native.Config(G=2.959e-4, slevels=L, substeps=2, level_capacity=1 << 16).params()
        sizes.append(lib.genga_workspace_bytes(4096, ctypes.byref(p)))
    assert sizes == sorted(sizes) and len(set(sizes)) == 4
    big = native.Config(G=2.959e-4, slevels=2, substeps=2, level_capacity=1 << 20).params()
    assert lib.genga_workspace_bytes(4096, ctypes.byref(big)) >= sizes[1] + 24 * ((1 << 20) - (1 << 16))


@pytest.mark.parametrize("n", [1, 63, 64, 65, 2048, 65536, 4_000_000])
def test_workspace_grows_with_n(n):
    from paper_2201_10058_amd import native
    lib = native.load()
    p = native.Config(G=2.959e-4).params()
    assert lib.genga_workspace_bytes(n, ctypes.byref(p)) >= 3 * 8 * n


def test_batch_plan_shape_on_host():
    import numpy as np
    from paper_2201_10058_amd import native as N
    lib = N.load()
    sizes = np.array([16, 300, 4096, 1000, 257])
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    dummy = ctypes.c_void_p(8)   # never dereferenced by the host-side planner
    bt = N.BatchC(len(sizes), offsets.ctypes.data, dummy, dummy, dummy, dummy)
    for block, ipt, cols in ((256, 1, 1024), (64, 2, 512), (64, 1, 300)):
        p = N.Config(G=2.959e-4, block=block, ipt=ipt, tile_cols=cols).params()
        info = (ctypes.c_int64 * 5)()
        assert lib.genga_batch_info(ctypes.byref(bt), ctypes.byref(p), info) == N.OK
        c = -(-cols // 64) * 64
        r = block * ipt
        tiles = sum(-(-n // r) * -(-n // c) for n in sizes)
        assert info[0] == tiles and info[2] == block and info[3] == ipt and info[4] == c
        assert lib.genga_batch_workspace_bytes(ctypes.byref(bt), ctypes.byref(p)) > 24 * sizes.sum()
    bad = offsets.copy()
    bad[2] = bad[1]          # an empty system is rejected
    btb = N.BatchC(len(sizes), bad.ctypes.data, dummy, dummy, dummy, dummy)
    p = N.Config(G=2.959e-4).params()
    assert lib.genga_batch_workspace_bytes(ctypes.byref(btb), ctypes.byref(p)) == 0


def test_kick_static_host_checks():
    # the no-workspace kick refuses, before any device work, a missing status
    # word and a system whose kick needs more than the static scratch
    from paper_2201_10058_amd import native
    lib = native.load()
    assert native.E_SCRATCH == -9
    assert lib.genga_strerror(native.E_SCRATCH).decode().startswith("genga_kick_static")
    fake = ctypes.c_void_p(256)     # never dereferenced by the host-side checks
    b = native.Bodies()
    for k in ("x", "y", "z", "vx", "vy", "vz", "m", "rc"):
        setattr(b, k, fake)
    p = native.Config(G=2.959e-4).params()
    b.n = 1000
    assert lib.genga_kick_static(ctypes.byref(b), ctypes.byref(p), 0.0, None, None, None, None,
                                 None, None) == native.E_INVAL
    for n in (20000, 65536):
        b.n = n
        assert lib.genga_workspace_bytes(n, ctypes.byref(p)) > (96 << 20)
        assert lib.genga_kick_static(ctypes.byref(b), ctypes.byref(p), 0.0, None, None, None, None,
                                     fake, None) == native.E_SCRATCH
