#!/usr/bin/env python3
"""Benchmark of the changeover-weighted kick path on one MI355X.

A step is one base step of the method (critical radii, half kick with the
encounter list, HC, Kepler drift, HC, half kick) on a synthetic planetesimal
disk of 65,536 bodies (0.5-4 AU, 5 Earth masses, dt = 6 days), inputs resident
in HBM.  The reported value is pair interactions per second over the timed
steps (2 N (N - 1) directed interactions per step).

The roofline entry prices the dominant kernel (the main kick kernel) at
20 FP64 flop per directed interaction against the FP64 vector peak; its
duration comes from HIP events recorded around that kernel inside the timed
steps, on the stream the kernel runs on.  The CPU baseline is the oracle's
plain FP64 kick timed on a bounded sample of rows of the same system.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

FLOP_PER_INTERACTION = 20
FP64_VECTOR_PEAK_TFLOPS = 78.6      # MI355X: 256 CU x 64 lanes x 2 flop x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak (packed FP32)
METRIC = "pair interactions/s (Ginter/s) + % vector roofline, FP64 vs mixed at N=65536"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the kick kernel settles within ~15 launches of a fresh process (2.0 ms
    # on the first, 1.6 ms from about the twelfth on): 10 untimed steps by default
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=65536, help="bodies (default: the 65,536-body disk)")
    ap.add_argument("--ipt", type=int, default=0)
    ap.add_argument("--slices", type=int, default=0)
    ap.add_argument("--kick-form", choices=("auto", "symmetric", "one-sided"), default="auto",
                    help="binary64 kick form (auto: symmetric from 8,192 bodies)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target duration of the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=30)
    ap.add_argument("--batch-kernels-only", action="store_true",
                    help="batched section without the autotuner and the per-system comparison "
                         "(for counter runs: the captured batched step alone)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-tp", action="store_true",
                    help="skip the test-particle mode timings")
    ap.add_argument("--no-levels", action="store_true",
                    help="skip the symplectic-level, direct-solver and GR timings")
    ap.add_argument("--no-pairs-run", action="store_true",
                    help="skip the 1000-step run with per-step encounter-list hashes")
    ap.add_argument("--no-sizes", action="store_true",
                    help="skip the binary64/mixed step timings at 16,384 and 32,768 bodies")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 2,048-body eager vs hipGraph step timing")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the mixed-precision error and energy-drift report")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device-to-device copy first (reference for HBM counters)")
    return ap.parse_args()


HERE = os.path.dirname(os.path.abspath(__file__))
KICK_SOURCES = ("kick.hip", "kick_sym.hip", "sym_common.h", "device_common.h", "genga_internal.h")
TRAFFIC_FILE = os.path.join(HERE, "profiles", "k_kick_sym_disk65536_traffic.txt")


def kick_source_hash() -> str:
    """SHA-256 over the sources of the FP64 kick kernel."""
    import hashlib
    h = hashlib.sha256()
    for f in KICK_SOURCES:
        with open(os.path.join(HERE, "paper_2201_10058_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per kick launch from the committed counter summary, or None if
    the kernel sources changed since the counters were taken."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha256") != kick_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


class HipEvents:
    """hipEvent_t handles from the HIP runtime already loaded by torch."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        ev = ctypes.c_void_p()
        rc = self.hip.hipEventCreate(ctypes.byref(ev))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed: {rc}")
        return ev.value

    def elapsed_ms(self, a, b) -> float:
        ms = ctypes.c_float()
        rc = self.hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(a), ctypes.c_void_p(b))
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
        return float(ms.value)

    def destroy(self, e):
        self.hip.hipEventDestroy(ctypes.c_void_p(e))


def cpu_baseline(d, rc, G, target_s):
    """Oracle plain FP64 kick on a bounded sample of the same system.

    The sample grows (first rows, then repeated full kicks) until one timed
    pass takes about half of target_s.
    """
    import oracle
    n = d["n"]
    rows, reps = 256, 1
    while True:
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.kick_acc(d["x"], d["y"], d["z"], d["m"], rc, G, rows=(0, rows), precise=False)
        t_used = time.perf_counter() - t0
        if t_used >= 0.5 * target_s:
            break
        grow = max(2.0, min(8.0, 0.6 * target_s / max(t_used, 1e-3)))
        if rows < n:
            rows = min(n, int(rows * grow))
        elif reps < 64:
            reps = min(64, int(reps * grow))
        else:
            break
    inter = reps * rows * (n - 1)
    what = (f"rows 0..{rows - 1}" if rows < n else f"{reps} full kick(s)")
    cores = oracle.num_threads()
    # the same loop on one core, on a sample of about a tenth of the time
    oracle.set_num_threads(1)
    rows1 = max(64, int(rows * reps * 0.1 / max(cores, 1)))
    rows1 = min(rows1, n)
    t0 = time.perf_counter()
    oracle.kick_acc(d["x"], d["y"], d["z"], d["m"], rc, G, rows=(0, rows1), precise=False)
    t1 = time.perf_counter() - t0
    oracle.set_num_threads(cores)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": inter / t_used / 1e9, "unit": "Ginter/s", "cores": cores,
            "kind": "oracle",
            "sample": f"plain FP64 kick (oracle), {what} of the {n}-body disk: "
                      f"{inter:.3e} interactions in {t_used:.1f} s",
            "one_core_value": rows1 * (n - 1) / t1 / 1e9,
            "one_core_sample": f"rows 0..{rows1 - 1}: {rows1 * (n - 1):.3e} interactions in {t1:.1f} s",
            "cpu_model": model}


def mixed_accuracy(N, W, torch, np, checkpoints=(0, 10, 100, 1000)):
    """Mixed-precision kick against the FP64 kick on the three mixed-precision
    disks (16,384 / 32,768 / 65,536 bodies) at t = 0, and on the 16,384-body
    disk also after 10, 100 and 1000 mixed-precision steps (both kicks on the
    state the mixed run reached): relative error per acceleration."""
    def compare(st, cfg, ws):
        N.rcrit(st, cfg, ws)
        a64 = N.kick(st, cfg, ws, 0.0, acc=True)
        a32 = N.kick(st, N.Config(**{**cfg.__dict__, "precision": N.MIXED}), ws, 0.0, acc=True)
        torch.cuda.synchronize()
        if N.read_status(ws) != N.OK:
            raise SystemExit("mixed accuracy status")
        rel = ((a32 - a64).norm(dim=0) / a64.norm(dim=0)).cpu().numpy()
        return {"max": float(rel.max()), "p99": float(np.quantile(rel, 0.99)),
                "p50": float(np.quantile(rel, 0.5))}

    out = {}
    for n_, spec in sorted(W.DISK_MIXED.items()):
        d = W.make_disk(spec)
        st = N.State.from_numpy(d)
        cfg = N.Config(G=d["G"], m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"])
        ws = N.Workspace(n_, cfg)
        out[f"n{n_}_t0"] = compare(st, cfg, ws)
        if n_ == 16384:
            mcfg = N.Config(**{**cfg.__dict__, "precision": N.MIXED, "flags": N.FLAG_NOSYNC})
            done = 0
            for t in checkpoints[1:]:
                for _ in range(t - done):
                    N.step(st, mcfg, ws)
                done = t
                out[f"n{n_}_t{t}"] = compare(st, cfg, ws)
    return out


def energy_drift(N, W, torch, np, steps=10_000, every=1000):
    """Relative drift (E(t) - E(0)) / |E(0)| of the FP64 and mixed steps on
    the 16,384-body disk over `steps` steps, energies in binary64, for E and
    for E_K (the changeover-potential energy, with the critical radii of the
    last step)."""
    d = W.make_disk(W.DISK_MIXED[16384])
    drift, drift_k = {}, {}
    for name, prec in (("fp64", N.FP64), ("mixed", N.MIXED)):
        st = N.State.from_numpy(d)
        cfg = N.Config(G=d["G"], m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"],
                       precision=prec, flags=N.FLAG_NOSYNC)
        ws = N.Workspace(st.n, cfg)
        pl = N.PairList(1 << 18)
        N.rcrit(st, cfg, ws)
        Es = [N.energy_k(st, cfg, ws, pl).clone()]
        for k in range(steps):
            N.step(st, cfg, ws)
            if (k + 1) % every == 0:
                Es.append(N.energy_k(st, cfg, ws, pl).clone())
        if N.read_status(ws) != N.OK:
            raise SystemExit("energy drift status")
        E = torch.stack(Es).cpu().numpy()
        drift[name] = (E[:, 0] - E[0, 0]) / abs(E[0, 0])
        drift_k[name] = (E[:, 5] - E[0, 5]) / abs(E[0, 5])
    return {"steps": steps, "n": int(d["n"]),
            "fp64_max_abs_drift": float(np.max(np.abs(drift["fp64"]))),
            "mixed_max_abs_drift": float(np.max(np.abs(drift["mixed"]))),
            "max_abs_mixed_minus_fp64": float(np.max(np.abs(drift["mixed"] - drift["fp64"]))),
            "fp64_max_abs_drift_e_k": float(np.max(np.abs(drift_k["fp64"]))),
            "mixed_max_abs_drift_e_k": float(np.max(np.abs(drift_k["mixed"])))}


def bench_small(N, W, torch, np, steps=100):
    """The 2,048-body disk (a launch-bound size): base steps issued one by
    one against the same step captured once in a hipGraph and replayed."""
    d = W.make_disk(W.DISK_2048)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=d["G"], m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"],
                   flags=N.FLAG_NOSYNC)
    ws = N.Workspace(st.n, cfg)
    pairs = N.PairList(1 << 16)

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    N.rcrit(st, cfg, ws)
    e_start = N.energy_k(st, cfg, ws, N.PairList(1 << 16)).cpu().numpy()
    eager = timed(lambda: N.step(st, cfg, ws, pairs))
    e_end = N.energy_k(st, cfg, ws, N.PairList(1 << 16)).cpu().numpy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        N.step(st, cfg, ws, pairs)
    graph = timed(g.replay)
    # several steps captured in one graph (one launch of the whole sequence)
    per_graph = 10
    g10 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g10):
        for _ in range(per_graph):
            N.step(st, cfg, ws, pairs)
    for _ in range(2):
        g10.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // per_graph):
        g10.replay()
    torch.cuda.synchronize()
    graph10 = (time.perf_counter() - t0) / (per_graph * (steps // per_graph))
    if N.read_status(ws) != N.OK:
        raise SystemExit("small-system status")
    inter = 2.0 * st.n * (st.n - 1)
    return {"workload": W.DISK_2048.name, "n": st.n, "steps": steps,
            "eager_step_us": round(eager * 1e6, 2), "graph_step_us": round(graph * 1e6, 2),
            "graph_10_steps_per_replay_step_us": round(graph10 * 1e6, 2),
            "eager_ginter_s": round(inter / eager / 1e9, 3),
            "graph_ginter_s": round(inter / graph / 1e9, 3),
            "graph_10_steps_ginter_s": round(inter / graph10 / 1e9, 3),
            "energy_rel_change_eager_steps": float((e_end[0] - e_start[0]) / abs(e_start[0])),
            "energy_k_rel_change_eager_steps": float((e_end[5] - e_start[5]) / abs(e_start[5]))}


def bench_tp(N, W, torch, np, steps=20):
    """Test-particle modes on the 65,536-body zero-inclination disk with 16
    massive bodies (the setup of the paper's test-particle timings): step time
    and interactions per second, counting the force terms each mode has."""
    d = W.make_tp_disk(65536, 16)
    n, nm = d["n"], d["n_massive"]
    out = {"workload": d["name"], "n": n, "n_massive": nm}
    for mode in (1, 2):
        st = N.State.from_numpy(d)
        cfg = N.Config(G=d["G"], m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"],
                       flags=N.FLAG_NOSYNC, tp_mode=mode, n_massive=nm)
        ws = N.Workspace(n, cfg)
        pairs = N.PairList(1 << 16)
        for _ in range(3):
            N.step(st, cfg, ws, pairs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            N.step(st, cfg, ws, pairs)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / steps
        if N.read_status(ws) != N.OK:
            raise SystemExit("test-particle status")
        terms = nm * (n - 1) + (n - nm) * nm if mode == 2 else nm * (nm - 1) + (n - nm) * nm
        out[f"tp{mode}"] = {"step_us": round(dt_s * 1e6, 2),
                            "ginter_s": round(2.0 * terms / dt_s / 1e9, 3),
                            "encounter_pairs_last_step": int(pairs.count.item())}
    return out


LEVEL_CANDIDATES = ((1, 1), (2, 2), (2, 4), (3, 2), (2, 10), (3, 4))
# (1, 1) with the direct solver is the original hybrid step (one symplectic
# level, Bulirsch-Stoer for every level-0 group): the baseline of Sect. 6.2
DIRECT_CANDIDATES = ((1, 1), (3, 4), (2, 10), (4, 4))


def bench_levels(N, W, torch, np, steps=10):
    """Symplectic levels on the 65,536-body disk: for each (levels, sub-steps)
    choice, with and without the direct solver for the deepest level's groups,
    from the same initial state, the time per step, the list sizes of its last
    step and the relative change of the total energy over its steps; then the
    native tuner's choice among the level choices (run on a fresh copy)."""
    from paper_2201_10058_amd import autotune as AT
    d = W.make_disk(W.DISK_65536)
    out = {"workload": d["name"], "steps": steps, "configs": {}}
    base = dict(G=d["G"], m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"],
                flags=N.FLAG_NOSYNC, level_capacity=1 << 20)
    runs = [(L, s, 0) for L, s in LEVEL_CANDIDATES] + [(L, s, 1) for L, s in DIRECT_CANDIDATES]
    for L, s, direct in runs:
        st = N.State.from_numpy(d)
        cfg = N.Config(**base, slevels=L, substeps=s, direct=direct)
        ws = N.Workspace(st.n, cfg)
        pairs = N.PairList(1 << 20)
        e0 = float(N.energy(st, cfg, ws)[0].item())
        N.step(st, cfg, ws, pairs)
        torch.cuda.synchronize()
        # the one-level direct step integrates a group of ~25,000 bodies by
        # Bulirsch-Stoer (about a second per step): fewer timed steps
        k_steps = 3 if (direct and L == 1) else steps
        t0 = time.perf_counter()
        for _ in range(k_steps):
            N.step(st, cfg, ws, pairs)
            if direct and L == 1:
                torch.cuda.synchronize()
                print(f"levels {L}x{s}+direct: step done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / k_steps
        code = N.read_status(ws)
        if code != N.OK and not (direct and code == N.E_GROUP):
            raise SystemExit(f"levels {L}x{s}: status {code}")
        e1 = float(N.energy(st, cfg, ws)[0].item())
        counts = (N.level_counts(st.n, cfg, ws).tolist() if L > 1 or direct
                  else [int(pairs.count.item())])
        rec = {"step_ms": round(dt_s * 1e3, 4), "list_sizes_last_step": counts,
               "energy_rel_change": (e1 - e0) / abs(e0), "steps": k_steps + 1}
        if direct:
            g, gmax = N.group_stats(st.n, cfg, ws)
            rec.update({"groups_last_step": g, "largest_group": gmax,
                        "status": "ok" if code == N.OK else "group over the solver's limit"})
        out["configs"][f"{L}x{s}" + ("+direct" if direct else "")] = rec
    st = N.State.from_numpy(d)
    out["tuner"] = AT.tune_levels(st, N.Config(**base), LEVEL_CANDIDATES, steps=3)
    out["direct_by_n"] = levels_by_n(N, W, torch)
    return out


LEVELS_BY_N = (2048, 4096, 8192, 16384, 32768)


def levels_by_n(N, W, torch, steps=3):
    """Sect. 6.2's comparison across N: disks of the benchmark's kind (0.5-4 AU,
    5 M_earth, seeds 40 + k) stepped by the original hybrid integrator (one
    level, every level-0 group by Bulirsch-Stoer) and with levels (3 x 4 and
    2 x 10, the direct solver on the deepest level): ms per step (after one
    untimed step) and the largest group of the last step."""
    out = {}
    for k, n_ in enumerate(LEVELS_BY_N):
        d = W.make_disk(W.DiskSpec(f"disk_n{n_}_a0.5-4_5Mearth_s{40 + k}", n_, 0.5, 4.0, 5.0,
                                   seed=40 + k))
        base = dict(G=d["G"], m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"],
                    flags=N.FLAG_NOSYNC, level_capacity=1 << 20, direct=1)
        rec = {}
        for L, s in ((1, 1), (3, 4), (2, 10)):
            st = N.State.from_numpy(d)
            cfg = N.Config(**base, slevels=L, substeps=s)
            ws = N.Workspace(st.n, cfg)
            N.step(st, cfg, ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                N.step(st, cfg, ws)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            if N.read_status(ws) != N.OK:
                raise SystemExit(f"levels by N {n_} {L}x{s}: status")
            g, gmax = N.group_stats(st.n, cfg, ws)
            rec[f"{L}x{s}+direct"] = {"step_ms": round(ms, 4), "largest_group": gmax}
        rec["levels_speedup_3x4"] = round(rec["1x1+direct"]["step_ms"] / rec["3x4+direct"]["step_ms"], 3)
        out[str(n_)] = rec
        print(f"levels by N, {n_} bodies: {rec}", file=sys.stderr, flush=True)
    return out


RING_SIZES = (2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768, 65536)


def bench_bs_ring(N, W, torch, np, steps=5):
    """The close-encounter performance test of Sect. 6.1 (Fig. BSTime): n
    bodies on a ring, each meeting its 8 nearest neighbours, so that all n
    form one close-encounter group; one-level steps with the direct solver
    (8 lanes per group up to 8 bodies, one workgroup up to 512, all
    workgroups beyond) against the same steps without it, per n."""
    out = {"neighbours": 8, "steps": steps, "sizes": {}}
    for n in RING_SIZES:
        d = W.make_bs_ring(n)
        rec = {}
        for direct in (1, 0):
            st = N.State.from_numpy(d)
            cfg = N.Config(G=d["G"], m_star=1.0, dt=d["dt"], n1=d["n1"], n2=0.0, slevels=1,
                           substeps=1, direct=direct, flags=N.FLAG_NOSYNC,
                           level_capacity=max(1 << 12, 16 * n))
            ws = N.Workspace(st.n, cfg)
            N.step(st, cfg, ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                N.step(st, cfg, ws)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            if N.read_status(ws) != N.OK:
                raise SystemExit(f"ring {n}: status")
            if direct:
                g, gmax = N.group_stats(st.n, cfg, ws)
                if (g, gmax) != (1, n):
                    raise SystemExit(f"ring {n}: groups {(g, gmax)}")
                rec["direct_step_ms"] = round(ms, 4)
            else:
                rec["plain_step_ms"] = round(ms, 4)
        rec["close_encounter_ms"] = round(rec["direct_step_ms"] - rec["plain_step_ms"], 4)
        rec["solver"] = "lanes" if n <= 8 else ("workgroup" if n <= 512 else "grid")
        out["sizes"][str(n)] = rec
        print(f"ring {n}: {rec}", file=sys.stderr, flush=True)
    return out


def bench_gr(N, W, torch, np, steps=10):
    """Post-Newtonian term on the 65,536-body disk: step time with and without
    it (the same initial state), and the GR update alone."""
    d = W.make_disk(W.DISK_65536)
    out = {"workload": d["name"], "c_light_au_per_day": 173.1446326846693}
    for label, c in (("without", 0.0), ("with", 173.1446326846693)):
        st = N.State.from_numpy(d)
        cfg = N.Config(G=d["G"], m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"],
                       flags=N.FLAG_NOSYNC, c_light=c)
        ws = N.Workspace(st.n, cfg)
        for _ in range(3):
            N.step(st, cfg, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            N.step(st, cfg, ws)
        torch.cuda.synchronize()
        out[f"step_ms_{label}"] = round((time.perf_counter() - t0) / steps * 1e3, 4)
        if c > 0:
            t0 = time.perf_counter()
            for _ in range(steps):
                N.gr_kick(st, cfg, ws, 0.5 * d["dt"])
            torch.cuda.synchronize()
            out["gr_update_us"] = round((time.perf_counter() - t0) / steps * 1e6, 2)
        if N.read_status(ws) != N.OK:
            raise SystemExit("gr status")
    return out


def bench_sizes(N, W, torch, np, steps=30):
    """Binary64 and mixed steps of the 16,384- and 32,768-body disks (the
    65,536-body disk is the main run), each from the same initial state:
    time per step; the two precisions alternate twice and the faster of each
    pair of runs is kept."""
    out = {}
    for n_ in (16384, 32768):
        d = W.make_disk(W.DISK_MIXED[n_])
        best = {}
        for _ in range(2):
            for name, prec in (("fp64", N.FP64), ("mixed", N.MIXED)):
                st = N.State.from_numpy(d)
                cfg = N.Config(G=d["G"], m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"],
                               precision=prec, flags=N.FLAG_NOSYNC)
                ws = N.Workspace(n_, cfg)
                pl = N.PairList(1 << 20)
                for _ in range(3):
                    N.step(st, cfg, ws, pl)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    N.step(st, cfg, ws, pl)
                torch.cuda.synchronize()
                dt_s = (time.perf_counter() - t0) / steps
                if N.read_status(ws) != N.OK:
                    raise SystemExit(f"sizes {n_} status")
                best[name] = min(best.get(name, 1e9), dt_s)
        inter = 2.0 * n_ * (n_ - 1)
        out[f"n{n_}"] = {"workload": d["name"],
                         "fp64_step_ms": round(best["fp64"] * 1e3, 4),
                         "mixed_step_ms": round(best["mixed"] * 1e3, 4),
                         "fp64_ginter_s": round(inter / best["fp64"] / 1e9, 3),
                         "mixed_ginter_s": round(inter / best["mixed"] / 1e9, 3),
                         "mixed_speedup": round(best["fp64"] / best["mixed"], 4)}
    return out


def bench_n2_zero(N, W, torch, np, steps=10):
    """The 65,536-body step with the critical radius of the Hill term alone
    (n2 = 0 in eq. rcrit) beside the main run's n2 = 0.4: time per step and
    encounter pairs of the last step."""
    d = W.make_disk(W.DISK_65536)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=d["G"], m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=0.0,
                   flags=N.FLAG_NOSYNC)
    ws = N.Workspace(st.n, cfg)
    pl = N.PairList(1 << 20)
    for _ in range(3):
        N.step(st, cfg, ws, pl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        N.step(st, cfg, ws, pl)
    torch.cuda.synchronize()
    dt_s = (time.perf_counter() - t0) / steps
    if N.read_status(ws) != N.OK:
        raise SystemExit("n2 = 0 status")
    n = st.n
    return {"n2": 0.0, "step_ms": round(dt_s * 1e3, 4),
            "ginter_s": round(2.0 * n * (n - 1) / dt_s / 1e9, 3),
            "encounter_pairs_last_step": int(pl.count.item()),
            "encounter_pairs_sha256_last_step": pair_list_sha256(pl)}


def pairs_run(N, W, torch, np, steps=1000):
    """The 65,536-body disk for 1000 base steps with the encounter list of
    every step (first half kick, positions the step starts from): per step
    its pair count and the SHA-256 of the canonical list (int32 i then int32
    j, little endian).  The per-step digests go to stderr; the JSON keeps the
    counts' range and the SHA-256 over the 1000 digests in step order."""
    import hashlib
    d = W.make_disk(W.DISK_65536)
    st = N.State.from_numpy(d)
    cfg = N.Config(G=d["G"], m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"],
                   flags=N.FLAG_NOSYNC)
    ws = N.Workspace(st.n, cfg)
    pl = N.PairList(1 << 20)
    chain = hashlib.sha256()
    counts = []
    t0 = time.perf_counter()
    for k in range(steps):
        N.step(st, cfg, ws, pl)
        c = int(pl.count.item())
        if c > pl.capacity:
            raise SystemExit(f"pairs run: {c} pairs beyond the list capacity at step {k}")
        dig = pair_list_sha256(pl)
        counts.append(c)
        chain.update(dig.encode())
        print(f"pairs step {k}: {c} {dig}", file=sys.stderr, flush=(k % 100 == 99))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if N.read_status(ws) != N.OK:
        raise SystemExit("pairs run status")
    return {"workload": d["name"], "steps": steps, "count_min": min(counts),
            "count_max": max(counts), "count_mean": round(float(np.mean(counts)), 1),
            "count_first": counts[0], "count_last": counts[-1],
            "sha256_of_step_digests": chain.hexdigest(), "wall_s": round(wall, 2)}


def oracle_run_cfg0(N, W, torch, np, steps=100):
    """The oracle's own 100-step run of the 2,048-body disk on the host (its
    plain binary64 step, all host cores), beside the GPU's step."""
    import oracle
    d = W.make_disk(W.DISK_2048)
    ref = oracle.state_copy(d)
    t0 = time.perf_counter()
    for _ in range(steps):
        oracle.step(ref, d["G"], d["m_star"], d["dt"], d["n1"], d["n2"])
    host_s = time.perf_counter() - t0
    n = d["n"]
    return {"workload": d["name"], "steps": steps, "cores": oracle.num_threads(),
            "host_s": round(host_s, 3), "host_step_ms": round(host_s / steps * 1e3, 3),
            "host_ginter_s": round(2.0 * n * (n - 1) * steps / host_s / 1e9, 3)}


def pair_list_sha256(pairs) -> str:
    """SHA-256 of the canonical list (int32 i then int32 j, little endian)."""
    import hashlib
    pi, pj, _ = pairs.result()
    h = hashlib.sha256()
    h.update(pi.astype("<i4").tobytes())
    h.update(pj.astype("<i4").tobytes())
    return h.hexdigest()


def bench_batched(args, N, W, torch, np):
    """The 512-system ensemble: one persistent kick per half step, the whole
    step captured in a hipGraph, against 512 single-system steps."""
    from paper_2201_10058_amd import autotune
    d = W.make_batch()
    G = d["G"]
    bt = N.Batch(d["offsets"], d["m_star"], d["dt"], d["n1"], d["n2"])
    st = N.State.from_numpy(d)
    base = N.Config(G=G, flags=N.FLAG_NOSYNC)
    # tile shape by the autotuner (rc from one plain step first)
    ws0 = N.BatchWorkspace(bt, base)
    N.step_batched(st, ws0, base)
    torch.cuda.synchronize()
    if args.batch_kernels_only:
        choice = {"block": 0, "ipt": 0, "tile_cols": 0, "grid": 0, "flags": base.flags}
        tune_ms, form = float("nan"), "default"
    else:
        choice = autotune.tune_batched(st, bt, base)
        tune_ms = choice.pop("ms")
        form = choice.pop("form")
    cfg = N.Config(**{**base.__dict__, **choice})
    ws = N.BatchWorkspace(bt, cfg)
    pairs = N.PairList(1 << 22)
    sizes = np.diff(d["offsets"])
    inter = float(np.sum(sizes * (sizes - 1))) * 2.0       # per step (two kicks)
    K = args.batch_steps

    def timed(fn, k):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    eager_s = timed(lambda: N.step_batched(st, ws, cfg, pairs), K)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        N.step_batched(st, ws, cfg, pairs)
    graph_s = timed(g.replay, K)
    code = N.read_status(ws)
    if code != N.OK:
        raise SystemExit(f"batched status: {code}")
    if args.batch_kernels_only:
        return {"systems": int(d["S"]), "graph_step_ms": round(graph_s * 1e3, 4),
                "eager_step_ms": round(eager_s * 1e3, 4), "form": "default"}
    # the other kick form on the same ensemble (captured step)
    forms = N.FLAG_DIRECTED | N.FLAG_SYMMETRIC
    other = N.FLAG_SYMMETRIC if form == "one-sided" else N.FLAG_DIRECTED
    cfg_o = N.Config(**{**cfg.__dict__, "flags": (cfg.flags & ~forms) | other})
    ws_o = N.BatchWorkspace(bt, cfg_o)
    N.step_batched(st, ws_o, cfg_o, pairs)
    torch.cuda.synchronize()
    g_o = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_o):
        N.step_batched(st, ws_o, cfg_o, pairs)
    other_s = timed(g_o.replay, K)
    if N.read_status(ws_o) != N.OK:
        raise SystemExit("batched status (other form)")
    # per-system launches (each system its own genga_step calls)
    views, wss = [], []
    for s_ in range(d["S"]):
        lo, hi = int(d["offsets"][s_]), int(d["offsets"][s_ + 1])
        views.append(N.system_view(st, lo, hi))
        wss.append(N.Workspace(hi - lo, base))
    cfgs = [N.Config(G=G, m_star=float(d["m_star"][k]), dt=float(d["dt"][k]), n1=float(d["n1"][k]),
                     n2=float(d["n2"][k]), flags=N.FLAG_NOSYNC) for k in range(d["S"])]
    pls = [N.PairList(max(16, 64 * int(sizes[k]))) for k in range(d["S"])]

    def per_system():
        for k in range(d["S"]):
            N.step(views[k], cfgs[k], wss[k], pls[k])

    per_sys_s = timed(per_system, max(2, K // 3))
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        per_system()
    per_sys_graph_s = timed(g2.replay, K)
    for w_ in wss:
        if N.read_status(w_) != N.OK:
            raise SystemExit("per-system status")
    return {"systems": int(d["S"]), "bodies": int(d["offsets"][-1]),
            "interactions_per_step": inter,
            "value": round(inter / graph_s / 1e9, 3), "unit": "Ginter/s",
            "graph_step_ms": round(graph_s * 1e3, 4), "eager_step_ms": round(eager_s * 1e3, 4),
            "per_system_eager_step_ms": round(per_sys_s * 1e3, 4),
            "per_system_graph_step_ms": round(per_sys_graph_s * 1e3, 4),
            "speedup_vs_per_system_graph": round(per_sys_graph_s / graph_s, 3),
            "speedup_vs_per_system_eager": round(per_sys_s / graph_s, 3),
            "tile_shape": {**choice, "form": form,
                           **({"tiles": ws.info["tiles"], "grid": ws.info["grid"]}
                              if form == "one-sided" else {}),
                           "autotuned_two_kicks_ms": round(tune_ms, 4)},
            "other_form": {"form": "symmetric" if form == "one-sided" else "one-sided",
                           "graph_step_ms": round(other_s * 1e3, 4)},
            "tuner_by_size": tune_by_size(N, W, torch, np, d)}


SIZE_BUCKETS = ((16, 64), (64, 256), (256, 1024), (1024, 4096))


def tune_by_size(N, W, torch, np, d):
    """The batched autotuner's choice for the ensemble's systems of each size
    bucket (N_s in [lo, hi)), each bucket tuned as an ensemble of its own
    (fresh, not from the cache), with the time of its tuned kick."""
    from paper_2201_10058_amd import autotune
    sizes = np.diff(d["offsets"])
    out = {}
    for lo, hi in SIZE_BUCKETS:
        idx = [k for k in range(d["S"]) if lo <= sizes[k] < hi]
        if not idx:
            continue
        parts = {f: np.concatenate([d[f][d["offsets"][k]:d["offsets"][k + 1]] for k in idx])
                 for f in ("x", "y", "z", "vx", "vy", "vz", "m")}
        offs = np.zeros(len(idx) + 1, dtype=np.int64)
        offs[1:] = np.cumsum(sizes[idx])
        bt = N.Batch(offs, d["m_star"][idx], d["dt"][idx], d["n1"][idx], d["n2"][idx])
        st = N.State.from_numpy(parts)
        cfg = N.Config(G=d["G"], flags=N.FLAG_NOSYNC)
        N.step_batched(st, N.BatchWorkspace(bt, cfg), cfg)   # radii for the kicks
        torch.cuda.synchronize()
        ch = autotune.tune_batched(st, bt, cfg, use_cache=False)
        inter = float(np.sum(sizes[idx] * (sizes[idx] - 1)))
        rec = {"systems": len(idx), "bodies": int(offs[-1]), "form": ch["form"],
               "two_kicks_ms": round(ch["ms"], 4),
               "kick_ginter_s": round(2.0 * inter / ch["ms"] / 1e6, 1)}
        if ch["form"] == "symmetric":
            rec["slice_columns"] = 512 // max(1, ch["slices"])
        else:
            rec.update(block=ch["block"], ipt=ch["ipt"], tile_cols=ch["tile_cols"], grid=ch["grid"])
        out[f"{lo}-{hi}"] = rec
        print(f"tuner, systems of {lo}-{hi} bodies: {rec}", file=sys.stderr, flush=True)
    return out


def bench_adjoint(N, W, torch, np, d65536_state, cfg65536, kick_ms_fp64=None):
    """Adjoint: the kick VJP kernel on the 65,536-body disk, and the gradient of
    a 200-step trajectory of the 4,096-body disk (checkpoints every 20 steps)."""
    from paper_2201_10058_amd import adjoint as A
    st, n = d65536_state, d65536_state.n
    ws = N.Workspace(n, cfg65536)
    adj = N.AdjointState(n)
    ab = [torch.randn(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    def vjp_time(cfg):
        wsv = N.Workspace(n, cfg)
        N.kick_vjp(st, cfg, wsv, 1.0, ab, adj)
        torch.cuda.synchronize()
        reps = 5
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            N.kick_vjp(st, cfg, wsv, 1.0, ab, adj)
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    vjp_ms = vjp_time(cfg65536)     # the default: the symmetric form at this size
    vjp_one_ms = vjp_time(N.Config(**{**cfg65536.__dict__, "flags": N.FLAG_DIRECTED}))
    kick_ms = None
    if kick_ms_fp64 is not None:
        kick_ms = kick_ms_fp64
    d = W.make_disk(W.DISK_ADJOINT)
    X = torch.tensor(np.stack([d["x"], d["y"], d["z"]]), device="cuda", requires_grad=True)
    V = torch.tensor(np.stack([d["vx"], d["vy"], d["vz"]]), device="cuda", requires_grad=True)
    m = torch.tensor(d["m"], device="cuda", requires_grad=True)
    cfg = N.Config(G=d["G"])
    # warm-up: one short differentiated trajectory
    XT, _ = A.simulate(X, V, m, 20, cfg, checkpoint_every=20)
    torch.autograd.grad((XT ** 2).sum(), (X, V, m))
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    XT, VT = A.simulate(X, V, m, 200, cfg, checkpoint_every=20)
    L = (XT ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    torch.autograd.grad(L, (X, V, m))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    peak = torch.cuda.max_memory_allocated() - base
    return {"kick_vjp_ms_n65536": round(vjp_ms, 4),
            "kick_vjp_form": "symmetric",
            "kick_vjp_ginter_s": round(n * (n - 1) / vjp_ms / 1e6, 3),
            "kick_vjp_one_sided_ms_n65536": round(vjp_one_ms, 4),
            "kick_vjp_over_kick_kernel": round(vjp_ms / kick_ms, 3) if kick_ms else None,
            "trajectory_n4096_200_steps_forward_s": round(t1 - t0, 4),
            "trajectory_n4096_200_steps_backward_s": round(t2 - t1, 4),
            "backward_over_forward": round((t2 - t1) / (t1 - t0), 3),
            "checkpoint_every": 20,
            "peak_device_bytes_forward_backward": int(peak)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2201_10058_amd import native as N
    from paper_2201_10058_amd import workload as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    N.load()

    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    spec = W.DISK_65536 if args.n == 65536 else W.DiskSpec(
        f"disk_n{args.n}_a0.5-4_5Mearth", args.n, 0.5, 4.0, 5.0, seed=1)
    d = W.make_disk(spec)
    n = d["n"]
    G = d["G"]
    hip = HipEvents()

    form_flags = {"auto": 0, "symmetric": N.FLAG_SYMMETRIC, "one-sided": N.FLAG_DIRECTED}
    sym = args.kick_form == "symmetric" or (args.kick_form == "auto" and n >= 8192)

    def run(precision, form=None):
        """Warm up, then time `steps` base steps; returns the measurements."""
        st = N.State.from_numpy(d)
        flags = N.FLAG_NOSYNC | form_flags[form or args.kick_form]
        cfg = N.Config(G=G, m_star=d["m_star"], dt=d["dt"], n1=d["n1"], n2=d["n2"],
                       precision=precision, flags=flags, ipt=args.ipt, slices=args.slices)
        ws = N.Workspace(n, cfg)
        pairs = N.PairList(max(1 << 20, 8 * n))
        for _ in range(args.warmup):
            N.step(st, cfg, ws, pairs)
        torch.cuda.synchronize()
        code = N.read_status(ws)
        if code != N.OK:
            raise SystemExit(f"warm-up status: {code}")
        evs = [[hip.create() for _ in range(4)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            cfg.events = tuple(evs[k])
            N.step(st, cfg, ws, pairs)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        cfg.events = (None, None, None, None)
        code = N.read_status(ws)
        if code != N.OK:
            raise SystemExit(f"timed-run status: {code}")
        kick_ms = []
        for e in evs:
            kick_ms.append(hip.elapsed_ms(e[0], e[1]))
            kick_ms.append(hip.elapsed_ms(e[2], e[3]))
            for h in e:
                hip.destroy(h)
        return dict(elapsed=elapsed, kick_s=float(np.mean(kick_ms)) / 1e3,
                    kick_ms_median=float(np.median(kick_ms)), kick_ms_min=float(np.min(kick_ms)),
                    pairs=int(pairs.count.item()), pairs_sha256=pair_list_sha256(pairs),
                    rc=st.t["rc"])

    r64 = run(N.FP64)
    print(f"fp64 step done: {r64['elapsed'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr,
          flush=True)
    r1s = None
    if sym:
        # the one-sided binary64 kick on the same workload, for comparison
        r1s = run(N.FP64, "one-sided")
        print(f"one-sided fp64 step done: {r1s['elapsed'] / args.steps * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)
    r32 = None
    if not args.no_mixed:
        r32 = run(N.MIXED)
        print(f"mixed step done: {r32['elapsed'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr,
              flush=True)

    inter_step = 2.0 * n * (n - 1)
    value = inter_step * args.steps / r64["elapsed"] / 1e9
    achieved = FLOP_PER_INTERACTION * n * (n - 1) / r64["kick_s"] / 1e12
    achieved32 = FLOP_PER_INTERACTION * n * (n - 1) / r32["kick_s"] / 1e12 if r32 else None
    value32 = inter_step * args.steps / r32["elapsed"] / 1e9 if r32 else None
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Ginter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": spec.name, "n": n, "dt_days": d["dt"], "n1": d["n1"], "n2": d["n2"],
                   "kicks_per_step": 2, "encounter_pairs_last_step": r64["pairs"],
                   "encounter_pairs_sha256_last_step": r64["pairs_sha256"],
                   "ipt": args.ipt, "slices": args.slices},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": recorded_traffic(),
                     "kernel": "k_kick_sym" if sym else "k_kick<256,1,KM_F64>",
                     "kernel_ms": round(r64["kick_s"] * 1e3, 4),
                     "kernel_ms_median": round(r64["kick_ms_median"], 4),
                     "kernel_ms_min": round(r64["kick_ms_min"], 4),
                     "flop_per_interaction": FLOP_PER_INTERACTION},
    }
    out["config"]["kick_form"] = "symmetric" if sym else "one-sided"
    if r1s:
        a1s = FLOP_PER_INTERACTION * n * (n - 1) / r1s["kick_s"] / 1e12
        out["one_sided"] = {"value": round(inter_step * args.steps / r1s["elapsed"] / 1e9, 3),
                            "unit": "Ginter/s",
                            "ms_per_step": round(r1s["elapsed"] / args.steps * 1e3, 4),
                            "kernel": "k_kick<256,1,KM_F64>",
                            "kernel_ms": round(r1s["kick_s"] * 1e3, 4),
                            "frac": round(a1s / FP64_VECTOR_PEAK_TFLOPS, 4),
                            "same_pairs": r1s["pairs_sha256"] == r64["pairs_sha256"]}
    if r32:
        out["mixed"] = {"value": round(value32, 3), "unit": "Ginter/s",
                        "ms_per_step": round(r32["elapsed"] / args.steps * 1e3, 4),
                        "kernel_ms": round(r32["kick_s"] * 1e3, 4),
                        "achieved_tflops": round(achieved32, 3),
                        "frac_fp32_vector_peak": round(achieved32 / FP32_VECTOR_PEAK_TFLOPS, 4),
                        "speedup_vs_fp64_kernel": round(r64["kick_s"] / r32["kick_s"], 3),
                        "encounter_pairs_last_step": r32["pairs"],
                        "encounter_pairs_sha256_last_step": r32["pairs_sha256"]}
        if not args.no_accuracy:
            out["mixed"]["accuracy_vs_fp64"] = mixed_accuracy(N, W, torch, np)
            out["mixed"]["energy_drift"] = energy_drift(N, W, torch, np)
            print(f"mixed accuracy done: {out['mixed']['accuracy_vs_fp64']} "
                  f"{out['mixed']['energy_drift']}", file=sys.stderr, flush=True)
    if not args.no_tp:
        out["test_particles"] = bench_tp(N, W, torch, np)
        print(f"test particles done: {out['test_particles']}", file=sys.stderr, flush=True)
    if not args.no_levels:
        out["levels"] = bench_levels(N, W, torch, np)
        print(f"levels done: {out['levels']}", file=sys.stderr, flush=True)
    if not args.no_levels:
        out["bs_ring"] = bench_bs_ring(N, W, torch, np)
        print(f"ring done: {out['bs_ring']}", file=sys.stderr, flush=True)
    if not args.no_levels:
        out["gr"] = bench_gr(N, W, torch, np)
        print(f"gr done: {out['gr']}", file=sys.stderr, flush=True)
    if not args.no_small:
        out["small_system"] = bench_small(N, W, torch, np)
        print(f"small system done: {out['small_system']}", file=sys.stderr, flush=True)
    if not args.no_sizes:
        out["sizes"] = bench_sizes(N, W, torch, np)
        out["sizes"]["n65536"] = {"workload": spec.name,
                                  "fp64_step_ms": out["ms_per_step"],
                                  "mixed_step_ms": out["mixed"]["ms_per_step"] if r32 else None}
        print(f"sizes done: {out['sizes']}", file=sys.stderr, flush=True)
        out["n2_zero"] = bench_n2_zero(N, W, torch, np)
        print(f"n2 = 0 done: {out['n2_zero']}", file=sys.stderr, flush=True)
    if not args.no_pairs_run:
        out["pairs_1000_steps"] = pairs_run(N, W, torch, np)
        print(f"pairs run done: {out['pairs_1000_steps']}", file=sys.stderr, flush=True)
    st_rc = r64["rc"]
    if not args.no_adjoint:
        st_adj = N.State.from_numpy(d, rc=st_rc.cpu().numpy())
        out["adjoint"] = bench_adjoint(N, W, torch, np, st_adj, N.Config(G=G),
                                       kick_ms_fp64=r64["kick_s"] * 1e3)
        print(f"adjoint done: {out['adjoint']}", file=sys.stderr, flush=True)
    if not args.no_batched:
        out["batched"] = bench_batched(args, N, W, torch, np)
        print(f"batched done: {out['batched']['graph_step_ms']} ms/step (graph)", file=sys.stderr,
              flush=True)
    if not args.no_cpu_baseline:
        import oracle
        rc = st_rc.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(d, rc, G, args.cpu_seconds)
        out["cpu_baseline"]["oracle_run_disk2048_100_steps"] = oracle_run_cfg0(N, W, torch, np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
