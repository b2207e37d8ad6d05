"""Benchmark of the batched ROK4E reaction substep on one MI355X.

One step = one reaction substep (Algorithm a:ROK4E over dt) for every cell of the batch,
with the cell states already resident in HBM.  Workload: the 53-species / 325-reaction
synthetic mechanism on a 256 x 256 flame slice (65,536 cells), M = 8, dt = 1e-5 s,
rtol = 1e-6, atol = 1e-12, pre-exponential factors scaled by 1e-8 (the calibrated
mechanism, whose attempt counts span one to a few hundred per cell).  The literal draw of
the generator (no multiplier; thousands to tens of thousands of attempts per cell) is
timed beside it on the 9- and 53-species workloads, and so is the stiffer mechanism
(multiplier 1e-5).

Prints one JSON line: FP64 cell-integrations/s as `value`, the mixed-precision figure
and speed-up beside it, the roofline of the integration kernel (algorithmic FP64
operations / kernel time against the FP64 vector peak), the standalone right-hand-side
and Arnoldi kernels against the same peak, the substep in conservative variables with
the auxiliary temperature on the flame slice, persistent vs per-attempt scheduling on the
262,144-cell bimodal batch and the throughput of its prefixes from 4,096 cells up, one
Simpler balanced splitting step on a 128^3 grid at CFL 0.5, and the CPU oracle timed on a
bounded sample on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ROK4E cell-integrations/s at 53 species, FP64 vs mixed, % of roofline"
A_SCALE = 1e-8
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (256 CUs x 128 flop/clk x 2.4 GHz)
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector, packed FP32 instructions
# HBM bytes of one integration launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
# (scaled by a plain device copy of known size); used only while the kernel sources
# hash to the value recorded with the measurement.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_integrate_53sp_flame.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def kernel_source_hash() -> str:
    """Hash of the HIP sources, the public header and the build flags."""
    from paper_1712_00953_amd import build
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1712_00953_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc)) + [os.path.join(ROOT, "include", "rok4e.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    h.update(" ".join(build.FLAGS).encode())
    return h.hexdigest()[:16]


def load_traffic():
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d


def timed_events(torch, stream, fn, reps):
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) * 1e-3 for a, b in ev]


def graph_replays(m, w, Y0, T0, p, torch, stream, reps=10):
    """The integration captured once in a HIP graph and replayed reps times on fresh
    copies of the inputs (copied before each replay, outside the timed region): the
    median replay time in ms (HIP events on the capture's replay stream)."""
    Y, T = Y0.clone(), T0.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(stream)
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            m.integrate(Y, T, p, w.dt, w.rtol, w.atol)
    stream.wait_stream(s)
    times = []
    for _ in range(reps + 1):
        Y.copy_(Y0)
        T.copy_(T0)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        g.replay()
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    del g
    return {"replays": reps, "median_ms": float(np.median(times[1:])), "min_ms": float(np.min(times[1:])),
            "max_ms": float(np.max(times[1:]))}


def run_gpu(w, precision, steps, warmup, R, torch, tune=True, graph_reps=10, layout=None):
    """The timed integration of the batch.  With tune, the launch tuner first picks the
    launch layout on a copy of the same batch (outside the timed region)."""
    from paper_1712_00953_amd import workmodel
    st = w.states
    n = st.n_cells
    dev = torch.device("cuda:0")
    Y0 = torch.tensor(st.Y, dtype=torch.float64, device=dev)
    T0 = torch.tensor(st.T, dtype=torch.float64, device=dev)
    p = torch.tensor(st.p, dtype=torch.float64, device=dev)
    # one private copy of the inputs per step, made before any timing
    copies = [(Y0.clone(), T0.clone()) for _ in range(warmup + steps)]
    m = R.Mech(w.mech, M=w.M, precision=precision, max_attempts=200000, **(layout or {}))
    m.reserve(n)
    tuning = m.tune(Y0, T0, p, w.dt, w.rtol, w.atol) if tune and not layout else None
    stream = torch.cuda.current_stream()   # the stream the library launches on
    for i in range(warmup):
        m.integrate(copies[i][0], copies[i][1], p, w.dt, w.rtol, w.atol)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        Yc, Tc = copies[warmup + i]
        ev[i][0].record(stream)
        m.integrate(Yc, Tc, p, w.dt, w.rtol, w.atol)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    graph_ms = graph_replays(m, w, Y0, T0, p, torch, stream) if graph_reps > 0 else None
    o = m.get_options()
    layout = {"lanes_per_cell": o.lanes_per_cell, "waves_per_block": o.waves_per_block,
              "jvp_gather": ["auto", "lds", "private"][o.jvp_gather], "waves_per_simd": o.waves_per_simd}
    stats = m.stats()
    acc = torch.zeros(n, dtype=torch.int32)
    rej = torch.zeros(n, dtype=torch.int32)
    sta = torch.zeros(n, dtype=torch.int32)
    m.cell_stats(acc, rej, sta)
    torch.cuda.synchronize()
    m.close()
    S = (acc + rej).numpy()
    Yl, Tl = copies[-1][0].cpu().numpy(), copies[-1][1].cpu().numpy()
    if stats["status_count"][0] != n:
        raise RuntimeError(f"cells failed: {stats}")
    ops = workmodel.batch_ops(w.mech, w.M, stats["accepted"], stats["rejected"])
    kavg = float(np.mean(kern_ms)) * 1e-3
    return dict(wall_s=wall, ms_per_step=wall / steps * 1e3, kernel_s=kavg,
                cells_per_s=n * steps / wall, attempts=stats["accepted"] + stats["rejected"],
                accepted=stats["accepted"], rejected=stats["rejected"],
                max_attempts=stats["max_attempts"], flops=ops["flops"],
                transcendentals=ops["transcendentals"],
                tflops=ops["flops"] / kavg * 1e-12,
                bytes=workmodel.state_bytes(w.mech, n),
                attempts_per_cell={q: int(np.percentile(S, float(q[1:]))) for q in ("p50", "p90", "p99")}
                | {"min": int(S.min()), "max": int(S.max()), "mean": float(S.mean())},
                attempts_per_s=(stats["accepted"] + stats["rejected"]) / kavg,
                final_state=(Yl, Tl), cell_counts=(acc.numpy(), rej.numpy()), layout=layout,
                tuning=tuning, graph=graph_ms)


def run_stiff(R, torch, synth, a_scale=1e-5):
    """The same 53-species flame slice on the stiffer mechanism (pre-exponential factors x
    1e-5 instead of 1e-8), where the Krylov stages pay against the explicit pair: one
    tuned FP64 integration, timed with HIP events after a warm-up call."""
    from paper_1712_00953_amd import workmodel
    w = synth.workload(2, a_scale=a_scale)
    st = w.states
    n = st.n_cells
    dev = torch.device("cuda:0")
    Y0 = torch.tensor(st.Y, dtype=torch.float64, device=dev)
    T0 = torch.tensor(st.T, dtype=torch.float64, device=dev)
    p = torch.tensor(st.p, dtype=torch.float64, device=dev)
    m = R.Mech(w.mech, M=w.M, max_attempts=2000000)
    m.reserve(n)
    # the tuning cache is keyed by the mechanism's size, which this mechanism shares with
    # the headline's: force a timing of its own
    tuning = m.tune(Y0, T0, p, w.dt, w.rtol, w.atol, force=True)
    stream = torch.cuda.current_stream()
    Y, T = Y0.clone(), T0.clone()
    m.integrate(Y, T, p, w.dt, w.rtol, w.atol)
    Y.copy_(Y0)
    T.copy_(T0)
    t = timed_events(torch, stream, lambda: m.integrate(Y, T, p, w.dt, w.rtol, w.atol), 1)[0]
    s = m.stats()
    m.close()
    ops = workmodel.batch_ops(w.mech, w.M, s["accepted"], s["rejected"])
    tf = ops["flops"] / t * 1e-12
    return {"workload": w.name + f" (pre-exponential factors x {a_scale:g})", "n_cells": n,
            "cells_per_s": n / t, "ms": t * 1e3, "attempts": s["accepted"] + s["rejected"],
            "max_attempts_cell": s["max_attempts"], "status_ok": s["status_count"][0],
            "tflops": tf, "frac_fp64_peak": tf / PEAK_FP64_TFLOPS, "tuning": tuning}


def run_literal(R, torch, synth, tuning=None):
    """The literal generator draw (pre-exponential factors log-uniform in [1e6, 1e14], no
    multiplier) on the 9-species batch and on the 53-species flame slice: one FP64
    integration each, timed with HIP events, in the headline's tuned layout (the tuner is
    not run here: one integration of the flame slice takes about half a minute)."""
    from paper_1712_00953_amd import workmodel
    out = {}
    for cfg in (1, 2):
        w = synth.workload(cfg, a_scale=1.0)
        st = w.states
        n = st.n_cells
        dev = torch.device("cuda:0")
        Y = torch.tensor(st.Y, dtype=torch.float64, device=dev)
        T = torch.tensor(st.T, dtype=torch.float64, device=dev)
        p = torch.tensor(st.p, dtype=torch.float64, device=dev)
        layout = {}
        if cfg == 2 and tuning:
            layout = {k: tuning[k] for k in ("lanes_per_cell", "waves_per_block", "jvp_gather",
                                             "waves_per_simd")}
        m = R.Mech(w.mech, M=w.M, max_attempts=1 << 22, **layout)
        m.reserve(n)
        stream = torch.cuda.current_stream()
        t = timed_events(torch, stream, lambda: m.integrate(Y, T, p, w.dt, w.rtol, w.atol), 1)[0]
        s = m.stats()
        acc = torch.zeros(n, dtype=torch.int32)
        rej = torch.zeros_like(acc)
        sta = torch.zeros_like(acc)
        m.cell_stats(acc, rej, sta)
        torch.cuda.synchronize()
        lanes = m.get_options().lanes_per_cell
        m.close()
        att = (acc + rej).numpy()
        ops = workmodel.batch_ops(w.mech, w.M, s["accepted"], s["rejected"])
        tf = ops["flops"] / t * 1e-12
        out[f"{w.mech.n_species}sp"] = {
            "workload": w.name + " (literal draw: A log-uniform in [1e6, 1e14])", "n_cells": n,
            "ms": t * 1e3, "cells_per_s": n / t, "attempts": int(att.sum()),
            "attempts_per_s": float(att.sum() / t),
            "attempts_per_cell": {"min": int(att.min()), "p50": float(np.percentile(att, 50)),
                                  "p95": float(np.percentile(att, 95)), "max": int(att.max()),
                                  "mean": float(att.mean())},
            "status_ok": s["status_count"][0], "lanes_per_cell": lanes, "tflops": tf,
            "frac_fp64_peak": tf / PEAK_FP64_TFLOPS}
    return out


def run_peak_check(R, torch, reps=5):
    """The attainable FP64 vector FMA rate (rok4e_fma_probe: eight independent FMA chains
    per thread, 2,048 blocks of 256) and HBM copy bandwidth (a 4 GiB device copy: 4 GiB
    read, 4 GiB written), medians of reps runs, beside the datasheet peaks the roofline
    fractions use."""
    stream = torch.cuda.current_stream()
    n, iters = 2048 * 256, 8192
    out = torch.empty(n, dtype=torch.float64, device="cuda:0")
    R.fma_probe(out, 64)
    t_fma = float(np.median(timed_events(torch, stream, lambda: R.fma_probe(out, iters), reps)))
    x = torch.ones(512 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    t_copy = float(np.median(timed_events(torch, stream, lambda: y.copy_(x), reps)))
    nbytes = 2 * x.numel() * 8
    del x, y, out
    torch.cuda.empty_cache()
    return {"fp64_fma_tflops": 16.0 * n * iters / t_fma * 1e-12, "fp64_datasheet_tflops": PEAK_FP64_TFLOPS,
            "hbm_copy_gbps": nbytes / t_copy * 1e-9, "hbm_datasheet_gbps": 8000.0,
            "note": "roofline fractions use the datasheet peaks"}


def run_subsystems(w, R, torch, reps=5):
    """The right-hand side and the Arnoldi basis (f(u_n), M JVPs, Gram-Schmidt) as
    standalone kernels over the same batch, against the FP64 vector peak."""
    from paper_1712_00953_amd import workmodel
    st = w.states
    n, N, M = st.n_cells, w.mech.n_species + 1, w.M
    dev = torch.device("cuda:0")
    Y = torch.tensor(st.Y, dtype=torch.float64, device=dev)
    T = torch.tensor(st.T, dtype=torch.float64, device=dev)
    p = torch.tensor(st.p, dtype=torch.float64, device=dev)
    dY, dT = torch.empty_like(Y), torch.empty_like(T)
    Q = torch.empty(n * M * N, dtype=torch.float64, device=dev)
    H = torch.empty(n * M * M, dtype=torch.float64, device=dev)
    Me = torch.empty(n, dtype=torch.int32, device=dev)
    m = R.Mech(w.mech, M=M)
    stream = torch.cuda.current_stream()
    m.rhs(Y, T, p, dY, dT)
    m.arnoldi(Y, T, p, Q, H, Me)
    t_rhs = float(np.median(timed_events(torch, stream, lambda: m.rhs(Y, T, p, dY, dT), reps)))
    t_arn = float(np.median(timed_events(torch, stream, lambda: m.arnoldi(Y, T, p, Q, H, Me), reps)))
    m.close()
    a = workmodel.attempt_ops(w.mech, M)
    out = {}
    for name, t, ops in (("rhs", t_rhs, a["rhs"]), ("arnoldi_basis", t_arn, a["basis"])):
        tf = ops * n / t * 1e-12
        out[name] = {"cells_per_s": n / t, "kernel_ms": t * 1e3, "algorithmic_flops_per_cell": ops,
                     "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": tf / PEAK_FP64_TFLOPS}
    return out


def run_schedules(R, torch, synth):
    """Persistent queue vs one launch per attempt on the 262,144-cell bimodal batch."""
    w = synth.workload(3, a_scale=A_SCALE)
    st = w.states
    n = st.n_cells
    dev = torch.device("cuda:0")
    Y0 = torch.tensor(st.Y, dtype=torch.float64, device=dev)
    T0 = torch.tensor(st.T, dtype=torch.float64, device=dev)
    p = torch.tensor(st.p, dtype=torch.float64, device=dev)
    out, res = {}, {}
    for name, sched, tune in (("persistent", R.PERSISTENT, False), ("persistent_tuned", R.PERSISTENT, True),
                              ("per_attempt", R.PER_ATTEMPT, False)):
        m = R.Mech(w.mech, M=w.M, max_attempts=200000, scheduling=sched)
        m.reserve(n)
        tuning = m.tune(Y0, T0, p, w.dt, w.rtol, w.atol, force=True) if tune else None
        Y, T = Y0.clone(), T0.clone()
        m.integrate(Y, T, p, w.dt, w.rtol, w.atol)
        Y.copy_(Y0)
        T.copy_(T0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.integrate(Y, T, p, w.dt, w.rtol, w.atol)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s = m.stats()
        o = m.get_options()
        m.close()
        res[name] = (Y, T)
        out[name] = {"cells_per_s": n / el, "ms": el * 1e3, "attempts": s["accepted"] + s["rejected"],
                     "max_attempts_cell": s["max_attempts"], "lanes_per_cell": o.lanes_per_cell,
                     "waves_per_block": o.waves_per_block, "jvp_gather": o.jvp_gather}
        if tuning is not None:
            out[name]["tuning"] = tuning
    out["speedup_persistent"] = out["persistent"]["cells_per_s"] / out["per_attempt"]["cells_per_s"]
    out["speedup_tuned_vs_default"] = out["persistent_tuned"]["cells_per_s"] / out["persistent"]["cells_per_s"]
    out["bitwise_equal"] = bool(torch.equal(res["persistent"][0], res["per_attempt"][0])
                                and torch.equal(res["persistent"][1], res["per_attempt"][1]))
    out["workload"] = w.name + " (pre-exponential factors x 1e-8)"
    return out


def run_conservative(w, R, torch, reps=3, v_scale=50.0, a=1e3, seed=5):
    """The reaction substep in conservative variables with the auxiliary temperature
    (rok4e_integrate_conservative) on the same 65,536-cell batch: the states moved to
    (rho Y_k, rho, rho u, rho E) with seeded velocities (50 m/s per component) and a
    seeded balancing constant on every row (1e3 /s times the row's magnitude)."""
    st = w.states
    n = st.n_cells
    rng = np.random.default_rng(seed)
    vel = v_scale * rng.standard_normal((3, n))
    Ru = 8.314462618
    Wk = np.asarray(w.mech.W)[:, None]
    cp = np.asarray(w.mech.cp)[:, None]
    hf = np.asarray(w.mech.hf)[:, None]
    rho = st.p / (Ru * st.T * (st.Y / Wk).sum(0))
    e = (st.Y * (hf + cp * (st.T - 298.15) - Ru * st.T / Wk)).sum(0)
    U = np.vstack([rho * st.Y, rho[None], rho * vel, (rho * (e + 0.5 * (vel * vel).sum(0)))[None]])
    S = a * np.abs(U) * rng.standard_normal(U.shape)
    dev = torch.device("cuda:0")
    U0 = torch.tensor(U, dtype=torch.float64, device=dev)
    Sd = torch.tensor(S, dtype=torch.float64, device=dev)
    Ta = torch.empty(n, dtype=torch.float64, device=dev)
    m = R.Mech(w.mech, M=w.M, max_attempts=200000)
    m.reserve(n)
    Ud = U0.clone()
    m.integrate_conservative(Ud, w.dt, w.rtol, w.atol, S=Sd, T_aux=Ta)
    times = []
    for _ in range(reps):
        Ud.copy_(U0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.integrate_conservative(Ud, w.dt, w.rtol, w.atol, S=Sd, T_aux=Ta)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    s = m.stats()
    m.close()
    el = float(np.median(times))
    return {"cells_per_s": n / el, "ms": el * 1e3, "attempts": s["accepted"] + s["rejected"],
            "max_attempts_cell": s["max_attempts"], "status_count": s["status_count"],
            "state_rows": int(w.mech.n_species) + 6,
            "inputs": "flame-slice states in conservative variables, velocities N(0, 50 m/s), "
                      "balancing constants 1e3/s x |U| x N(0, 1)"}


def run_curve(R, torch, synth, sizes=(4096, 16384, 32768, 65536, 131072, 262144), reps=2):
    """Throughput against batch size on the 262,144-cell bimodal batch (its cells are
    shuffled, so a prefix is a random subset): how far one GPU's share of a batch split
    over several GPUs (32,768 cells at eight) stays from the full-batch rate."""
    w = synth.workload(3, a_scale=A_SCALE)
    st = w.states
    dev = torch.device("cuda:0")
    Y0 = torch.tensor(st.Y, dtype=torch.float64, device=dev)
    T0 = torch.tensor(st.T, dtype=torch.float64, device=dev)
    p0 = torch.tensor(st.p, dtype=torch.float64, device=dev)
    m = R.Mech(w.mech, M=w.M, max_attempts=200000)
    m.reserve(st.n_cells)
    out = []
    for n in sizes:
        Yn, Tn, pn = Y0[:, :n].contiguous(), T0[:n].contiguous(), p0[:n].contiguous()
        Y, T = Yn.clone(), Tn.clone()
        m.integrate(Y, T, pn, w.dt, w.rtol, w.atol)
        times = []
        for _ in range(reps):
            Y.copy_(Yn)
            T.copy_(Tn)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m.integrate(Y, T, pn, w.dt, w.rtol, w.atol)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        s = m.stats()
        el = min(times)
        out.append({"n_cells": n, "ms": el * 1e3, "cells_per_s": n / el,
                    "attempts": s["accepted"] + s["rejected"], "max_attempts_cell": s["max_attempts"]})
    m.close()
    return {"workload": w.name + " (prefixes)", "points": out}


def run_splitting(R, torch, synth, nx=128, h=5e-6, reps=2):
    """One Simpler balanced splitting step on an nx^3 periodic grid carrying the 53-species
    flame profile along x (advection 10 m/s, diffusivity 2e-5 m^2/s, dx = 1e-4 m, so
    h = 5e-6 s is CFL 0.5): the whole step, and its reaction substep alone (same
    forcing), timed with HIP events."""
    w = synth.workload(2, a_scale=A_SCALE, n_cells=4)
    mech = w.mech
    ns = mech.n_species
    n = nx ** 3
    st = synth.states_flame(mech, nx, nx * nx, 4500)
    dev = torch.device("cuda:0")
    Y0 = torch.tensor(st.Y, dtype=torch.float64, device=dev)
    T0 = torch.tensor(st.T, dtype=torch.float64, device=dev)
    p = torch.tensor(st.p, dtype=torch.float64, device=dev)
    g = R.grid(nx, nx, nx, 1e-4, 10.0, 2e-5)
    m = R.Mech(mech, M=w.M, max_attempts=200000)
    m.reserve(n)
    work = torch.empty(m.workspace_bytes(g) // 8, dtype=torch.float64, device=dev)
    F = torch.empty((ns + 1) * n, dtype=torch.float64, device=dev)
    R.transport(g, ns, Y0, T0, F)
    stream = torch.cuda.current_stream()
    Y, T = Y0.clone(), T0.clone()

    def reset():
        Y.copy_(Y0)
        T.copy_(T0)

    def step():
        m.split_step(g, R.SPLIT_SIMPLER, Y, T, p, h, w.rtol, w.atol, work)

    def reaction():
        m.integrate(Y, T, p, h, w.rtol, w.atol, S=F)

    out = {}
    for name, fn in (("split_step", step), ("reaction_substep", reaction)):
        ts = []
        for _ in range(reps + 1):
            reset()
            ts += timed_events(torch, stream, fn, 1)
        out[name + "_ms"] = float(np.median(ts[1:])) * 1e3
    s = m.stats()
    m.close()
    # the transport operator alone (one evaluation of T(U): reads the [ns + 1][n] state,
    # writes [ns + 1][n]), timed directly
    top = timed_events(torch, stream, lambda: R.transport(g, ns, Y0, T0, F), 10)
    t_op = float(np.median(top))
    obytes = 8.0 * (ns + 1) * n * 2
    t_split = out["split_step_ms"] * 1e-3
    out.update({"grid": f"{nx}^3", "n_cells": n, "h": h, "scheme": "simpler", "rk4_substeps": 1,
                "cells_per_s": n / t_split,
                "transport_share_ms": max(t_split - out["reaction_substep_ms"] * 1e-3, 0.0) * 1e3,
                "transport_operator_ms": t_op * 1e3,
                "transport_operator_GBps": obytes / t_op * 1e-9,
                "transport_operator_frac_hbm": obytes / t_op * 1e-9 / PEAK_HBM_GBS,
                "reaction_attempts": s["accepted"] + s["rejected"]})
    return out


def run_study(R, torch, synth, n_cells=16384, t_end=1e-5, rtol=1e-4, atol=1e-8):
    """Efficiency study in the manner of Sec. 5 (Fig. 5): the cells integrate the same
    physical window t_end as a sequence of calls of length h_CFL (each call restarts the
    integrator at h0 = h_CFL, as a CFD code calling the reaction substep would), for
    h_CFL = 1e-9 .. 1e-5 s, with ROK4E at M = 4, 6, 8 and the explicit Dormand-Prince
    5(4) pair, at rtol = 1e-4, atol = 1e-8.  Cells: a stratified draw from the 53-species
    flame slice, on the calibrated mechanism (pre-exponential factors x 1e-8) and on a
    stiffer one (x 1e-5).  Reported per point: GPU time of the whole window (HIP events
    around the call sequence), attempts, and the error of the final state against ROK4E
    M = 8 at rtol = 1e-10, atol = 1e-14 over the window in one call (max relative error
    of T, 99th percentile over cells of the largest species error relative to
    max(|Y|, atol / rtol), the size below which the absolute tolerance governs)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for a_scale in (A_SCALE, 1e-5):
        w = synth.workload(2, a_scale=a_scale)
        idx = synth.stratified_sample(w.states.T, n_cells, 991)
        st = w.states.subset(idx)
        Y0 = torch.tensor(st.Y, dtype=torch.float64, device=dev)
        T0 = torch.tensor(st.T, dtype=torch.float64, device=dev)
        p = torch.tensor(st.p, dtype=torch.float64, device=dev)
        ref = R.Mech(w.mech, M=8, max_attempts=10_000_000)
        Yr, Tr = Y0.clone(), T0.clone()
        ref.integrate(Yr, Tr, p, t_end, 1e-10, 1e-14)
        torch.cuda.synchronize()
        Yr, Tr = Yr.cpu().numpy(), Tr.cpu().numpy()
        ok_ref = ref.stats()["status_count"][0] == st.n_cells
        ref.close()
        for method, M in (("rok4e", 4), ("rok4e", 6), ("rok4e", 8), ("rkdp45", 0)):
            m = R.Mech(w.mech, M=max(M, 1), max_attempts=10_000_000,
                       method=R.METHOD_RKDP45 if method == "rkdp45" else R.METHOD_ROK4E)
            for h_cfl in (1e-9, 1e-8, 1e-7, 1e-6, 1e-5):
                calls = int(round(t_end / h_cfl))
                Y, T = Y0.clone(), T0.clone()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record(stream)
                for _ in range(calls):
                    m.integrate(Y, T, p, h_cfl, rtol, atol)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                s = m.stats()
                att = s["accepted"] + s["rejected"]        # last call only
                bad = st.n_cells - s["status_count"][0]   # last call only
                Yg, Tg = Y.cpu().numpy(), T.cpu().numpy()
                errT = float(np.max(np.abs(Tg - Tr) / Tr))
                errY = float(np.percentile(np.max(np.abs(Yg - Yr) / np.maximum(np.abs(Yr), atol / rtol), axis=0),
                                           99))
                rows.append(dict(a_scale=a_scale, method=method, M=M or None, h_cfl=h_cfl, calls=calls,
                                 gpu_ms=ms, attempts_last_call=int(att), failed_cells_last_call=int(bad),
                                 err_T_max=errT, err_Y_p99=errY, reference_ok=bool(ok_ref)))
                log(f"study a={a_scale:g} {method}{'' if not M else f' M={M}'} h_cfl={h_cfl:g}: "
                    f"{ms:9.2f} ms, errT {errT:.2e}, errY {errY:.2e}")
            m.close()
    return dict(n_cells=n_cells, t_end=t_end, rtol=rtol, atol=atol, rows=rows)


def run_cpu_baseline(w, target_s=10.0):
    """The oracle on a uniformly drawn sample of the batch, all host threads.  Returns the
    baseline record and the oracle's results on the sample (indices, Y, T, accepted,
    rejected, status) for the parity check of the GPU result."""
    from oracle import oracle as O
    st = w.states
    threads = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(77)
    pilot = st.subset(np.sort(rng.choice(st.n_cells, 256, replace=False)))
    t0 = time.perf_counter()
    O.integrate(w.mech, pilot.Y, pilot.T, pilot.p, w.dt, w.rtol, w.atol, w.M, nthreads=threads)
    per_cell = (time.perf_counter() - t0) / 256
    n = int(min(st.n_cells, max(256, target_s / max(per_cell, 1e-9))))
    idx = np.sort(np.random.default_rng(78).choice(st.n_cells, n, replace=False))
    sub = st.subset(idx)
    t0 = time.perf_counter()
    res = O.integrate(w.mech, sub.Y, sub.T, sub.p, w.dt, w.rtol, w.atol, w.M, nthreads=threads)
    el = time.perf_counter() - t0
    rec = dict(value=n / el, unit="cell-integrations/s", cores=threads, kind="oracle",
               sample=f"{n} cells drawn uniformly (seed 78) from the {st.n_cells}-cell batch, "
                      f"{el:.1f} s wall on {threads} threads of {cpu_model()}")
    # one thread on an equal share of the sample: the per-core rate
    n1 = max(16, n // threads)
    sub1 = st.subset(idx[:n1])
    t0 = time.perf_counter()
    O.integrate(w.mech, sub1.Y, sub1.T, sub1.p, w.dt, w.rtol, w.atol, w.M, nthreads=1)
    el1 = time.perf_counter() - t0
    rec["single_thread"] = {"value": n1 / el1, "unit": "cell-integrations/s", "cores": 1,
                            "sample": f"the first {n1} cells of that sample, {el1:.1f} s wall"}
    return rec, (idx, *res)


def sample_parity(gpu, oracle_sample, rtol, atol, bar=1e-10, floor=1e-14):
    """FP64 GPU result of the full batch against the oracle on its timing sample:
    relative error on species above `floor` and on T, graded on the cells whose
    accept/reject counts equal the oracle's (several step sequences are correct; the
    others are counted and their tolerance-normalised difference reported), and the
    cells above the bar."""
    idx, Yo, To, ao, ro, so = oracle_sample
    (Yg, Tg), (ag, rg) = gpu["final_state"], gpu["cell_counts"]
    Yg, Tg, ag, rg = Yg[:, idx], Tg[idx], ag[idx], rg[idx]
    match = (ag == ao) & (rg == ro)
    graded = np.maximum(np.abs(Yo), np.abs(Yg)) >= floor
    rel = np.where(graded, np.abs(Yg - Yo) / np.maximum(np.abs(Yo), 1e-300), 0.0).max(axis=0)
    rel = np.maximum(rel, np.abs(Tg - To) / np.abs(To))
    norm = np.maximum((np.abs(Yg - Yo) / (atol + rtol * np.abs(Yo))).max(axis=0),
                      np.abs(Tg - To) / (atol + rtol * np.abs(To)))
    return {"cells": int(idx.size), "oracle_status_ok": int((so == 0).sum()),
            "count_match_frac": float(match.mean()),
            "max_rel_err_count_matched": float(rel[match].max()) if match.any() else None,
            "p99_rel_err_count_matched": float(np.percentile(rel[match], 99)) if match.any() else None,
            "cells_above_bar": int((rel[match] > bar).sum()), "bar": bar,
            "max_norm_err_all": float(norm.max()),
            "max_norm_err_count_mismatched": float(norm[~match].max()) if (~match).any() else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the standalone subsystem kernels and the scheduling comparison")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the measurement, copy 1 GiB device-to-device (a plain copy "
                         "kernel of known size, to scale HBM byte counters)")
    ap.add_argument("--print-source-hash", action="store_true",
                    help="print the kernel source hash that a traffic measurement must carry")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the automatic launch layout without running the launch tuner first")
    ap.add_argument("--layout", type=str, default=None,
                    help="launch options as JSON (e.g. '{\"waves_per_simd\": 4}') for the headline "
                         "integrations instead of tuning (profiling runs of the tuned kernel)")
    ap.add_argument("--study", action="store_true",
                    help="run only the efficiency study (ROK4E M = 4, 6, 8 vs Dormand-Prince 5(4) "
                         "over h_CFL = 1e-9 .. 1e-5) and print it as one JSON line")
    args = ap.parse_args()
    if args.print_source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the reaction substep is cell-parallel and "
              f"this build runs on a single MI355X; --gpus {args.gpus} is not supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1712_00953_amd import rok4e as R
    from paper_1712_00953_amd import synth
    R.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.study:
        print(json.dumps({"study": "efficiency vs h_CFL", **run_study(R, torch, synth)}), flush=True)
        return
    w = synth.workload(2, a_scale=A_SCALE)
    log(f"workload {w.name}: {w.states.n_cells} cells, M={w.M}, dt={w.dt}")
    layout = json.loads(args.layout) if args.layout else None
    fp64 = run_gpu(w, R.FP64, args.steps, args.warmup, R, torch, tune=not args.no_tune,
                   graph_reps=0 if args.no_extras else 10, layout=layout)
    log(f"fp64: {fp64['cells_per_s']:.4e} cells/s, {fp64['ms_per_step']:.2f} ms/step, "
        f"{fp64['attempts']} attempts/step, {fp64['tflops']:.3f} TFLOP/s")
    mixed = None
    if not args.no_mixed:
        mixed = run_gpu(w, R.MIXED, args.steps, args.warmup, R, torch, tune=not args.no_tune,
                        graph_reps=0, layout=layout)
        log(f"mixed: {mixed['cells_per_s']:.4e} cells/s, {mixed['ms_per_step']:.2f} ms/step")
    subsystems = schedules = splitting = conservative = curve = stiff = literal = peaks = None
    if not args.no_extras:
        stiff = run_stiff(R, torch, synth)
        log(f"stiffer mechanism: {stiff['ms']:.1f} ms, {stiff['attempts']} attempts, "
            f"{stiff['frac_fp64_peak'] * 100:.1f}% of FP64 peak")
        literal = run_literal(R, torch, synth, fp64["tuning"])
        log("literal draw: " + ", ".join(f"{k} {v['ms']:.1f} ms ({v['cells_per_s']:.3e} cells/s, "
                                         f"{v['attempts_per_cell']['p50']:.0f} attempts/cell median, "
                                         f"{v['frac_fp64_peak'] * 100:.1f}% of FP64 peak)"
                                         for k, v in literal.items()))
        peaks = run_peak_check(R, torch)
        log(f"peak check: FP64 FMA {peaks['fp64_fma_tflops']:.1f} TFLOP/s (datasheet "
            f"{PEAK_FP64_TFLOPS}), HBM copy {peaks['hbm_copy_gbps']:.0f} GB/s (datasheet 8000)")
        subsystems = run_subsystems(w, R, torch)
        log("subsystems: " + ", ".join(f"{k} {v['kernel_ms']:.3f} ms ({v['frac'] * 100:.1f}% of FP64 peak)"
                                       for k, v in subsystems.items()))
        conservative = run_conservative(w, R, torch)
        log(f"conservative variables: {conservative['ms']:.1f} ms, {conservative['attempts']} attempts")
        schedules = run_schedules(R, torch, synth)
        curve = run_curve(R, torch, synth)
        log("batch-size curve: " + ", ".join(f"{q['n_cells']} cells {q['cells_per_s']:.3e}/s"
                                            for q in curve["points"]))
        log(f"schedules: persistent {schedules['persistent']['ms']:.1f} ms, per-attempt "
            f"{schedules['per_attempt']['ms']:.1f} ms, bitwise equal {schedules['bitwise_equal']}")
        splitting = run_splitting(R, torch, synth)
        log(f"splitting: {splitting['grid']} Simpler step {splitting['split_step_ms']:.1f} ms "
            f"(reaction {splitting['reaction_substep_ms']:.1f} ms; transport operator "
            f"{splitting['transport_operator_ms']:.2f} ms, {splitting['transport_operator_GBps']:.0f} GB/s)")
    if args.copy_calibration:
        # write a 1 GiB buffer, evict it from the caches with a second one, then copy it:
        # the copy kernel reads 1 GiB and writes 1 GiB
        x = torch.ones(128 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        evict = torch.ones_like(x)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 1073741824 bytes read, 1073741824 bytes written "
            f"(last elementwise kernel), check {float(y[0] + evict[0])}")
        del x, y, evict
    cpu = parity = None
    if not args.no_cpu_baseline:
        cpu, oracle_sample = run_cpu_baseline(w, args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.4e} cells/s ({cpu['sample']})")
        parity = sample_parity(fp64, oracle_sample, w.rtol, w.atol)
        log(f"parity on the oracle sample: {parity}")

    traffic = load_traffic()
    achieved = fp64["tflops"]
    out = {
        "metric": METRIC,
        "value": fp64["cells_per_s"],
        "unit": "cell-integrations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name + " (pre-exponential factors x 1e-8)",
                   "n_species": w.mech.n_species, "n_reactions": w.mech.n_reactions,
                   "n_cells": w.states.n_cells, "M": w.M, "dt": w.dt, "rtol": w.rtol,
                   "atol": w.atol, "a_scale": A_SCALE, "precision": "fp64",
                   "attempts_per_step": fp64["attempts"], "max_attempts_cell": fp64["max_attempts"]},
        "attempts": {"per_cell": fp64["attempts_per_cell"], "per_s": fp64["attempts_per_s"],
                     "accepted": fp64["accepted"], "rejected": fp64["rejected"]},
        "layout": fp64["layout"],
        "tuning": fp64["tuning"],
        "graph_replay": fp64["graph"],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": traffic["hbm_bytes_per_launch"] if traffic else None,
                     "kernel": "k_integrate (persistent ROK4E integration)",
                     "kernel_ms": fp64["kernel_s"] * 1e3,
                     "algorithmic_flops_per_launch": fp64["flops"],
                     "transcendentals_per_launch": fp64["transcendentals"],
                     "state_bytes_per_launch": fp64["bytes"],
                     "hbm_frac_algorithmic": fp64["bytes"] / fp64["kernel_s"] / 1e9 / PEAK_HBM_GBS},
    }
    if traffic:
        out["roofline"]["traffic_detail"] = {k: traffic[k] for k in (
            "fetch_bytes_per_launch", "write_bytes_per_launch", "copy_scale_fetch", "copy_scale_write",
            "profile")}
        if "executed_fp64_ops_per_launch" in traffic:
            # FP64 operations the hardware executed (counters, every lane, FMA as two) over
            # the same launch time: the work the kernel issues, against the algorithmic work
            ex = traffic["executed_fp64_ops_per_launch"] / fp64["kernel_s"] * 1e-12
            out["roofline"]["executed"] = {"tflops": ex, "frac": ex / PEAK_FP64_TFLOPS,
                                           "issued_over_algorithmic": ex / achieved,
                                           "profile": traffic.get("counters_profile")}
    if mixed is not None:
        # error of the mixed result against the FP64 result of the same batch (every cell;
        # species above 1e-14 and T)
        (Ym, Tm), (Yd, Td) = mixed["final_state"], fp64["final_state"]
        graded = np.maximum(np.abs(Ym), np.abs(Yd)) >= 1e-14
        relY = np.abs(Ym - Yd)[graded] / np.abs(Yd)[graded]
        relT = np.abs(Tm - Td) / np.abs(Td)
        # cells whose accept/reject counts equal the FP64 run's: their difference is the
        # FP32 rounding alone; elsewhere FP32 rounding moved an error estimate across 1
        # and the two runs are different solutions within the tolerance
        (am, rm), (ad, rd) = mixed["cell_counts"], fp64["cell_counts"]
        same = (am == ad) & (rm == rd)
        rel_cell = np.where(graded, np.abs(Ym - Yd) / np.maximum(np.abs(Yd), 1e-300), 0.0).max(axis=0)
        rel_cell = np.maximum(rel_cell, relT)
        out["mixed"] = {"value": mixed["cells_per_s"], "unit": "cell-integrations/s",
                        "ms_per_step": mixed["ms_per_step"], "dtype": "f32 rates / f64 state",
                        "speedup_vs_fp64": mixed["cells_per_s"] / fp64["cells_per_s"],
                        "attempts_per_step": mixed["attempts"], "layout": mixed["layout"],
                        "tuning": mixed["tuning"],
                        "tflops_fp64_equivalent": mixed["tflops"],
                        # the same algorithmic operations (FP32 and FP64 counted alike)
                        # against the FP32 vector peak (reached only with packed FP32
                        # instructions, which this build does not use) and the FP64 one
                        "frac_fp32_peak": mixed["tflops"] / PEAK_FP32_TFLOPS,
                        "frac_fp64_peak": mixed["tflops"] / PEAK_FP64_TFLOPS,
                        "max_rel_err_vs_fp64": float(max(relY.max(), relT.max())),
                        "bar_rel_err": 1e-5,
                        "cells_above_bar": int((rel_cell > 1e-5).sum()),
                        "within_bar": bool(rel_cell.max() <= 1e-5),
                        "p99_rel_err_vs_fp64": float(np.percentile(relY, 99)),
                        "same_step_sequence_frac": float(same.mean()),
                        "max_rel_err_vs_fp64_same_steps": float(rel_cell[same].max()) if same.any() else None,
                        "max_abs_err_vs_fp64_other_cells": float(np.abs(Ym - Yd)[:, ~same].max())
                        if (~same).any() else None}
    if stiff is not None:
        out["stiffer_mechanism"] = stiff
    if literal is not None:
        out["literal_draw"] = literal
    if subsystems is not None:
        out["subsystems"] = subsystems
    if peaks is not None:
        out["peak_check"] = peaks
    if schedules is not None:
        out["schedules"] = schedules
    if splitting is not None:
        out["splitting"] = splitting
    if conservative is not None:
        out["conservative"] = conservative
    if curve is not None:
        out["batch_size_curve"] = curve
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if parity is not None:
        out["parity_fp64_vs_oracle"] = parity
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
