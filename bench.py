"""Benchmark of the coupled LBM + WENO step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 3d|2d]

A step is one coupled time step of the whole hot path: moments + force,
BGK-Guo collide + in-place stream (D3Q19 or D2Q9), and the three TVD-RK3
WENO5 stages of the particle concentration (plus the S update in 2D), with
inputs already resident in device memory.  The throughput comes from K
steps with nothing recorded between launches; the phase and per-kernel
durations (and the roofline's) from a second pass of K steps with the
library's HIP events around every launch.  The default workload is the 3D
D3Q19 FP32 (shifted populations) run on 256x256x512 cells; the 2D D2Q9 FP32
run with the second scalar S on 1024x2048 is timed in the same invocation
and reported under "also".  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
METRIC = "coupled LBM+WENO MLUPS & HBM GB/s vs roofline; adjoint/forward time ratio"
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def _alg_bytes(wl) -> dict:
    """Algorithmic bytes per cell update (minimum the method must move).

    step: read + write every population and every transported scalar once
    (each particle size class is a transported scalar).
    collide_stream kernel: read + write every population, read the scalars
    that set the buoyancy force.
    transport (the three RK stages, per step): stage 1 reads C and the
    velocity and writes a1; stages 2 and 3 also read C; each reads its input
    stage and writes one value (the S update adds S read and written)."""
    s = 4 if wl.precision == "fp32_shifted" else 8
    nsc = max(1, wl.n_classes) + (1 if wl.has_s else 0)
    ncls = max(1, wl.n_classes)
    u = wl.dim * s
    stages = ncls * ((2 * s + u) + 2 * (3 * s + u)) + (2 * s if wl.has_s else 0)
    return {"step": 2 * wl.q * s + 2 * nsc * s,
            "collide_stream": 2 * wl.q * s + nsc * s,
            "transport": stages}


_SOURCES = {"collide_stream": ("lbm.hip", "lbm_device.h"),
            "transport": ("transport_tiled.h", "transport_tiled.hip", "transport_device.h")}


def _kernel_hash(kind: str = "collide_stream") -> str:
    """Hash of what a phase's kernels are built from: their source files and
    the run descriptor they read (the RunDev struct)."""
    csrc = os.path.join(ROOT, "paper_2106_07694_amd", "csrc")
    h = hashlib.sha256()
    for name in _SOURCES[kind]:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "lbw_internal.h")) as fh:
        text = fh.read()
    start = text.index("struct RunDev {")
    h.update(text[start:text.index("};", start)].encode())
    return h.hexdigest()[:16]


def _traffic(wl_name: str, kernel: str):
    """HBM bytes per launch (collide_stream: the mean of the two kernels of
    the in-place pair) or per step (transport: its three stages) from
    committed rocprofv3 counter runs, if they were taken on the current
    kernel source; else None."""
    try:
        with open(PROFILE_COUNTERS) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(wl_name, {}).get(kernel)
    if not e or e.get("source_hash") != _kernel_hash(kernel):
        return None
    return e.get("bytes_per_launch")


def ingest_counters(fetch_csv: str, write_csv: str, workload: str, cells: int,
                    copy_bytes: int = 256 << 20) -> dict:
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; CSV output
    of the same bench command) into per-kernel HBM bytes, each counter scaled
    by what it reads for the known-size copy kernel of that run, and store
    them in profiles/hbm_traffic.json under `workload` with the current
    source hashes."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        vals = defaultdict(list)
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                vals[row["Kernel_Name"]].append(float(row["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in vals.items()}, {k: len(v) for k, v in vals.items()}

    fetch, n_f = per_kernel(fetch_csv, "FETCH_SIZE")
    write, _ = per_kernel(write_csv, "WRITE_SIZE")
    copy = [k for k in fetch if "AUnaryFunctor" in k or "MulFunctor" in k]
    if not copy:
        raise ValueError("the copy kernel (torch.mul of a 256 MiB tensor) is not in the counter runs")
    fs = copy_bytes / 1024.0 / fetch[copy[0]]
    ws = copy_bytes / 1024.0 / write[copy[0]]
    kernels = {}
    for k in fetch:
        if k in copy or k not in write or "lbw::" not in k:
            continue
        short = k.replace("(anonymous namespace)::", "").replace("lbw::", "")
        short = short[5:] if short.startswith("void ") else short
        short = short.split("(")[0]
        fb, wb = fetch[k] * 1024.0 * fs, write[k] * 1024.0 * ws
        kernels[short] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                          "bytes_per_cell": (fb + wb) / cells, "launches": n_f[k]}
    entry = {"_calibration": {"kernel": "torch.mul(src, 1.0, out=dst), 256 MiB float32 each way",
                              "fetch_kib_read": fetch[copy[0]], "write_kib_read": write[copy[0]],
                              "fetch_scale": fs, "write_scale": ws},
             "kernels": kernels}
    cs = [v for k, v in kernels.items() if k.startswith("k_collide_stream<")]
    if cs:
        f, w = (sum(v[x] for v in cs) / len(cs) for x in ("fetch_bytes", "write_bytes"))
        entry["collide_stream"] = {"source_hash": _kernel_hash("collide_stream"), "fetch_bytes": f,
                                   "write_bytes": w, "bytes_per_launch": f + w}
    st = [v for k, v in kernels.items() if k.startswith("k_stage_tiled<")]
    if len(st) == 3:
        f, w = (sum(v[x] for v in st) for x in ("fetch_bytes", "write_bytes"))
        entry["transport"] = {"source_hash": _kernel_hash("transport"), "fetch_bytes": f,
                              "write_bytes": w, "bytes_per_launch": f + w}
    try:
        with open(PROFILE_COUNTERS) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        d = {}
    d = {k: v for k, v in d.items() if not k.startswith("_")}
    d[workload] = entry
    with open(PROFILE_COUNTERS, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    return entry


def run_gpu(wl, steps: int, warmup: int, diagnostics: bool = True, tuned_as=None) -> dict:
    """tuned_as: the workload whose autotuned launch shapes to use (default
    wl itself)."""
    import torch
    from paper_2106_07694_amd import lbw

    cfg = lbw.RunConfig.from_workload(wl)
    sol = lbw.Solver(cfg)
    tuned = _tuned_launch(tuned_as or wl)
    if tuned:
        sol.set_launch(**tuned)
    sol.setup_workload(wl)
    sol.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    # the throughput pass: the steps alone, bracketed by two events on the
    # solver's stream
    start.record(sol.stream)
    sol.step(steps)
    stop.record(sol.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    # the phase pass: the same number of steps again with the library's HIP
    # events around every launch (per-phase and per-kernel durations, the
    # roofline's kernel time); the events themselves cost time between
    # launches (about 15 us per step of the 2D workload), so the throughput
    # is taken from the pass without them
    sol.timing_begin()
    torch.cuda.synchronize()
    start.record(sol.stream)
    sol.step(steps)
    stop.record(sol.stream)
    torch.cuda.synchronize()
    ms_instr = start.elapsed_time(stop)
    phases = sol.timing_end()
    # untimed sanity: the particle budget must close
    mass = sol.reduce(lbw.MASS_C)[0] + sol.reduce(lbw.DEPOSIT)[0]
    diag = run_diagnostics(sol, wl) if diagnostics else None
    sol.close()
    cells = wl.cells
    ab = _alg_bytes(wl)
    nst = max(phases["steps"], 1)
    cs_ms = phases["collide_stream_ms"] / nst
    tr_ms = phases["transport_ms"] / nst
    step_ms = ms / steps
    cs_gbs = cells * ab["collide_stream"] / (cs_ms * 1e-3) / 1e9
    tr_gbs = cells * ab["transport"] / (tr_ms * 1e-3) / 1e9
    step_gbs = cells * ab["step"] / (step_ms * 1e-3) / 1e9
    cs_traffic = _traffic(wl.name, "collide_stream")
    tr_traffic = _traffic(wl.name, "transport")
    step_traffic = (cs_traffic + tr_traffic) if cs_traffic and tr_traffic else None
    return {
        "mlups": cells * steps / (ms * 1e-3) / 1e6,
        "ms_per_step": step_ms,
        "ms_per_step_with_phase_events": ms_instr / steps,
        "phase_ms_per_step": {"collide_stream": cs_ms, "transport": tr_ms},
        "step_alg_gbs": step_gbs,
        # the coupled step against the HBM roofline: the method's algorithmic
        # bytes per cell update over the measured time per step; the phases
        # below it (HIP events around their launches in the second pass)
        "roofline": {"bound": "hbm", "scope": "coupled step", "achieved": step_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": step_gbs / HBM_PEAK_GBS,
                     "traffic": step_traffic, "alg_bytes_per_cell": ab["step"],
                     "cells_per_step": cells,
                     "kernels": {
                         "collide_stream": {
                             "bound": "hbm", "achieved": cs_gbs, "frac": cs_gbs / HBM_PEAK_GBS,
                             "ms": cs_ms, "alg_bytes_per_cell": ab["collide_stream"],
                             "traffic": cs_traffic, "cells_per_launch": cells},
                         "transport": {
                             "bound": "valu (vector-issue bound at the power-limited clock)", "achieved": tr_gbs,
                             "frac": tr_gbs / HBM_PEAK_GBS, "ms": tr_ms, "launches": 3,
                             "alg_bytes_per_cell": ab["transport"], "traffic": tr_traffic}}},
        "particle_budget": mass,
        "diagnostics": diag,
    }


def run_diagnostics(sol, wl, reps: int = 20) -> dict:
    """Time the in-situ diagnostics on the state the timed steps left (outside
    the timed region): front height per column at C0/2, its spectrum averaged
    over the rows along each lateral axis, and the mass below the mid plane.
    The front scan stops at the first cell that reaches the threshold, so its
    algorithmic bytes are the cells scanned (from the heights it returns)
    plus the heights written."""
    import numpy as np
    import torch

    thr = 0.5 * wl.c0
    st = sol.stream
    esize = 4 if wl.precision == "fp32_shifted" else 8
    h = sol.front_height(thr)
    psd = {axis: sol.front_psd(h, axis, -1) for axis in range(wl.dim - 1)}
    torch.cuda.synchronize()

    def timed(fn) -> float:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms_front = timed(lambda: sol.front_height(thr, out=h))
    ms_psd = {axis: timed(lambda axis=axis: sol.front_psd(h, axis, -1, out=psd[axis]))
              for axis in psd}
    plane = wl.nvert // 2
    ms_mass = timed(lambda: sol.mass_below(plane))
    hv = h.cpu().numpy().ravel()
    scanned = np.where(hv >= wl.nvert, wl.nvert,
                       np.clip(np.ceil(hv - 0.5), 0, wl.nvert - 1) + 1).sum()
    front_bytes = float(scanned) * esize + hv.size * 8
    mass_bytes = float(plane) * (wl.cells // wl.nvert) * esize
    return {
        "threshold": thr,
        "front_height_ms": ms_front,
        "front_height_alg_gbs": front_bytes / (ms_front * 1e-3) / 1e9,
        "front_cells_scanned": int(scanned),
        "front_psd_ms": {("x", "y")[a]: v for a, v in ms_psd.items()},
        "psd_bins": {("x", "y")[a]: int(psd[a].numel()) for a in psd},
        "mass_below_ms": ms_mass,
        "mass_below_alg_gbs": mass_bytes / (ms_mass * 1e-3) / 1e9,
        "mass_below_note": "includes the device-to-host copy and stream synchronisation",
        "mean_front_height": float(hv.mean()),
    }


def _tuned_launch(wl):
    from paper_2106_07694_amd import autotune
    return autotune.lookup(wl.name)


def run_sweep(steps: int, warmup: int) -> dict:
    """The 64-run parameter sweep (uneven 2D grids): all runs batched into one
    persistent launch per phase and replayed through a HIP graph, against the
    same runs advanced one at a time through the single-run path."""
    import torch
    from paper_2106_07694_amd import autotune, lbw, workloads as W

    runs = W.sweep_runs()
    cfgs = [lbw.RunConfig.from_workload(w) for w in runs]
    cells = sum(w.cells for w in runs)
    side = torch.cuda.Stream()
    sol = lbw.Solver(cfgs, stream=side)
    launch = autotune.lookup("sweep_64") or {}
    launch = dict(launch, graph=1)
    sol.set_launch(**launch)
    for i, w in enumerate(runs):
        sol.setup_workload(w, run=i)
    sol.step(warmup)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(side)
    sol.step(steps)
    stop.record(side)
    torch.cuda.synchronize()
    ms_batched = start.elapsed_time(stop)
    sol.close()
    del sol
    # one at a time: each run's own solver with the sweep's tuned launch
    # shape, same stream; once with a host launch per kernel and once
    # replaying each run's two-step HIP graph
    def sequential(graph: int) -> float:
        singles = []
        for w, c in zip(runs, cfgs):
            one = lbw.Solver(c, stream=side)
            one.set_launch(**dict(launch, graph=graph))
            one.setup_workload(w)
            one.step(2)
            singles.append(one)
        torch.cuda.synchronize()
        start.record(side)
        for one in singles:
            one.step(steps)
        stop.record(side)
        torch.cuda.synchronize()
        t = start.elapsed_time(stop)
        for one in singles:
            one.close()
        return t

    ms_seq = sequential(0)
    ms_seq_graph = sequential(1)
    return {"workload": "sweep_64_uneven_2d_fp32", "runs": len(runs), "cells": cells,
            "steps": steps, "batched_mlups": cells * steps / (ms_batched * 1e-3) / 1e6,
            "sequential_mlups": cells * steps / (ms_seq * 1e-3) / 1e6,
            "sequential_graph_mlups": cells * steps / (ms_seq_graph * 1e-3) / 1e6,
            "speedup": ms_seq / ms_batched,
            "speedup_vs_graph_replayed_sequential": ms_seq_graph / ms_batched,
            "launch": launch}


def run_precision(nsteps: int, marks=(1000, 5000, 10000, 20000), wl=None) -> dict:
    """Form (1) against the plain FP64 step on the same GPU: a workload (the
    2D two-scalar one unless wl is given) run in FP32 with shifted
    populations and in FP64 from the same seeded state; relative L2 differences of u, C and the per-column deposit
    (and of the total deposited mass) at several step counts.  The FP64 GPU
    path is the reference here because it equals the FP64 oracle to 1e-12 on
    every size the oracle can step; at this size the oracle would need tens
    of minutes on the host."""
    import numpy as np
    import torch
    from paper_2106_07694_amd import autotune, lbw, workloads as W

    wl = wl or W.C2
    marks = [m for m in marks if m <= nsteps] or [nsteps]
    runs = {}
    for prec in ("fp64", "fp32_shifted"):
        cfg = lbw.RunConfig.from_workload(wl.replace(precision=prec))
        sol = lbw.Solver(cfg)
        tuned = autotune.lookup(wl.name)
        if tuned:
            sol.set_launch(**tuned)
        sol.setup_workload(wl)
        snaps, done = {}, 0
        for m in marks:
            sol.step(m - done)
            done = m
            torch.cuda.synchronize()
            snaps[m] = {k: sol.field(k).double().cpu().numpy() for k in ("u", "c", "deposit")}
            snaps[m]["deposited"] = float(sol.reduce(lbw.DEPOSIT)[0])
        sol.close()
        runs[prec] = snaps
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    out = {"workload": wl.name, "reference": "fp64 (GPU)", "steps": marks, "l2_rel": {}}
    for m in marks:
        a, b = runs["fp32_shifted"][m], runs["fp64"][m]
        out["l2_rel"][str(m)] = {
            "u": rel(a["u"], b["u"]), "c": rel(a["c"], b["c"]),
            "deposit": rel(a["deposit"], b["deposit"]),
            # the front has not reached the floor here: the deposit is the sum
            # of the seeded +-1e-3 noise of the clear layer, near zero, so the
            # totals are given with their absolute difference
            "deposited_mass_fp64": b["deposited"], "deposited_mass_fp32": a["deposited"],
            "deposited_mass_abs_diff": abs(a["deposited"] - b["deposited"])}
    return out


def run_precision_oracle(nsteps: int, wl=None) -> dict:
    """Form (1) and the plain FP64 step against the FP64 oracle itself: the
    2D two-scalar workload (full grid) advanced nsteps from the same seeded
    state on the GPU (FP32 shifted and FP64) and by the oracle on the host;
    relative L2 differences of u, C, S and the per-column deposit."""
    import numpy as np
    import torch
    import oracle
    from paper_2106_07694_amd import autotune, lbw, workloads as W

    wl = wl or W.C2
    gpu = {}
    for prec in ("fp64", "fp32_shifted"):
        cfg = lbw.RunConfig.from_workload(wl.replace(precision=prec))
        sol = lbw.Solver(cfg)
        tuned = autotune.lookup(wl.name)
        if tuned:
            sol.set_launch(**tuned)
        sol.setup_workload(wl)
        sol.step(nsteps)
        torch.cuda.synchronize()
        gpu[prec] = {k: sol.field(k).double().cpu().numpy() for k in ("u", "c", "s", "deposit")}
        sol.close()
    ocfg = oracle.OracleConfig(q=wl.q, nx=wl.nx, ny=wl.ny, nz=wl.nz, tau=wl.tau, vs=wl.vs,
                               kappa_c=wl.kappa_c, gp_c=wl.gp_c, has_s=wl.has_s,
                               kappa_s=wl.kappa_s, gp_s=wl.gp_s)
    c, s = W.initial_scalars(wl)
    t0 = time.perf_counter()
    _, oc, os_, od, ou = oracle.run(ocfg, oracle.equilibrium(ocfg), c, s, nsteps=nsteps, want_u=True)
    dt = time.perf_counter() - t0
    ref = {"u": ou, "c": oc, "s": os_, "deposit": od}
    rel = lambda a, b: float(np.linalg.norm(a.ravel() - b.ravel()) / max(np.linalg.norm(b), 1e-300))
    return {"workload": wl.name, "reference": "FP64 oracle (host)", "steps": nsteps,
            "oracle_s": dt,
            "l2_rel": {prec: {k: rel(gpu[prec][k], ref[k]) for k in ref} for prec in gpu}}


def run_adjoint(nsteps: int) -> dict:
    """Gradient of the deposited mass for the 512x1024 FP32 run: the plain
    forward, the checkpointed forward (a checkpoint every ~sqrt(N) steps) and
    the backward (segment replay + reverse steps), each timed end to end."""
    import torch
    from paper_2106_07694_amd import adjoint, autotune, lbw, workloads as W

    wl = W.C5
    cfg = lbw.RunConfig.from_workload(wl)
    launch = autotune.lookup(wl.name)
    c0, _ = W.initial_scalars(wl)
    sol = lbw.Solver(cfg)
    if launch:
        sol.set_launch(**launch)
    sol.setup_workload(wl)
    sol.step(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol.step(nsteps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    sol.close()
    # warm-up of the gradient path (untimed, like the forward's warm-up
    # steps): a short forward and backward, so the reverse kernels' first
    # launches are not inside the timed backward
    c0w = torch.from_numpy(c0).to("cuda", torch.float32).requires_grad_(True)
    vsw = torch.tensor(cfg.vs, dtype=torch.float64, requires_grad=True)
    adjoint.DepositedMass.apply(c0w, vsw, cfg, 4, None, launch).backward()
    torch.cuda.synchronize()
    c0t = torch.from_numpy(c0).to("cuda", torch.float32).requires_grad_(True)
    vst = torch.tensor(cfg.vs, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = adjoint.DepositedMass.apply(c0t, vst, cfg, nsteps, None, launch)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    seg = adjoint.default_segment(nsteps)
    return {"workload": wl.name, "steps": nsteps, "checkpoint_every": seg,
            "forward_s": t_plain, "forward_checkpointed_s": t_fwd, "backward_s": t_bwd,
            "adjoint_forward_ratio": t_bwd / t_plain,
            "adjoint_vs_checkpointed_forward_ratio": t_bwd / t_fwd,
            "J": float(J.item()), "dJ_dVs": float(vst.grad.item()),
            "grad_c0_l2": float(c0t.grad.double().norm().item())}


def calibrate_copy(mib: int = 256, reps: int = 10) -> dict:
    """A plain copy-like kernel of known size (read mib MiB, write mib MiB),
    run so that profiler counters can be scaled against its known bytes, and
    timed as the achievable-bandwidth reference (one untimed call first, so
    the kernel's first launch is not in the timing)."""
    import torch
    n = mib * 1024 * 1024 // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    return {"bytes_read": n * 4, "bytes_written": n * 4, "ms": ms,
            "gbs": 2 * n * 4 / (ms * 1e-3) / 1e9}


def cpu_baseline(wl, nz_crop: int, ny_crop: int, steps: int, one_thread=None) -> dict:
    """The FP64 oracle as it stands, timed on the host cores on a crop of
    the workload (vertical extent cut), reported as MLUPS.  one_thread =
    (nz_crop, ny_crop, steps): also time it on one thread, in a child
    process started with OMP_NUM_THREADS=1 (the thread count of the
    oracle's OpenMP runtime is fixed when it starts)."""
    import oracle
    from paper_2106_07694_amd import workloads as W

    out1 = None
    if one_thread:
        import subprocess
        code = ("import json, sys; sys.path.insert(0, %r); import bench; "
                "from paper_2106_07694_amd import workloads as W; "
                "print(json.dumps(bench.cpu_baseline(W.%s, %d, %d, %d)))"
                % (ROOT, wl_var(wl), *one_thread))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=600)
        if r.returncode == 0:
            out1 = json.loads(r.stdout.strip().splitlines()[-1])
        else:
            out1 = {"error": r.stderr[-400:]}
    sample = wl.replace(nz=nz_crop) if wl.dim == 3 else wl.replace(ny=ny_crop)
    ocfg = oracle.OracleConfig(q=sample.q, nx=sample.nx, ny=sample.ny, nz=sample.nz,
                               shifted=True, tau=sample.tau, vs=sample.vs,
                               kappa_c=sample.kappa_c, gp_c=sample.gp_c, has_s=sample.has_s,
                               kappa_s=sample.kappa_s, gp_s=sample.gp_s)
    c, s = W.initial_scalars(sample)
    f = oracle.equilibrium(ocfg)
    t0 = time.perf_counter()
    oracle.run(ocfg, f, c, s, nsteps=steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    res = {"value": sample.cells * steps / dt / 1e6, "unit": "MLUPS", "cores": cores,
           "kind": "oracle",
           "sample": f"{steps} FP64 oracle steps on a {sample.nx}x{sample.ny}x{sample.nz} crop "
                     f"of the workload ({dt:.1f} s)"}
    if out1 is not None:
        res["one_thread"] = out1
    return res


def wl_var(wl) -> str:
    """Name of the workloads-module variable holding wl."""
    from paper_2106_07694_amd import workloads as W
    for k, v in vars(W).items():
        if v is wl:
            return k
    raise KeyError(wl.name)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=["3d", "2d"], default="3d")
    ap.add_argument("--grid", type=int, nargs=3, metavar=("NX", "NY", "NZ"),
                    help="time the main workload's physics on this grid instead (2D: NZ = 1), "
                         "with that workload's tuned launch; the run must fit the device "
                         "(3D FP32: 100 B per cell)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-also", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=5000)
    ap.add_argument("--no-classes", action="store_true",
                    help="skip the four-size-class run of the 3D workload")
    ap.add_argument("--no-full-force", action="store_true",
                    help="skip the 2D two-scalar run with the full force and settling")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32-vs-FP64 error report of the 2D workload")
    ap.add_argument("--precision-steps", type=int, default=20000)
    ap.add_argument("--precision-3d", type=int, default=2000, metavar="STEPS",
                    help="compare FP32 against FP64 on the 3D workload over STEPS steps "
                         "(reported under fp32_vs_fp64_3d; 0 skips it)")
    ap.add_argument("--precision-oracle", type=int, default=0, metavar="STEPS",
                    help="also compare the 2D two-scalar workload's FP32 and FP64 runs with the "
                         "FP64 oracle after STEPS steps (full grid; the oracle takes about 0.1 s "
                         "per step on 16 cores; reported under fp32_vs_oracle; off by default)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="store per-kernel HBM bytes from two rocprofv3 --pmc runs of this "
                         "command (FETCH_SIZE, WRITE_SIZE) in profiles/hbm_traffic.json and exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run the known-size copy kernel (profiler counter calibration); it runs "
                         "by default unless --no-copy")
    ap.add_argument("--no-copy", action="store_true",
                    help="skip the copy kernel that measures the achievable bandwidth")
    args = ap.parse_args()
    if args.ingest_counters:
        from paper_2106_07694_amd import workloads as W
        wl = W.C3 if args.workload == "3d" else W.C2
        e = ingest_counters(*args.ingest_counters, workload=wl.name, cells=wl.cells)
        print(json.dumps({k: v for k, v in e.items() if k != "kernels"}))
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        return 2

    import torch
    from paper_2106_07694_amd import lbw, workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1
    if not os.path.exists(lbw.LIB_PATH):
        from paper_2106_07694_amd import build
        build.build()

    main_wl, other = (W.C3, W.C2) if args.workload == "3d" else (W.C2, W.C3)
    base_wl = main_wl
    if args.grid:
        nx, ny, nz = args.grid
        if (main_wl.dim == 2) != (nz == 1):
            print("--grid: NZ must be 1 for the 2D workload and above 1 for the 3D one",
                  file=sys.stderr)
            return 2
        size = f"{nx}x{ny}x{nz}" if main_wl.dim == 3 else f"{nx}x{ny}"
        main_wl = main_wl.replace(name=f"{main_wl.name.rsplit('_', 1)[0]}_{size}", nx=nx, ny=ny, nz=nz)
    print(f"[bench] {main_wl.name}: warmup {args.warmup}, timing {args.steps} steps", file=sys.stderr,
          flush=True)
    res = run_gpu(main_wl, args.steps, args.warmup, tuned_as=base_wl)
    print(f"[bench] {main_wl.name}: {res['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    also = None
    if not args.no_also:
        o = run_gpu(other, args.steps, args.warmup)
        print(f"[bench] {other.name}: {o['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        also = {"workload": other.name, "value": o["mlups"], "unit": "MLUPS",
                "ms_per_step": o["ms_per_step"],
                "ms_per_step_with_phase_events": o["ms_per_step_with_phase_events"],
                "phase_ms_per_step": o["phase_ms_per_step"],
                "step_alg_gbs": o["step_alg_gbs"], "roofline": o["roofline"],
                "diagnostics": o["diagnostics"]}
    sweep = None
    if not args.no_sweep:
        sweep = run_sweep(min(args.steps, 200), 4)
        print(f"[bench] sweep: batched {sweep['batched_mlups']:.0f} MLUPS, one at a time "
              f"{sweep['sequential_mlups']:.0f} MLUPS ({sweep['speedup']:.1f}x), one at a time "
              f"with graph replay {sweep['sequential_graph_mlups']:.0f} MLUPS "
              f"({sweep['speedup_vs_graph_replayed_sequential']:.1f}x)", file=sys.stderr, flush=True)
    adj = None
    if not args.no_adjoint:
        adj = run_adjoint(args.adjoint_steps)
        print(f"[bench] adjoint: forward {adj['forward_s']:.3f} s, backward {adj['backward_s']:.3f} s "
              f"(ratio {adj['adjoint_forward_ratio']:.2f})", file=sys.stderr, flush=True)
    poly = None
    if not args.no_classes and main_wl.dim == 3:
        p = run_gpu(W.C6, min(args.steps, 200), args.warmup, diagnostics=False, tuned_as=W.C3)
        poly = {"workload": W.C6.name, "classes": W.C6.n_classes, "value": p["mlups"],
                "unit": "MLUPS", "ms_per_step": p["ms_per_step"],
                "phase_ms_per_step": p["phase_ms_per_step"], "step_alg_gbs": p["step_alg_gbs"],
                "step_alg_bytes_per_cell": _alg_bytes(W.C6)["step"],
                "collide_stream_alg_gbs": p["roofline"]["achieved"]}
        print(f"[bench] {W.C6.name}: {p['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    full = None
    if not args.no_full_force:
        p = run_gpu(W.C7, min(args.steps, 500), args.warmup, diagnostics=False, tuned_as=W.C2)
        full = {"workload": W.C7.name, "vs_s": W.C7.vs_s, "phi_c": W.C7.phi_c, "value": p["mlups"],
                "unit": "MLUPS", "ms_per_step": p["ms_per_step"],
                "phase_ms_per_step": p["phase_ms_per_step"], "step_alg_gbs": p["step_alg_gbs"]}
        print(f"[bench] {W.C7.name}: {p['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    prec = None
    if not args.no_precision:
        prec = run_precision(args.precision_steps)
        last = prec["l2_rel"][str(prec["steps"][-1])]
        print(f"[bench] fp32 vs fp64 after {prec['steps'][-1]} steps: u {last['u']:.2e}, "
              f"C {last['c']:.2e}, deposit {last['deposit']:.2e}", file=sys.stderr, flush=True)
    prec_orc = None
    if args.precision_oracle > 0:
        prec_orc = run_precision_oracle(args.precision_oracle)
        print(f"[bench] fp32/fp64 vs oracle after {args.precision_oracle} steps: "
              f"{json.dumps(prec_orc['l2_rel'])}", file=sys.stderr, flush=True)
    prec3 = None
    if args.precision_3d > 0:
        prec3 = run_precision(args.precision_3d, marks=(500, 1000, 2000), wl=W.C3)
        last = prec3["l2_rel"][str(prec3["steps"][-1])]
        print(f"[bench] 3d fp32 vs fp64 after {prec3['steps'][-1]} steps: u {last['u']:.2e}, "
              f"C {last['c']:.2e}, deposit {last['deposit']:.2e}", file=sys.stderr, flush=True)
    copy = calibrate_copy() if (args.calibrate_copy or not args.no_copy) else None
    if copy:
        # the achievable-bandwidth reference: a plain copy of known size on
        # this device (the roofline's peak stays the vendor figure)
        res["roofline"]["copy_gbs"] = copy["gbs"]
        res["roofline"]["frac_of_copy"] = res["roofline"]["achieved"] / copy["gbs"]
        cs = res["roofline"]["kernels"]["collide_stream"]
        cs["frac_of_copy"] = cs["achieved"] / copy["gbs"]
    cpu = None
    if not args.no_cpu_baseline:
        cpu = (cpu_baseline(base_wl, nz_crop=128, ny_crop=0, steps=20, one_thread=(32, 0, 4))
               if base_wl.dim == 3
               else cpu_baseline(base_wl, nz_crop=0, ny_crop=2048, steps=40,
                                 one_thread=(0, 256, 8)))
        print(f"[bench] cpu baseline: {cpu['value']:.2f} MLUPS on {cpu['cores']} cores, "
              f"{cpu.get('one_thread', {}).get('value', float('nan')):.2f} MLUPS on one",
              file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": res["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if main_wl.precision == "fp32_shifted" else "f64",
        "data": "synthetic (seeded two-layer initial state, fluid at rest)",
        "config": {"workload": main_wl.name, "lattice": f"D{main_wl.dim}Q{main_wl.q}",
                   "grid": [main_wl.nx, main_wl.ny, main_wl.nz], "cells": main_wl.cells,
                   "precision": main_wl.precision, "scheme": "WENO5-JS + TVD-RK3",
                   "parallelism": "single GPU"},
        "timing": ("value and ms_per_step: K steps with no instrumentation; phase times and the "
                   "roofline kernel duration: a second pass of K steps with the library's HIP "
                   "events around every launch (ms_per_step_with_phase_events)"),
        "ms_per_step_with_phase_events": res["ms_per_step_with_phase_events"],
        "phase_ms_per_step": res["phase_ms_per_step"],
        "step_alg_gbs": res["step_alg_gbs"],
        "roofline": res["roofline"],
        "diagnostics": res["diagnostics"],
        "cpu_baseline": cpu,
        "also": also,
        "sweep": sweep,
        "adjoint": adj,
        "fp32_vs_fp64": prec,
        "fp32_vs_fp64_3d": prec3,
        "fp32_vs_oracle": prec_orc,
        "size_classes": poly,
        "full_force": full,
        "copy_calibration": copy,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
