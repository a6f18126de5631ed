"""Benchmark of the binary Shan-Chen capillary step on one MI355X.

Workload: the roofline-scale capillary, a 16384 x 1024 box with walls over the central half
(x in [4096, 12288)), G = 0.9, G_w = (-0.2, +0.2), tau = (1, 1), FP32 state, seeded synthetic
initial fields.  One step = one pass of the whole hot path (pull streaming with bounce-back,
densities, bulk and wall forces, common velocity, shifted equilibrium, BGK collision, store)
over every node.  The metric is MLUPS (million lattice-node updates per second, both
components); the roofline object prices the dominant kernel against HBM bandwidth with its
algorithmic traffic per launch: 144 bytes per node (2 components x 9 populations x 4 bytes, read
once and written once) whether the launch advances one time step or two (temporal blocking keeps
the intermediate populations on chip).  `single_step_equiv_gbs` gives the same launch priced at
144 bytes per node update, the bandwidth a one-step-per-launch kernel would need for the same
MLUPS (it can pass the HBM peak).

The default line also carries two sub-objects measured in the same run: `sweep`, the batched
calibration sweep (64 channels of the sweep_64_channels draws, 50 000 steps each, samples every
100 steps; points per hour, stable points per hour, aggregate MLUPS), and `surrogate`, the learned
surrogate scored on the same 64 trajectories (points per hour of inference against the LBM's,
the fraction of channels within 1 lattice unit of the LBM front and the largest error).

Prints ONE JSON line.  Options: --steps K (timed), --warmup W, --gpus N (only 1 is supported),
--variant fused|two_kernel, --no-cpu-baseline, --calibrate-copy (runs only a plain copy kernel,
for counter calibration under rocprofv3), --tile BX CY ORDER [FUSE] (skip the autotuner; FUSE 2
runs two time steps per launch), --cy3 N (duct3d: rows of y per tile, 0 = two kernels),
--summarize-counters (fold rocprofv3 FETCH_SIZE / WRITE_SIZE CSVs into the committed traffic
summaries), --no-sweep (skip the sweep and surrogate sub-objects).  `traffic` gives the measured
HBM bytes per launch from the committed counter summary of the same kernel source, and
`traffic_frac` the measured rate over the peak.

Further workloads (--workload): small (the 200 x 24 parity capillary, microseconds per step for
direct and graph launches and the oracle on the whole run), washburn (MLUPS on the 4096 x 202
capillary), duct3d (MLUPS of the 3-D D3Q19 duct, 512 x 182 x 182).

--workload surrogate measures the learned surrogate against the batched LBM on 64 fresh
channels drawn like its training set (seed 3): the LBM simulates them (points/hour of the LBM)
and scores the network's curves (max |z_surrogate - z_LBM| per channel, lattice units); the
network's points/hour come from timed inference of the same curves.

--workload sweep measures the batched calibration sweep instead: 64 channels with H in
{20, 40, 80, 160}, L in {512, ..., 4096}, G_wA uniform in [-0.3, 0.3] (G_wB = -G_wA) and a
viscosity-ratio tau pair, advanced together (one launch per step or per two steps over all their
tiles, HIP graphs of 100 steps plus the recorded observation), 50 000 steps with z(t) and the precursor
recorded every 100 steps.  The value is sweep points per hour (one point = one channel's whole
trajectory).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from typing import Optional

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D2Q9 binary-SC MLUPS & % HBM peak; batched sweep vs surrogate at fixed z error"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = {"fused": 144, "two_kernel": 232}
KERNEL_SRC = os.path.join(ROOT, "paper_0807_0602_amd", "csrc", "scf_kernels.hip")
# the tile planner (strip widths, band heights) lives in the runtime: counters go stale with it too
RUNTIME_SRC = os.path.join(ROOT, "paper_0807_0602_amd", "csrc", "scf_runtime.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_fused_capillary_16384x1024_traffic.json")
KERNEL3_SRC = os.path.join(ROOT, "paper_0807_0602_amd", "csrc", "scf3d_kernels.hip")
TRAFFIC3_FILE = os.path.join(ROOT, "profiles", "k3_fused_duct3d_512x182x182_traffic.json")
DUCT3D = (512, 182, 182, 128, 384)   # nx, ny, nz, x0, x1 of the 3-D duct workload


def kernel_hash(src: Optional[str] = None) -> str:
    """First 16 hex digits of the sha256 of the kernel source (the 2-D kernels together with the
    runtime that plans their tiles, by default)."""
    h = hashlib.sha256()
    for p in ([src] if src else [KERNEL_SRC, RUNTIME_SRC]):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(cells: int, schedule: dict, path: Optional[str] = None, src: Optional[str] = None,
                     keys=("bx", "cy", "order", "fuse")):
    """HBM bytes per launch of a fused step from the committed counter summary for this
    schedule (the 2-D capillary's file by default), or None if the kernel source (for the 2-D
    capillary: the kernels and the runtime that plans their tiles) changed since the counters
    were taken."""
    path = path or TRAFFIC_FILE
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash(src) or t.get("cells") != cells:
        return None
    for e in t.get("schedules", []):
        if all(e["schedule"].get(k, 1 if k == "fuse" else None) == schedule.get(k, 1 if k == "fuse" else None)
               for k in keys):
            return e["bytes_per_launch"]
    return None


def kernel_name(fuse: int) -> str:
    return "k_step_fused2" if fuse == 2 else "k_step_fused"


def parse_tile(vals):
    """--tile BX CY ORDER [FUSE] -> (bx, cy, order, fuse)."""
    if vals is None:
        return None
    if len(vals) not in (3, 4):
        raise SystemExit("--tile takes BX CY ORDER [FUSE]")
    return (vals[0], vals[1], vals[2], vals[3] if len(vals) == 4 else 1)


def _counter_mean(path: str, kernel: str, counter: str) -> float:
    import csv
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        raise SystemExit(f"no {counter} rows for {kernel} in {path}")
    return sum(vals) / len(vals)


def summarize_counters(args) -> int:
    """Fold rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE CSVs of the fused step and of the 1 GiB
    calibration copy into TRAFFIC_FILE (one entry per schedule).  Each counter is scaled by
    (bytes the copy kernel moves) / (what the counter reads for it)."""
    fetch, write, fetch_copy, write_copy = args.summarize_counters
    if args.workload == "duct3d":
        if args.cy3 < 1:
            raise SystemExit("counter summaries of the 3-D duct cover the fused step (--cy3 >= 1)")
        kname, path, src, label = "k3_fused<", TRAFFIC3_FILE, KERNEL3_SRC, "k3_fused"
        nx, ny, nz = DUCT3D[:3]
        cells, workload = nx * ny * nz, "duct3d_%dx%dx%d" % (nx, ny, nz)
        sched = {"cy": min(args.cy3, ny)}
    else:
        path, src, label = TRAFFIC_FILE, None, "k_step_fused / k_step_fused2"
        from paper_0807_0602_amd import inputs
        case = inputs.capillary_roofline(seed=1)
        cells, workload = case.geom.nx * case.geom.ny, case.name
        if getattr(args, "variant", "fused") == "two_kernel":
            # one step = one k_density and one k_collide launch
            kname, sched = ("k_density(", "k_collide("), {"variant": "two_kernel"}
        else:
            if not args.tile:
                raise SystemExit("--summarize-counters needs --tile BX CY ORDER")
            bx, cy, order, fuse = args.tile
            kname = kernel_name(fuse) + "<"    # template instantiations only (not the other kernel)
            sched = {"bx": bx, "cy": cy, "order": order, "fuse": fuse}
    copy_kib = (1 << 30) / 1024.0
    f_scale = copy_kib / _counter_mean(fetch_copy, "copyBuffer", "FETCH_SIZE")
    w_scale = copy_kib / _counter_mean(write_copy, "copyBuffer", "WRITE_SIZE")
    knames = kname if isinstance(kname, tuple) else (kname,)
    rd = sum(_counter_mean(fetch, k, "FETCH_SIZE") for k in knames) * f_scale * 1024.0
    wr = sum(_counter_mean(write, k, "WRITE_SIZE") for k in knames) * w_scale * 1024.0
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        t = {}
    if t.get("kernel_sha256_16") != kernel_hash(src) or t.get("cells") != cells:
        t = {"kernel": label, "workload": workload, "cells": cells,
             "kernel_sha256_16": kernel_hash(src), "schedules": []}
    t["schedules"] = [e for e in t["schedules"] if e["schedule"] != sched]
    t["schedules"].append({"schedule": sched, "read_bytes_per_launch": round(rd),
                           "write_bytes_per_launch": round(wr), "bytes_per_launch": round(rd + wr),
                           "read_bytes_per_node": round(rd / cells, 2), "write_bytes_per_node": round(wr / cells, 2),
                           "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)})
    with open(path, "w") as f:
        json.dump(t, f, indent=1)
    print(json.dumps(t["schedules"][-1]))
    return 0


def cpu_baseline(case, budget_s: float = 12.0, max_steps: int = 40) -> dict:
    """The FP64 oracle as it stands on the host cores, on the same workload: whole-box steps
    until the time budget is spent."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    oracle.set_threads(threads)
    o = oracle.Oracle.from_case(case).init(*case.fields())
    o.step(1)   # first touch of the arrays
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps and time.perf_counter() - t0 < budget_s:
        o.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    cells = case.geom.nx * case.geom.ny
    cores = oracle.lib().orc_threads()
    # one thread, two steps, for the single-core rate
    oracle.set_threads(1)
    t1 = time.perf_counter()
    o.step(2)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    return {"value": round(cells * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps} whole-box FP64 steps of the {case.geom.nx}x{case.geom.ny} capillary "
                      f"({cells * steps / 1e6:.0f} M node updates, {dt:.1f} s)",
            "single_thread_mlups": round(2 * cells / dt1 / 1e6, 3),
            "host": _host_cpu()}


def _host_cpu() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def calibrate_copy(nbytes: int = 1 << 30, reps: int = 5) -> None:
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": nbytes, "reps": reps}), flush=True)


def run_sweep(steps: int, tile=None, every: int = 100) -> dict:
    """The batched calibration sweep (sweep_64_channels draws, seed 0) for `steps` steps with
    z(t) and the precursor recorded every `every` steps; autotuned unless `tile` is given.
    Returns the timing, the schedule, the cases and the trajectories [n, samples, 5] (t, z,
    precursor, flags, unstable-so-far)."""
    import numpy as np
    import torch
    from paper_0807_0602_amd import inputs
    from paper_0807_0602_amd.scf import Batch

    cases = inputs.sweep_draws(64, seed=0, steps=steps, sample_every=every)
    cells = sum(c.geom.nx * c.geom.ny for c in cases)
    stream = torch.cuda.current_stream()
    b = Batch(cases, sample_every=every, max_samples=steps // every + 1, stream=stream)
    if tile:
        bx, cy, order, fuse = tile
        b.set_tile(bx, cy, every, order, fuse)
    else:
        b.autotune(5)
        t = b.tile()
        b.set_tile(t["bx"], t["cy"], every, t["order"], t["fuse"])
    sched = b.tile()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    recs, ns = b.observe(allow_unstable=True)
    b.close()
    del b
    torch.cuda.empty_cache()
    traj = np.full((len(cases), ns, 5), np.nan)
    for c, r in enumerate(recs):
        bad = False
        for k, x in enumerate(r):
            bad = bad or bool(x["flags"] & 2)
            traj[c, k] = (x["t"], x["z"], x["precursor"], x["flags"], float(bad))
    unstable = int(sum(1 for r in recs if any(x["flags"] & 2 for x in r)))
    return {"cases": cases, "traj": traj, "cells": cells, "wall": wall, "samples": ns,
            "event_step_s": e0.elapsed_time(e1) / 1e3 / steps, "schedule": sched, "unstable": unstable}


def score_surrogate(weights: str, cases, traj, lbm_wall: float, reps: int = 20) -> dict:
    """The learned surrogate on the sweep's own channels: per-channel max |z_surrogate - z_LBM| in
    lattice units over the LBM's samples (up to a channel's instability flag), and the network's
    points per hour from timed inference of the same curves."""
    import numpy as np
    import torch
    from paper_0807_0602_amd import surrogate as S

    net = S.Network.load(weights)
    wl = net.cfg.d_in == 5
    errs, inside = S.curve_errors(net, cases, traj, wl)
    X, _, _, keep = S.dataset(cases, traj, wl)
    _, in_hull = net.predict(X)           # also the warm-up
    ns = traj.shape[1]
    # channels with any kept query outside the training box: answered by the LBM
    fallback = sum(1 for c in range(len(cases)) if not in_hull[c * ns:(c + 1) * ns][keep[c * ns:(c + 1) * ns]].all())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.predict(X)
    sur_s = (time.perf_counter() - t0) / reps
    net.close()
    ok = np.isfinite(errs[:, 0])
    within = float(np.mean(errs[ok, 0] <= 1.0)) if ok.any() else 0.0
    sur_pph = len(cases) * 3600.0 / sur_s
    lbm_pph = len(cases) * 3600.0 / lbm_wall
    # one-off cost of the network (LBM data and training, GPU seconds, stored with the weights) and
    # the number of answered curves after which it has cost less than the LBM would have
    z = np.load(weights)
    info = json.loads(str(z["info"])) if "info" in z.files else {}
    train_s, data_s = info.get("seconds"), info.get("data_seconds")
    cost = {"training_seconds": train_s, "data_seconds": data_s, "break_even_points": None}
    if train_s is not None and data_s is not None:
        cost["break_even_points"] = round((train_s + data_s) / 3600.0 / (1.0 / lbm_pph - 1.0 / sur_pph), 1)
    return {"inputs": int(net.cfg.d_in), "surrogate_points_per_hour": round(sur_pph, 1),
            "lbm_points_per_hour": round(lbm_pph, 1), "speedup": round(sur_pph / lbm_pph, 1),
            "scored_channels": int(ok.sum()), "fraction_within_1lu": round(within, 4),
            "points_per_hour_within_1lu": round(sur_pph * within, 1),
            "max_dz_lu": round(float(np.nanmax(errs[:, 0])), 4),
            "median_max_dz_lu": round(float(np.nanmedian(errs[:, 0])), 4),
            "inside_training_hull": round(inside, 4), "fallback_channels": int(fallback),
            "samples_per_point": int(traj.shape[1]), **cost}


def sweep_summary(sw: dict, steps: int) -> dict:
    n = len(sw["cases"])
    return {"channels": n, "steps": steps, "nodes": sw["cells"], "sample_every": 100,
            "points_per_hour": round(n * 3600.0 / sw["wall"], 1),
            "stable_points_per_hour": round((n - sw["unstable"]) * 3600.0 / sw["wall"], 1),
            "unstable_channels": sw["unstable"], "wall_s": round(sw["wall"], 3),
            "aggregate_mlups": round(sw["cells"] * steps / sw["wall"] / 1e6, 1),
            "schedule": sw["schedule"]}


def sweep(args) -> int:
    steps = args.steps if args.steps != 10000 else 50_000
    sw = run_sweep(steps, args.tile)
    cells, tile = sw["cells"], sw["schedule"]
    step_s = sw["event_step_s"]
    launch_s = step_s * tile["fuse"]
    # algorithmic bytes of one launch: 144 B per node (one read and one write of both population
    # sets), whether it advances one step or two
    achieved = 144 * cells / launch_s / 1e9
    summ = sweep_summary(sw, steps)
    line = {
        "metric": "calibration-sweep points/hour, batched LBM (one point = one channel trajectory)",
        "value": summ["points_per_hour"], "unit": "points/h", "n_gpus": 1,
        "stable_points_per_hour": summ["stable_points_per_hour"],
        "steps": steps, "warmup": 0, "ms_per_step": round(sw["wall"] * 1e3 / steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sweep_64_channels", "channels": len(sw["cases"]), "nodes": cells,
                   "sample_every": 100, "samples_recorded": sw["samples"], "schedule": tile,
                   "aggregate_mlups": summ["aggregate_mlups"], "unstable_channels": sw["unstable"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": kernel_name(tile["fuse"]) + " (all channels per launch) + observation every 100 steps",
                     "bytes_per_node_per_launch": 144, "steps_per_launch": tile["fuse"],
                     "single_step_equiv_gbs": round(144 * cells / step_s / 1e9, 1)},
    }
    print(json.dumps(line), flush=True)
    return 0


def surrogate_gain(args) -> int:
    """The surrogate against the batched LBM on 64 fresh channels drawn like its training set."""
    import torch
    from paper_0807_0602_amd import surrogate as S

    steps = args.steps if args.steps != 10000 else 50_000
    every = 100
    cases = S.draw_cases(64, seed=3, steps=steps, every=every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    traj = S.simulate(cases, steps, every)
    torch.cuda.synchronize()
    lbm_s = time.perf_counter() - t0
    sc = score_surrogate(args.weights, cases, traj, lbm_s)
    line = {
        "metric": "calibration-sweep points/hour: learned surrogate vs batched LBM (one point = one channel's z(t), p(t))",
        "value": sc["surrogate_points_per_hour"], "unit": "points/h", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 MFMA / f32 accumulate (network), f32 (LBM)", "data": "synthetic",
        "config": {"workload": "surrogate_vs_lbm_64_channels", **sc},
    }
    print(json.dumps(line), flush=True)
    return 0


def duct3d(args) -> int:
    """MLUPS of the three-dimensional (D3Q19) duct capillary: 512 x 182 x 182 nodes (17.0 M),
    walls on y and z over the middle half of x; the fused one-kernel step by default (--cy3 rows
    of y per tile), the two-kernel step with --cy3 0."""
    import numpy as np
    import torch
    from paper_0807_0602_amd import inputs
    from paper_0807_0602_amd.scf import Channel3

    nx, ny, nz, x0, x1 = DUCT3D
    steps = args.steps if args.steps != 10000 else 1000
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    liq = X < x0
    a = np.where(liq, 2.0, 0.06) + 1e-3 * inputs.uniform_pm1(1, 0, Y * nz + Z, X)
    b = np.where(liq, 0.06, 2.0) + 1e-3 * inputs.uniform_pm1(1, 1, Y * nz + Z, X)
    del Z, Y, X, liq
    stream = torch.cuda.current_stream()
    ch = Channel3(nx, ny, nz, x0, x1, inputs.Params(G=0.9, gw=(-0.2, 0.2)), a, b, walls_y=True, walls_z=True,
                  stream=stream)
    del a, b
    fused = args.cy3 > 0
    ch.set_schedule(fused=fused, cy=max(args.cy3, 1))
    ch.step(min(args.warmup, 50))
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    ch.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    obs = ch.observe(allow_unstable=True)
    cells = nx * ny * nz
    step_s = e0.elapsed_time(e1) / 1e3 / steps
    # algorithmic bytes per node update: the fused step pulls 2 x 19 FP32 populations once
    # (152 B) and stores as many (152 B); the two-kernel step pulls twice (304 B), writes and
    # reads the density field once (16 B) and stores 152 B
    bpl = 304 if fused else 472
    achieved = bpl * cells / step_s / 1e9
    sched = ch.schedule()
    traffic = measured_traffic(cells, {"cy": sched["cy"]}, TRAFFIC3_FILE, KERNEL3_SRC, ("cy",)) if fused else None
    line = {
        "metric": "D3Q19 binary-SC MLUPS (3-D duct capillary)", "value": round(cells * steps / wall / 1e6, 1),
        "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 50),
        "ms_per_step": round(wall * 1e3 / steps, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "duct3d_512x182x182", "nx": nx, "ny": ny, "nz": nz, "channel_x": [x0, x1],
                   "G": 0.9, "gw": [-0.2, 0.2], "tau": [1.0, 1.0], "nodes": cells},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_gbs": round(traffic / step_s / 1e9, 1) if traffic else None,
                     "traffic_frac": round(traffic / step_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                     "kernel": ("k3_fused, %d rows of y per 64 x 4 tile" % sched["cy"]) if fused
                     else "k3_density + k3_collide", "bytes_per_node_update": bpl,
                     "event_ms_per_step": round(step_s * 1e3, 5)},
        "health": {"flags": obs["flags"], "z": obs["z"], "mass": list(obs["mass"])},
    }
    print(json.dumps(line), flush=True)
    return 0


def small(args) -> int:
    """The 200 x 24 parity capillary (4 800 nodes): launch-latency bound, so microseconds per step
    for direct launches and for captured graphs, one and two steps per launch, and the FP64
    oracle on the whole 2000-step run."""
    import torch
    import oracle
    from paper_0807_0602_amd import inputs
    from paper_0807_0602_amd.scf import Channel

    case = inputs.capillary_small(seed=1)
    steps = 2000
    out = {}
    stream = torch.cuda.current_stream()
    probe = Channel.from_case(case, stream=stream)
    tuned = probe.autotune(50)
    probe.close()
    out["schedule"] = tuned
    for fuse in (1, 2):
        for gs, name in ((0, "eager"), (200, "graph")):
            ch = Channel.from_case(case, stream=stream)
            ch.set_tile(tuned["bx"], tuned["cy"], gs, tuned["order"], fuse)
            ch.step(200)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ch.step(steps)
            torch.cuda.synchronize()
            out[f"{name}_fuse{fuse}_us_per_step"] = round((time.perf_counter() - t0) * 1e6 / steps, 2)
            ch.close()
    oracle.set_threads(1)
    o = oracle.Oracle.from_case(case).init(*case.fields())
    t0 = time.perf_counter()
    o.step(steps)
    dto = time.perf_counter() - t0
    cells = case.geom.nx * case.geom.ny
    timings = {k: v for k, v in out.items() if k.endswith("_us_per_step")}
    best_key = min(timings, key=timings.get)
    best = timings[best_key]
    # the autotuned tile shape is shared by the four runs; `best` names the launch mode and the
    # steps per launch of the reported value
    out["best"] = best_key[: -len("_us_per_step")]
    line = {"metric": "microseconds per step, 200 x 24 capillary (launch-latency bound)", "value": best,
            "unit": "us/step", "n_gpus": 1, "steps": steps, "warmup": 200, "ms_per_step": best / 1e3,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": {"workload": "capillary_200x24", "nodes": cells, **out},
            "cpu_baseline": {"value": round(cells * steps / dto / 1e6, 3), "unit": "MLUPS", "cores": 1,
                             "kind": "oracle", "sample": f"the whole 2000-step run ({dto:.2f} s)"}}
    print(json.dumps(line), flush=True)
    return 0


def washburn(args) -> int:
    """MLUPS on the 4096 x 202 Washburn capillary (H = 200, capillary length 3072), autotuned."""
    import torch
    from paper_0807_0602_amd import inputs
    from paper_0807_0602_amd.scf import Channel

    case = inputs.with_params(inputs.capillary_washburn(seed=1), tau=(1.25, 1.0))
    steps = args.steps if args.steps != 10000 else 20000
    stream = torch.cuda.current_stream()
    ch = Channel.from_case(case, stream=stream)
    ch.autotune(20)
    tile = ch.tile()
    ch.step(min(args.warmup, 200))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    obs = ch.observe(allow_unstable=True)
    cells = case.geom.nx * case.geom.ny
    line = {"metric": "D2Q9 binary-SC MLUPS (Washburn capillary)", "value": round(cells * steps / wall / 1e6, 1),
            "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 200),
            "ms_per_step": round(wall * 1e3 / steps, 5), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": case.name, "nx": case.geom.nx, "ny": case.geom.ny, "tau": list(case.params.tau),
                       "gw": list(case.params.gw), "schedule": tile, "nodes": cells},
            "health": {"flags": obs["flags"], "z": obs["z"]}}
    print(json.dumps(line), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--variant", choices=["fused", "two_kernel"], default="fused")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="roofline workload: leave out the sweep and surrogate sub-objects")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--tile", type=int, nargs="+", default=None, metavar="N",
                    help="BX CY ORDER [FUSE]: fixed schedule instead of the autotuner")
    ap.add_argument("--workload", choices=["roofline", "sweep", "surrogate", "duct3d", "small", "washburn"],
                    default="roofline")
    ap.add_argument("--cy3", type=int, default=16,
                    help="duct3d: rows of y per tile of the fused 3-D step; 0 = the two-kernel step")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_0807_0602_amd", "surrogate_weights_5in.npz"))
    ap.add_argument("--summarize-counters", nargs=4, default=None,
                    metavar=("FETCH_CSV", "WRITE_CSV", "FETCH_COPY_CSV", "WRITE_COPY_CSV"),
                    help="write the traffic summary for the schedule given by --tile and exit")
    args = ap.parse_args()
    args.tile = parse_tile(args.tile)
    if args.summarize_counters:
        return summarize_counters(args)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (a channel "
              "would be split into x-slabs with a halo exchange per step or pass).",
              file=sys.stderr, flush=True)
        return 2

    import torch
    if args.calibrate_copy:
        calibrate_copy()
        return 0
    if args.workload == "sweep":
        return sweep(args)
    if args.workload == "surrogate":
        return surrogate_gain(args)
    if args.workload == "duct3d":
        return duct3d(args)
    if args.workload == "small":
        return small(args)
    if args.workload == "washburn":
        return washburn(args)

    from paper_0807_0602_amd import _lib as L
    from paper_0807_0602_amd import inputs
    from paper_0807_0602_amd.scf import Channel

    case = inputs.capillary_roofline(seed=1)
    g = case.geom
    cells = g.nx * g.ny
    stream = torch.cuda.current_stream()
    ch = Channel.from_case(case, stream=stream)
    variant = L.SCF_VARIANT_FUSED if args.variant == "fused" else L.SCF_VARIANT_TWO_KERNEL
    if args.tile:
        bx, cy, order, fuse = args.tile
        ch.set_tile(bx, cy, 64, order, fuse)
    else:
        ch.autotune(20)
    tile = ch.tile()
    ch.set_variant(variant)
    fuse = tile["fuse"] if args.variant == "fused" else 1
    ch.step(args.warmup)
    torch.cuda.synchronize()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    ch.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    obs = ch.observe(allow_unstable=True)

    mlups = cells * args.steps / wall / 1e6
    step_s = ev_ms / 1e3 / args.steps
    launch_s = step_s * fuse                   # one launch advances `fuse` steps
    bpl = BYTES_PER_LUP[args.variant]
    # algorithmic bytes of one launch: 144 B per node for the fused kernels (one read and one
    # write of both population sets, for one step or two), 232 B per node for the two-kernel step
    achieved = bpl * cells / launch_s / 1e9
    single_equiv = bpl * cells * fuse / launch_s / 1e9
    if args.variant == "fused":
        traffic = measured_traffic(cells, tile)
    else:
        traffic = measured_traffic(cells, {"variant": "two_kernel"}, keys=("variant",))
    line = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": case.name, "nx": g.nx, "ny": g.ny, "channel_x": [g.x0, g.x1],
                   "G": case.params.G, "gw": list(case.params.gw), "tau": list(case.params.tau),
                   "variant": args.variant, "schedule": tile, "nodes": cells},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kernel_name(fuse) if args.variant == "fused" else "k_density+k_collide",
                     "bytes_per_node_per_launch": bpl, "steps_per_launch": fuse,
                     "event_ms_per_launch": round(launch_s * 1e3, 5),
                     # the same launch priced per node update (two steps share one read and one
                     # write, so this can pass the HBM peak)
                     "single_step_equiv_gbs": round(single_equiv, 1),
                     "traffic_gbs": round(traffic / launch_s / 1e9, 1) if traffic else None,
                     "traffic_frac": round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None},
        "health": {"flags": obs["flags"], "z": obs["z"], "mass": list(obs["mass"])},
    }
    if not args.no_sweep:
        # the calibration sweep and the surrogate scored on its trajectories (the second half of
        # the metric), after the roofline channel's memory is released
        ch.close()
        del ch
        torch.cuda.empty_cache()
        sw_steps = 50_000
        sw = run_sweep(sw_steps)
        line["sweep"] = sweep_summary(sw, sw_steps)
        line["surrogate"] = score_surrogate(args.weights, sw["cases"], sw["traj"], sw["wall"])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
