"""Benchmark of the binary Shan-Chen capillary step on one MI355X.

Workload: the roofline-scale capillary, a 16384 x 1024 box with walls over the central half
(x in [4096, 12288)), G = 0.9, G_w = (-0.2, +0.2), tau = (1, 1), FP32 state, seeded synthetic
initial fields.  One step = one pass of the whole hot path (pull streaming with bounce-back,
densities, bulk and wall forces, common velocity, shifted equilibrium, BGK collision, store)
over every node.  The metric is MLUPS (million lattice-node updates per second, both
components); the roofline object prices the fused step kernel against HBM bandwidth with the
algorithmic traffic of 144 bytes per node update (2 components x 9 populations x 4 bytes, read
once and written once).

Prints ONE JSON line.  Options: --steps K (timed), --warmup W, --gpus N (only 1 is supported),
--variant fused|two_kernel, --no-cpu-baseline, --calibrate-copy (runs only a plain copy kernel,
for counter calibration under rocprofv3), --tile BX CY ORDER (skip the autotuner).
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

METRIC = "D2Q9 binary-SC MLUPS & % HBM peak; batched sweep vs surrogate at fixed z error"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = {"fused": 144, "two_kernel": 232}
KERNEL_SRC = os.path.join(ROOT, "paper_0807_0602_amd", "csrc", "scf_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_fused_capillary_16384x1024_traffic.json")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(cells: int):
    """HBM bytes per launch of the fused step from the committed counter summary, or None if
    the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash() or t.get("cells") != cells:
        return None
    return t.get("bytes_per_launch")


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
    return {"value": round(cells * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": oracle.lib().orc_threads(),
            "kind": "oracle",
            "sample": f"{steps} whole-box FP64 steps of the {case.geom.nx}x{case.geom.ny} capillary "
                      f"({cells * steps / 1e6:.0f} M node updates, {dt:.1f} s)"}


def calibrate_copy(nbytes: int = 1 << 30, reps: int = 5) -> None:
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": nbytes, "reps": reps}), flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--variant", choices=["fused", "two_kernel"], default="fused")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--tile", type=int, nargs=3, default=None, metavar=("BX", "CY", "ORDER"))
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU; multi-GPU runs are not part of this build "
              "(the channel would be split into x-slabs with a halo exchange per step).",
              file=sys.stderr, flush=True)
        return 2

    import torch
    if args.calibrate_copy:
        calibrate_copy()
        return 0

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
        ch.set_tile(args.tile[0], args.tile[1], 64, args.tile[2])
    else:
        ch.autotune(20)
    tile = ch.tile()
    ch.set_variant(variant)
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
    step_s = ev_ms / 1e3 / args.steps          # one kernel launch per fused step
    bpl = BYTES_PER_LUP[args.variant]
    achieved = bpl * cells / step_s / 1e9
    traffic = measured_traffic(cells) if args.variant == "fused" else None
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
                     "kernel": "k_step_fused" if args.variant == "fused" else "k_density+k_collide",
                     "bytes_per_node_update": bpl, "event_ms_per_step": round(step_s * 1e3, 5)},
        "health": {"flags": obs["flags"], "z": obs["z"], "mass": list(obs["mass"])},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
