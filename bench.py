"""Throughput benchmark of the multi-channel Lenia step on one MI355X.

Default workload: a 4096 x 4096 torus, 3 channels, 15 kernels (R = 12, 1-3
ring shells), localized m/s/h genes with diffusion and alpha masking, 2000
blobs each carrying its own genotype (seeded synthetic input).  A step is one
full update of (A, P) through lenia_step; inputs are resident in HBM before
the timed region.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
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

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = 384        # read A 12 + write A 12 + read P 180 + write P 180 (FP32)
STEP_SRC = os.path.join(ROOT, "paper_2304_05639_amd", "csrc", "lenia_step.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_4096.json")


def kernel_sha() -> str:
    with open(STEP_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(cells: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if absent or taken on another version of the step kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha() or t.get("cells") != cells:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(world, budget_s: float = 12.0):
    """The FP64 oracle, as it stands, on a 1024 x 1024 crop of the same world
    (treated as its own torus), stepping until the time budget is spent."""
    import numpy as np
    from oracle import oracle as O
    n = 1024
    A = np.ascontiguousarray(world.A[:, :n, :n])
    P = np.ascontiguousarray(world.P[:, :, :n, :n])
    d = O.Desc(n, n, 3, 15, world.src, world.dst, world.R, world.n_shells, world.beta,
               world.dt, 1, 1)
    steps = 0
    t0 = time.perf_counter()
    while True:
        r = O.step(d, A, P)
        A, P = r["A"], r["P"]
        steps += 1
        if time.perf_counter() - t0 >= budget_s or steps >= 8:
            break
    dt = time.perf_counter() - t0
    return {"value": n * n * steps / dt, "unit": "cell-updates/s", "cores": O.threads(),
            "kind": "oracle",
            "sample": f"{steps} step(s) of a {n}x{n} crop of the 4096^2 workload (FP64 direct "
                      f"convolution, OpenMP over rows), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", type=str, default="")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (--gpus {args.gpus} requested); "
              "the path shards by domain decomposition, which is designed but not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_05639_amd import inputs, lenia

    world = inputs.config3()
    cells = world.H * world.W
    tile = tuple(int(x) for x in args.tile.split("x")) if args.tile else None
    plan = lenia.Plan(world, tile=tile)
    info = plan.info()
    dev = torch.device("cuda", 0)
    A = torch.tensor(world.A, device=dev)
    P = torch.tensor(world.P, device=dev)
    A2, P2 = torch.empty_like(A), torch.empty_like(P)
    stream = torch.cuda.current_stream()

    # warm-up, then exactly K steps in one timed region (one kernel launch per
    # step on `stream`, ping-ponging through the plan's workspace)
    plan.step(A, P, A2, P2, n_steps=args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    plan.step(A2, P2, A, P, n_steps=args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = gpu_ms / args.steps
    value = cells * args.steps / (gpu_ms / 1e3)

    achieved = BYTES_PER_CELL * cells / (ms_per_step / 1e3) / 1e9
    traffic = measured_traffic(cells)
    out = {
        "metric": "cell-updates/s (cells x steps / s) at 4096^2, 3 channels, 15 kernels",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lenia-3ch15k-4096x4096-localized-genes-2000-blobs",
                   "world": [world.H, world.W], "channels": 3, "kernels": 15, "R": world.R,
                   "dt": world.dt, "tile": [info.tile_y, info.tile_x], "conv": "direct_f32",
                   "wall_s": wall},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic},
    }
    del A2, P2
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(world)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
