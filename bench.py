"""Throughput benchmark of the multi-channel Lenia step on one MI355X.

Default workload: a 4096 x 4096 torus, 3 channels, 15 kernels (R = 12, 1-3
ring shells), localized m/s/h genes with diffusion and alpha masking, 2000
blobs each carrying its own genotype (seeded synthetic input).  A step is one
full update of (A, P) through lenia_step; inputs are resident in HBM before
the timed region.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Secondary legs in the same line: Algorithm 2's operators (walls, mutation,
penalization) around the step, the split DFT forms on MFMA, the adjoint's
backward/forward time ratio, the ring-decomposed kernel form (and, with
--batched, the 256-world batched workload).
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
CSRC = os.path.join(ROOT, "paper_2304_05639_amd", "csrc")
STEP_SRCS = [os.path.join(CSRC, f) for f in ("lenia_step.hip", "lenia_device.h", "lenia_internal.h")]
DFT_SRCS = [os.path.join(CSRC, f) for f in ("lenia_dft.hip", "lenia_device.h", "lenia_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_4096.json")
DFT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_dft_conv_4096.json")
RING_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_ring_step_4096.json")
# ring-decomposed kernels (9 gene types per kernel): read A 12 + write A 12 +
# read P 540 + write P 540 (FP32)
RING_BYTES_PER_CELL = 1104
# the algorithmic counts assume every gene plane is read and written each step;
# the kernels skip gene reads where alpha cannot hold and, within a multi-step
# call, gene writes whose output buffer already holds 0 there, so the counter
# traffic is the HBM figure
ROOFLINE_NOTE = ("achieved counts algorithmic bytes (every gene plane read and written); "
                 "traffic is the HBM bytes measured by counters per launch")


def kernel_sha(srcs=STEP_SRCS) -> str:
    """Hash of a kernel's sources (counters are only valid for them)."""
    h = hashlib.sha256()
    for fn in srcs:
        with open(fn, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(cells: int, path: str = TRAFFIC_FILE, srcs=STEP_SRCS):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None if absent or taken on another version of the kernel."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha(srcs) or t.get("cells") != cells:
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
    # the same oracle on one thread, on a 256 x 256 crop
    m = 256
    A1 = np.ascontiguousarray(world.A[:, :m, :m])
    P1 = np.ascontiguousarray(world.P[:, :, :m, :m])
    d1 = O.Desc(m, m, 3, 15, world.src, world.dst, world.R, world.n_shells, world.beta,
                world.dt, 1, 1)
    O.set_threads(1)
    s1 = 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < 3.0:
        O.step(d1, A1, P1)
        s1 += 1
    dt1 = time.perf_counter() - t1
    O.set_threads(O.threads())
    return {"value": n * n * steps / dt, "unit": "cell-updates/s", "cores": O.threads(),
            "kind": "oracle",
            "sample": f"{steps} step(s) of a {n}x{n} crop of the 4096^2 workload (FP64 direct "
                      f"convolution, OpenMP over rows), {dt:.1f} s",
            "value_1_thread": m * m * s1 / dt1,
            "sample_1_thread": f"{s1} step(s) of a {m}x{m} crop on one thread, {dt1:.1f} s"}


def backward_forward_ratio(steps_T: int = 64, ckpt: int = 8, reps: int = 3, conv: int = 1):
    """256^2 differentiable rollout (T = 64, checkpoint every 8, MSE to a
    random target): time of the backward pass (recomputing each segment with
    saved potentials, then the adjoint) over the forward pass (with checkpoint
    saves), median of `reps`.  `conv` picks the forward's potential form."""
    import torch
    from paper_2304_05639_amd import inputs, lenia
    from paper_2304_05639_amd.autograd import rollout
    w = inputs.config5()
    plan = lenia.Plan(w, conv=conv)
    A0 = torch.tensor(w.A, device="cuda", requires_grad=True)
    P0 = torch.tensor(w.P, device="cuda", requires_grad=True)
    beta = torch.tensor(w.beta, dtype=torch.float32, device="cuda", requires_grad=True)
    target = torch.tensor(w.target, device="cuda")
    fw, bw = [], []
    for _ in range(reps + 1):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record()
        AT, _ = rollout(A0, P0, beta, plan, steps_T, ckpt)
        loss = ((AT - target) ** 2).mean()
        e1.record()
        loss.backward()
        e2.record()
        torch.cuda.synchronize()
        fw.append(e0.elapsed_time(e1))
        bw.append(e1.elapsed_time(e2))
        A0.grad = P0.grad = beta.grad = None
    fw, bw = sorted(fw[1:]), sorted(bw[1:])
    f, b = fw[len(fw) // 2], bw[len(bw) // 2]
    return {"value": b / f, "forward_ms": f, "backward_ms": b,
            "conv": "dft_split_bf16" if conv == lenia.CONV_DFT_SPLIT_BF16 else "direct_f32",
            "workload": "256x256, 3 channels, 15 kernels, T=64, checkpoint every 8, MSE loss"}


def batched_throughput(steps: int = 20, warmup: int = 2):
    """256 independent worlds of sides 128..1024 stepped together in one
    launch per step over the (world, tile) work list (graph replay): cell-updates/s
    over all worlds."""
    import torch
    from paper_2304_05639_amd import inputs, lenia
    worlds = inputs.config4()
    cells = sum(w.H * w.W for w in worlds)
    bp = lenia.BatchedPlan(worlds, autotune=True)
    As = [torch.tensor(w.A, device="cuda") for w in worlds]
    Ps = [torch.tensor(w.P, device="cuda") for w in worlds]
    bp.step(As, Ps, n_steps=warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    bp.step(As, Ps, n_steps=steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    info = bp.info()
    return {"value": cells / (ms / 1e3), "unit": "cell-updates/s", "ms_per_step": ms,
            "cells": cells, "worlds": len(worlds), "tile": [info.tile_y, info.tile_x],
            "roofline_frac_algorithmic": BYTES_PER_CELL * cells / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}


# MFMA instructions (v_mfma_f32_16x16x32_bf16, 16384 flops each) per tile of
# the DFT form: forward transforms 3 channels x (192 + 384), inverse 15 kernels
# x (240 + 108); every product is issued three times (hi*hi, hi*lo, lo*hi).
DFT_MFMA_PER_TILE = 3 * (192 + 384) + 15 * (240 + 108)
MFMA_FLOPS = 16 * 16 * 32 * 2
BF16_PEAK_TFLOPS = 2500.0


def dft_form(world, steps: int = 20, warmup: int = 2, conv: int = 2):
    """A split DFT-as-GEMM form (bf16 or fp16 hi+lo operands) on the same world:
    full-step throughput, and the MFMA kernel alone (lenia_potentials) against
    the dense peak of its operand type (2.5 PFLOP/s for both)."""
    import torch
    from paper_2304_05639_amd import lenia
    plan = lenia.Plan(world, conv=conv)
    V = plan.info().tile_y
    n_tiles = -(-world.H // V) * -(-world.W // V)
    A = torch.tensor(world.A, device="cuda")
    P = torch.tensor(world.P, device="cuda")
    U = torch.empty(world.n_kernels, world.H, world.W, device="cuda")
    for _ in range(warmup):
        plan.potentials(A, U)
    e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        plan.potentials(A, U)
    e1.record()
    A2, P2 = torch.empty_like(A), torch.empty_like(P)
    plan.step(A, P, A2, P2, n_steps=warmup)
    e2.record()
    plan.step(A2, P2, A, P, n_steps=steps)
    e3.record()
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / steps
    s_ms = e2.elapsed_time(e3) / steps
    flops = n_tiles * DFT_MFMA_PER_TILE * MFMA_FLOPS
    achieved = flops / (k_ms / 1e3) / 1e12
    return {"value": world.H * world.W / (s_ms / 1e3), "unit": "cell-updates/s",
            "ms_per_step": s_ms, "mfma_kernel_ms": k_ms,
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / BF16_PEAK_TFLOPS,
                         "traffic": (measured_traffic(world.H * world.W, DFT_TRAFFIC_FILE, DFT_SRCS)
                                     if conv == lenia.CONV_DFT_SPLIT_BF16 else None)},
            "note": f"{n_tiles} tiles of 64x64 (valid {V}x{V}), {DFT_MFMA_PER_TILE} MFMA per tile"}


def oracle_timing(fn, n: int, budget_s: float, what: str):
    """The FP64 oracle as it stands on a bounded sample: calls fn() (one step of
    an n x n crop) until the time budget is spent."""
    from oracle import oracle as O
    steps = 0
    t0 = time.perf_counter()
    while True:
        fn()
        steps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": n * n * steps / dt, "unit": "cell-updates/s", "cores": O.threads(),
            "kind": "oracle", "sample": f"{steps} step(s) of a {n}x{n} crop of {what}, {dt:.1f} s"}


def small_worlds():
    """The 64^2 single-channel world (global genes, one R = 13 kernel) timed as
    latency over 100 steps in one call, and the 512^2 three-channel world as
    throughput over 100 steps (its working set stays in the 256 MB
    Infinity Cache)."""
    import torch
    from paper_2304_05639_amd import inputs, lenia
    out = {}
    for name, w, n in (("c1_64x64_global", inputs.config1(), 100), ("c2_512x512", inputs.config2(), 100)):
        plan = lenia.Plan(w)
        A = torch.tensor(w.A, device="cuda")
        P = torch.tensor(w.P, device="cuda") if w.P is not None else None
        A2 = torch.empty_like(A)
        P2 = torch.empty_like(P) if P is not None else None
        plan.step(A, P, A2, P2, n_steps=10)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        plan.step(A2, P2, A, P, n_steps=n)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        out[name] = {"us_per_step": ms * 1e3, "steps_per_s": 1e3 / ms,
                     "cell_updates_per_s": w.H * w.W / (ms / 1e3), "steps": n}
    return out


def ring_form(steps: int = 20, warmup: int = 10):
    """The 4096^2 workload with ring-decomposed kernels (24 rings, localized
    kernel genes): full-step throughput against the HBM floor of its
    algorithmic bytes."""
    import torch
    from paper_2304_05639_amd import inputs, lenia
    world = inputs.config_ring()
    cells = world.H * world.W
    plan = lenia.Plan(world)
    A = torch.tensor(world.A, device="cuda")
    P = torch.tensor(world.P, device="cuda")
    A2, P2 = torch.empty_like(A), torch.empty_like(P)
    plan.step(A, P, A2, P2, n_steps=warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    plan.step(A2, P2, A, P, n_steps=steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    achieved = RING_BYTES_PER_CELL * cells / (ms / 1e3) / 1e9
    import numpy as np
    from oracle import oracle as O
    n = 256
    Ac = np.ascontiguousarray(world.A[:, :n, :n])
    Pc = np.ascontiguousarray(world.P[:, :, :n, :n])
    dc = O.Desc(n, n, 3, 15, world.src, world.dst, world.R, world.n_shells, world.beta, world.dt,
                1, 1, n_ring=world.n_ring)
    cpu = oracle_timing(lambda: O.ring_step(dc, Ac, Pc), n, 4.0, "the ring-form workload")
    return {"value": cells / (ms / 1e3), "unit": "cell-updates/s", "ms_per_step": ms,
            "cpu_baseline": cpu,
            "steps": steps, "warmup": warmup,
            "workload": "lenia-ring-3ch15k-4096x4096: 24 rings of the R = 12 disk, 9 gene types "
                        "per kernel, 2000 blobs with their own genes",
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "traffic": measured_traffic(cells, RING_TRAFFIC_FILE, STEP_SRCS),
                         "note": ROOFLINE_NOTE}}


# the step's 384 B/cell plus the wall mask read (1), the flags written and read
# twice (3) and the two area masks written and read (4)
EVOLVE_BYTES_PER_CELL = 392


def evolve_form(world, steps: int = 20, warmup: int = 5, r_oxy: int = 6):
    """Algorithm 2's operators around each step of the same world: walls every
    512 rows and columns, mutation (rate 1, squares of side 16) and the
    penalization of exploding patterns (rate 0.2, oxygen radius r_oxy), with
    seeded random draws per step."""
    import numpy as np
    import torch
    from paper_2304_05639_amd import lenia
    H, W = world.H, world.W
    plan = lenia.Plan(world)
    walls = np.zeros((H, W), np.uint8)
    walls[::512, :] = 1
    walls[:, ::512] = 1
    wt = torch.tensor(walls, device="cuda")
    rng = np.random.default_rng(2304056390 + 7)
    events = []
    for _ in range(warmup + steps):
        p = int(rng.integers(2))
        events.append(dict(mut_p=int(rng.integers(3)), mut_k=int(rng.integers(15)),
                           mut_delta=float(rng.uniform(-0.01, 0.01)), mut_y0=int(rng.integers(H)),
                           mut_x0=int(rng.integers(W)), pen_p=p, pen_k=int(rng.integers(15)),
                           pen_delta=float((1 if p == 0 else -1) * rng.uniform(0, 0.01))))
    kw = dict(walls=wt, gamma_mut=1.0, mut_half=8, gamma_pen=0.2, r_oxy=r_oxy)
    A = torch.tensor(world.A, device="cuda")
    P = torch.tensor(world.P, device="cuda")
    A2, P2 = torch.empty_like(A), torch.empty_like(P)
    plan.step_evolve(A, P, A2, P2, n_steps=warmup, events=events[:warmup], **kw)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    plan.step_evolve(A2, P2, A, P, n_steps=steps, events=events[warmup:], **kw)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    achieved = EVOLVE_BYTES_PER_CELL * H * W / (ms / 1e3) / 1e9
    from oracle import oracle as O
    n = 512
    Ac = np.ascontiguousarray(world.A[:, :n, :n])
    Pc = np.ascontiguousarray(world.P[:, :, :n, :n])
    dc = O.Desc(n, n, 3, 15, world.src, world.dst, world.R, world.n_shells, world.beta, world.dt, 1, 1)
    ev0 = dict(events[0], mut_y0=events[0]["mut_y0"] % n, mut_x0=events[0]["mut_x0"] % n)
    cpu = oracle_timing(lambda: O.evolve_step(dc, Ac, Pc, walls=walls[:n, :n], gamma_mut=1.0, mut_half=8,
                                              gamma_pen=0.2, r_oxy=r_oxy, event=ev0),
                        n, 4.0, "the operators workload")
    return {"value": H * W / (ms / 1e3), "unit": "cell-updates/s", "ms_per_step": ms,
            "cpu_baseline": cpu,
            "steps": steps, "warmup": warmup,
            "workload": f"the 4096^2 workload with walls every 512 cells, mutation (rate 1, side 16) "
                        f"and penalization (rate 0.2, r_oxy {r_oxy}) each step",
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", type=str, default="")
    ap.add_argument("--conv", choices=["direct", "dft"], default="direct",
                    help="potential form of the timed step: direct FP32 (default) or the "
                         "split-bf16 DFT-as-GEMM form on MFMA")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-dft", action="store_true", help="skip the MFMA DFT-form leg")
    ap.add_argument("--no-evolve", action="store_true",
                    help="skip the leg with walls, mutation and penalization")
    ap.add_argument("--no-ring", action="store_true",
                    help="skip the ring-decomposed kernel leg (slow input generation)")
    ap.add_argument("--only", choices=["ratio", "batched", "dft", "ring", "evolve", "small"],
                    default=None,
                    help="run a single secondary leg (for profiling) and print its JSON")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a 1 GiB fill, copy and sum (reference kernels for the "
                         "HBM byte counters)")
    ap.add_argument("--batched", action="store_true",
                    help="also time the 256-world batched workload (slow input generation)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (--gpus {args.gpus} requested); "
              "the path shards by domain decomposition, which is designed but not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_05639_amd import inputs, lenia

    if args.calibrate:
        # reference kernels of known size for the HBM byte counters: a 1 GiB
        # fill (writes), copy and sum (reads)
        src = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        print(f"calibration sum {float(src.sum()):.0f}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        del src, dst
    if args.only == "ratio":
        print(json.dumps({"bwd_fwd_ratio": backward_forward_ratio(),
                          "bwd_fwd_ratio_dft": backward_forward_ratio(
                              conv=lenia.CONV_DFT_SPLIT_BF16)}), flush=True)
        return
    if args.only == "batched":
        print(json.dumps({"batched": batched_throughput()}), flush=True)
        return
    if args.only == "small":
        print(json.dumps({"small_worlds": small_worlds()}), flush=True)
        return
    if args.only == "ring":
        print(json.dumps({"ring_form": ring_form()}), flush=True)
        return
    world = inputs.config3()
    if args.only == "evolve":
        print(json.dumps({"evolve": evolve_form(world)}), flush=True)
        return
    if args.only == "dft":
        print(json.dumps({"dft_split_bf16": dft_form(world),
                          "dft_split_f16": dft_form(world, conv=lenia.CONV_DFT_SPLIT_F16)}), flush=True)
        return
    cells = world.H * world.W
    tile = tuple(int(x) for x in args.tile.split("x")) if args.tile else None
    conv = lenia.CONV_DFT_SPLIT_BF16 if args.conv == "dft" else lenia.CONV_AUTO
    plan = lenia.Plan(world, tile=tile, conv=conv)
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
                   "dt": world.dt, "tile": [info.tile_y, info.tile_x],
                   "conv": "dft_split_bf16" if args.conv == "dft" else "direct_f32",
                   "wall_s": wall},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "note": ROOFLINE_NOTE},
    }
    del A2, P2, A, P
    if not args.no_evolve and args.conv == "direct":
        out["evolve"] = evolve_form(world)
    if args.conv == "direct":
        out["small_worlds"] = small_worlds()
    if not args.no_dft and args.conv == "direct":
        out["dft_split_bf16"] = dft_form(world)
        out["dft_split_f16"] = dft_form(world, conv=lenia.CONV_DFT_SPLIT_F16)
    if not args.no_backward:
        out["bwd_fwd_ratio"] = backward_forward_ratio()
        if not args.no_dft:
            out["bwd_fwd_ratio_dft"] = backward_forward_ratio(conv=lenia.CONV_DFT_SPLIT_BF16)
    if args.batched:
        out["batched"] = batched_throughput()
    if not args.no_ring:
        out["ring_form"] = ring_form()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(world)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
