"""Throughput benchmark of the multi-channel Lenia step on one MI355X.

Headline workload: a 4096 x 4096 torus, 3 channels, 15 kernels (R = 12, 1-3
ring shells), localized m/s/h genes with diffusion and alpha masking, 2000
blobs each carrying its own genotype (seeded synthetic input), run for
10,000 steps.  The world needs a few hundred steps to fill: about 3% of the
cells are alive (alpha = 1) over its first 25 steps, 75% at step 400 and
95-99% from step 1000 on, where a step costs about four times what it costs
at the start.  The headline therefore times K steps of the sustained phase:
the world is advanced ADVANCE = 2000 steps untimed, then W warm-up steps,
then K timed steps in one call, with every input already resident in HBM.
The whole 10,000-step run is timed too (`full_run`), as is the early phase.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
  python bench.py --only LEG          (one leg, for profiling)

Prints one JSON line.  Each leg's roofline takes its achieved figure from the
algorithmic bytes (or flops) over the leg's kernel time measured here with
HIP events, and its `traffic` from a committed counter profile of the same
command and window (profiles/traffic_<leg>.json), or null when that profile
was taken on other kernel sources.  `python bench.py --summarize ...` turns
the two rocprofv3 counter runs of a leg into that profile.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0     # dense bf16 / fp16 MFMA
BYTES_PER_CELL = 384          # read A 12 + write A 12 + read P 180 + write P 180 (FP32)
RING_BYTES_PER_CELL = 1104    # 9 gene types per kernel: A 24 + P 540 read + 540 written
EVOLVE_BYTES_PER_CELL = 392   # the step's 384 + wall mask 1 + flags 3 + area masks 4
ADVANCE = 2000                # untimed steps before the headline window
RING_ADVANCE = 500            # the ring-form world's advance
FULL_RUN_STEPS = 10000
CSRC = os.path.join(ROOT, "paper_2304_05639_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
# sources whose kernels each leg's counter profile describes
LEG_SRCS = {
    "headline": ("lenia_step.hip", "lenia_device.h", "lenia_internal.h", "lenia_plan.cpp"),
    "ring": ("lenia_step.hip", "lenia_device.h", "lenia_internal.h", "lenia_plan.cpp"),
    "batched": ("lenia_step.hip", "lenia_device.h", "lenia_internal.h", "lenia_plan.cpp"),
    "dft_f16": ("lenia_dft.hip", "lenia_device.h", "lenia_internal.h"),
    "dft_f16_step": ("lenia_dft.hip", "lenia_device.h", "lenia_internal.h", "lenia_plan.cpp"),
}
# the kernel each leg's roofline is about (a substring of its name in the trace)
LEG_KERNEL = {"headline": "step_kernel<lenia::Table3x15, 12, 8, 32>",
              "ring": "ring_step_kernel", "batched": "step_batch_kernel",
              # as the trace names them: potentials only, and the whole (fused) step
              "dft_f16": "15dft_conv_kernelINS_9Table3x15ELi12EDF16_Lb0E",
              "dft_f16_step": "15dft_conv_kernelINS_9Table3x15ELi12EDF16_Lb1E"}


def sources_sha(names) -> str:
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(CSRC, n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(leg: str, window: dict):
    """HBM bytes per launch of the leg's kernel from its committed counter
    profile, or None if it is absent, was taken on other kernel sources, or
    over another window."""
    try:
        with open(os.path.join(PROFILES, f"traffic_{leg}.json")) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != sources_sha(LEG_SRCS[leg]) or t.get("window") != window:
        return None
    return t.get("bytes_per_launch")


def hbm_roofline(bytes_alg: float, kernel_ms: float, leg: str, window: dict, kernel: str):
    achieved = bytes_alg / (kernel_ms / 1e3) / 1e9
    traffic = counter_traffic(leg, window)
    r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
         "kernel_ms": kernel_ms}
    if traffic is not None:
        r["traffic_frac"] = traffic / (kernel_ms / 1e3) / 1e9 / HBM_PEAK_GBS
    return r


def timed(fn, stream=None):
    """(result, ms) of fn() between two HIP events on the current stream."""
    import torch
    s = stream or torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    out = fn()
    e1.record(s)
    torch.cuda.synchronize()
    return out, e0.elapsed_time(e1)


def alive(P) -> float:
    """Fraction of cells whose alpha held in the step that wrote P: there every
    diffused gene exceeds eps > 0, elsewhere every gene is 0."""
    return float((P[0, 0] > 0).float().mean())


class Pair:
    """The state and its ping-pong partner on the device."""

    def __init__(self, A, P):
        import torch
        self.A, self.P = A, P
        self.A2, self.P2 = torch.empty_like(A), torch.empty_like(P)

    def step(self, plan, n):
        plan.step(self.A, self.P, self.A2, self.P2, n_steps=n)
        self.A, self.A2, self.P, self.P2 = self.A2, self.A, self.P2, self.P


# ---- legs -------------------------------------------------------------------------

def headline(world, steps: int, warmup: int, advance: int = ADVANCE):
    """K steps of the 4096^2 workload's sustained phase in one call."""
    import torch
    from paper_2304_05639_amd import lenia
    plan = lenia.Plan(world)
    st = Pair(torch.tensor(world.A, device="cuda"), torch.tensor(world.P, device="cuda"))
    if advance:
        st.step(plan, advance)
    if warmup:
        st.step(plan, warmup)
    a0 = alive(st.P)
    _, ms = timed(lambda: st.step(plan, steps))
    cells = world.H * world.W
    info = plan.info()
    out = {"ms_per_step": ms / steps, "value": cells * steps / (ms / 1e3),
           "alive_frac": [a0, alive(st.P)], "tile": [info.tile_y, info.tile_x],
           "window": {"advance": advance, "warmup": warmup, "steps": steps}}
    return out, st


def early_phase(world, steps: int = 20, warmup: int = 5):
    """The same workload's first steps (t = 5 .. 25), when few cells are alive."""
    r, _ = headline(world, steps, warmup, advance=0)
    return {"value": r["value"], "unit": "cell-updates/s", "ms_per_step": r["ms_per_step"],
            "alive_frac": r["alive_frac"], "steps": steps, "warmup": warmup,
            "note": "steps 5-25 of the run: tiles without matter take exact shortcuts"}


def full_run(world, n: int = FULL_RUN_STEPS):
    """All n steps of the 4096^2 workload from its initial state in one call."""
    import torch
    from paper_2304_05639_amd import lenia
    plan = lenia.Plan(world)
    st = Pair(torch.tensor(world.A, device="cuda"), torch.tensor(world.P, device="cuda"))
    _, ms = timed(lambda: st.step(plan, n))
    return {"value": world.H * world.W * n / (ms / 1e3), "unit": "cell-updates/s",
            "ms_per_step": ms / n, "steps": n, "seconds": ms / 1e3, "alive_frac_end": alive(st.P),
            "note": "the whole run, steps 0 to 10,000, one call"}


def cpu_baseline(A, P, world, budget_s: float = 8.0):
    """The FP64 oracle, as it stands, on a 1024 x 1024 crop (its own torus) of
    the state the headline times, until the budget is spent."""
    import numpy as np
    from oracle import oracle as O
    n = 1024
    Ac = np.ascontiguousarray(A[:, :n, :n])
    Pc = np.ascontiguousarray(P[:, :, :n, :n])
    d = O.Desc(n, n, 3, 15, world.src, world.dst, world.R, world.n_shells, world.beta,
               world.dt, 1, 1)
    r = oracle_timing(lambda: O.step(d, Ac, Pc), n, budget_s,
                      "the headline's state (FP64 direct convolution, OpenMP over rows)")
    m = 256
    A1 = np.ascontiguousarray(A[:, :m, :m])
    P1 = np.ascontiguousarray(P[:, :, :m, :m])
    d1 = O.Desc(m, m, 3, 15, world.src, world.dst, world.R, world.n_shells, world.beta,
                world.dt, 1, 1)
    O.set_threads(1)
    one = oracle_timing(lambda: O.step(d1, A1, P1), m, 3.0, "the same state on one thread")
    O.set_threads(O.threads())
    r["value_1_thread"] = one["value"]
    r["sample_1_thread"] = one["sample"]
    return r


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


def evolve_form(world, A, P, steps: int = 20, warmup: int = 5, r_oxy: int = 6,
                with_cpu: bool = True):
    """Algorithm 2's operators around each step, from the headline's state:
    walls every 512 rows and columns, mutation (rate 1, squares of side 16)
    and the penalization of exploding patterns (rate 0.2, oxygen radius r_oxy),
    with seeded random draws per step."""
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
    A, P = A.clone(), P.clone()
    A2, P2 = torch.empty_like(A), torch.empty_like(P)
    plan.step_evolve(A, P, A2, P2, n_steps=warmup, events=events[:warmup], **kw)
    _, ms = timed(lambda: plan.step_evolve(A2, P2, A, P, n_steps=steps, events=events[warmup:], **kw))
    ms /= steps
    out = {"value": H * W / (ms / 1e3), "unit": "cell-updates/s", "ms_per_step": ms,
           "steps": steps, "warmup": warmup, "alive_frac_end": alive(P),
           "workload": f"the headline's state (after {ADVANCE} steps) with walls every 512 cells, "
                       f"mutation (rate 1, side 16) and penalization (rate 0.2, r_oxy {r_oxy}) "
                       "each step",
           "roofline": {"bound": "hbm", "achieved": EVOLVE_BYTES_PER_CELL * H * W / (ms / 1e3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": EVOLVE_BYTES_PER_CELL * H * W / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                        "traffic": None, "kernel": "the whole iteration (step, walls, disk tests, events)"}}
    if with_cpu:
        from oracle import oracle as O
        n = 512
        Ah, Ph = A.cpu().numpy(), P.cpu().numpy()
        Ac = np.ascontiguousarray(Ah[:, :n, :n])
        Pc = np.ascontiguousarray(Ph[:, :, :n, :n])
        dc = O.Desc(n, n, 3, 15, world.src, world.dst, world.R, world.n_shells, world.beta,
                    world.dt, 1, 1)
        ev0 = dict(events[0], mut_y0=events[0]["mut_y0"] % n, mut_x0=events[0]["mut_x0"] % n)
        out["cpu_baseline"] = oracle_timing(
            lambda: O.evolve_step(dc, Ac, Pc, walls=walls[:n, :n], gamma_mut=1.0, mut_half=8,
                                  gamma_pen=0.2, r_oxy=r_oxy, event=ev0),
            n, 4.0, "the operators workload")
    return out


# MFMA instructions (16x16x32, 16384 flops each) per 64 x 64 tile of the DFT
# forms, every product issued three times (hi*hi, hi*lo, lo*hi): per channel
# the half-spectrum forward transform, 16 output tiles x 2 k-steps (row DFT)
# and 16 x 4 (column DFT); per kernel the inverse, 10 x 4 (columns) and 9 x 2
# (rows, back to real values).
DFT_MFMA_PER_TILE = 3 * 3 * (16 * 2 + 16 * 4) + 15 * 3 * (10 * 4 + 9 * 2)
MFMA_FLOPS = 16 * 16 * 32 * 2


def dft_form(world, A, P, conv: int, steps: int = 20, warmup: int = 5, pot_reps: int = 20):
    """A split DFT-as-GEMM form from the headline's state.  `roofline` is the
    potentials-only MFMA kernel (lenia_potentials, timed alone) against the
    dense MFMA peak of its operand type (2.5 PFLOP/s for bf16 and fp16);
    `value` and `fused_step` are the whole step, one kernel in which the
    potentials never leave the chip."""
    import torch
    from paper_2304_05639_amd import lenia
    plan = lenia.Plan(world, conv=conv)
    V = plan.info().tile_y
    n_tiles = -(-world.H // V) * -(-world.W // V)
    U = torch.empty(world.n_kernels, world.H, world.W, device="cuda")
    for _ in range(2):
        plan.potentials(A, U)

    def pots():
        for _ in range(pot_reps):
            plan.potentials(A, U)
    _, k_ms = timed(pots)
    k_ms /= pot_reps
    st = Pair(A.clone(), P.clone())
    st.step(plan, warmup)
    _, s_ms = timed(lambda: st.step(plan, steps))
    s_ms /= steps
    flops = n_tiles * DFT_MFMA_PER_TILE * MFMA_FLOPS
    pot = flops / (k_ms / 1e3) / 1e12
    roof = {"bound": "mfma", "achieved": pot, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": pot / BF16_PEAK_TFLOPS, "kernel": "dft_conv_kernel (potentials only)",
            "kernel_ms": k_ms, "traffic": None}
    step = {"kernel": "dft_conv_kernel (whole step, fused)", "ms": s_ms,
            "mfma_tflops": flops / (s_ms / 1e3) / 1e12,
            "mfma_frac": flops / (s_ms / 1e3) / 1e12 / BF16_PEAK_TFLOPS,
            "hbm_gbs_algorithmic": BYTES_PER_CELL * world.H * world.W / (s_ms / 1e3) / 1e9,
            "traffic": None}
    if conv == lenia.CONV_DFT_SPLIT_F16:
        roof["traffic"] = counter_traffic("dft_f16", {"reps": pot_reps})
        step["traffic"] = counter_traffic("dft_f16_step", {"warmup": warmup, "steps": steps})
    return {"value": world.H * world.W / (s_ms / 1e3), "unit": "cell-updates/s",
            "ms_per_step": s_ms, "alive_frac_end": alive(st.P), "roofline": roof,
            "fused_step": step,
            "note": f"{n_tiles} tiles of 64x64 (valid {V}x{V}), {DFT_MFMA_PER_TILE} MFMA per tile; "
                    f"timed from the headline's state"}


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
        _, ms = timed(lambda: plan.step(A2, P2, A, P, n_steps=n))
        ms /= n
        out[name] = {"us_per_step": ms * 1e3, "steps_per_s": 1e3 / ms,
                     "cell_updates_per_s": w.H * w.W / (ms / 1e3), "steps": n}
    return out


def ring_form(steps: int = 20, warmup: int = 5, advance: int = RING_ADVANCE, with_cpu: bool = True):
    """The 4096^2 workload with ring-decomposed kernels (24 rings, localized
    kernel genes; drawn on the device), advanced `advance` steps untimed, then
    timed against the HBM floor of its algorithmic bytes."""
    from paper_2304_05639_amd import inputs, lenia
    world, A, P = inputs.device_config_ring()
    cells = world.H * world.W
    plan = lenia.Plan(world)
    st = Pair(A, P)
    del A, P
    st.step(plan, advance + warmup)
    a0 = alive(st.P)
    _, ms = timed(lambda: st.step(plan, steps))
    ms /= steps
    window = {"advance": advance, "warmup": warmup, "steps": steps}
    out = {"value": cells / (ms / 1e3), "unit": "cell-updates/s", "ms_per_step": ms,
           "steps": steps, "warmup": warmup, "advance": advance, "alive_frac": [a0, alive(st.P)],
           "workload": "lenia-ring-3ch15k-4096x4096: 24 rings of the R = 12 disk, 9 gene types "
                       "per kernel, 2000 blobs with their own genes (drawn on the device)",
           "roofline": hbm_roofline(RING_BYTES_PER_CELL * cells, ms, "ring", window,
                                    "ring_step_kernel<Table3x15, 12, 8, 32>")}
    if with_cpu:
        import numpy as np
        from oracle import oracle as O
        n = 256
        Ac = np.ascontiguousarray(st.A[:, :n, :n].cpu().numpy())
        Pc = np.ascontiguousarray(st.P[:, :, :n, :n].cpu().numpy())
        dc = O.Desc(n, n, 3, 15, world.src, world.dst, world.R, world.n_shells, world.beta,
                    world.dt, 1, 1, n_ring=world.n_ring)
        out["cpu_baseline"] = oracle_timing(lambda: O.ring_step(dc, Ac, Pc), n, 4.0,
                                            "the ring-form workload's state")
    return out


def batched_throughput(steps: int = 500, with_cpu: bool = True):
    """256 independent worlds of sides 128..1024 (drawn on the device) stepped
    together for 500 steps in one call: one launch per step over the (world,
    tile) work list, replayed from a HIP graph, autotuned tile."""
    import numpy as np
    import torch
    from paper_2304_05639_amd import inputs, lenia
    ws = inputs.device_config4()
    worlds = [w for w, _, _ in ws]
    As = [A for _, A, _ in ws]
    Ps = [P for _, _, P in ws]
    del ws
    cells = sum(w.H * w.W for w in worlds)
    bp = lenia.BatchedPlan(worlds, autotune=True)
    _, ms = timed(lambda: bp.step(As, Ps, n_steps=steps))
    ms /= steps
    info = bp.info()
    window = {"steps": steps}
    alive_end = float(sum(float((P[0, 0] > 0).float().sum()) for P in Ps) / cells)
    out = {"value": cells / (ms / 1e3), "unit": "cell-updates/s", "ms_per_step": ms,
           "cells": cells, "worlds": len(worlds), "steps": steps, "tile": [info.tile_y, info.tile_x],
           "alive_frac_end": alive_end,
           "roofline": hbm_roofline(BYTES_PER_CELL * cells, ms, "batched", window,
                                    "step_batch_kernel (autotuned tile)")}
    if with_cpu:
        from oracle import oracle as O
        i = min(range(len(worlds)), key=lambda j: worlds[j].H)
        w = worlds[i]
        Ac, Pc = As[i].cpu().numpy(), Ps[i].cpu().numpy()
        d = O.Desc(w.H, w.W, 3, 15, w.src, w.dst, w.R, w.n_shells, w.beta, w.dt, 1, 1)
        out["cpu_baseline"] = oracle_timing(lambda: O.step(d, Ac, Pc), w.H, 4.0,
                                            f"world {i} of the batch ({w.H}x{w.W}, whole torus)")
    return out


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
    name = {lenia.CONV_DFT_SPLIT_BF16: "dft_split_bf16", lenia.CONV_DFT_SPLIT_F16: "dft_split_f16"}
    return {"value": b / f, "forward_ms": f, "backward_ms": b, "conv": name.get(conv, "direct_f32"),
            "workload": "256x256, 3 channels, 15 kernels, T=64, checkpoint every 8, MSE loss"}


# ---- counter profiles ----------------------------------------------------------------

def _counter_rows(path_glob: str):
    rows = []
    for fn in sorted(glob.glob(path_glob, recursive=True)):
        with open(fn, newline="") as f:
            rows += list(csv.DictReader(f))
    return rows


def _per_dispatch(rows, counter: str):
    """{dispatch id: (kernel name, value)} of one counter (summed over
    instances)."""
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        d = int(r["Dispatch_Id"])
        name, v = r["Kernel_Name"], float(r["Counter_Value"])
        out[d] = (name, out.get(d, (name, 0.0))[1] + v)
    return out


def summarize(leg: str, fetch_glob: str, write_glob: str, window: dict, first: int, count: int,
              commands):
    """profiles/traffic_<leg>.json from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE) of `bench.py --only <leg> --calibrate`: the leg kernel's
    dispatches first .. first + count - 1 in launch order (the timed window;
    first < 0 counts from the end), each counter scaled by what it reads for a
    1 GiB read (a torch sum) and a 1 GiB write (a torch fill) in the same
    process."""
    f = _per_dispatch(_counter_rows(fetch_glob), "FETCH_SIZE")
    w = _per_dispatch(_counter_rows(write_glob), "WRITE_SIZE")
    gib_kib = 1024.0 * 1024.0

    def first_match(d, pat):
        for k in sorted(d):
            if pat in d[k][0]:
                return d[k][1]
        raise SystemExit(f"no dispatch matching {pat!r}")
    fetch_factor = gib_kib / first_match(f, "reduce_kernel")
    write_factor = gib_kib / first_match(w, "FillFunctor")
    all_f = [v for k, (n, v) in sorted(f.items()) if LEG_KERNEL[leg] in n]
    all_w = [v for k, (n, v) in sorted(w.items()) if LEG_KERNEL[leg] in n]
    # a counter run can miss a few records of graph-launched kernels; the
    # window is then whatever that run holds of it (at least half), counted
    # from the same end, and the dispatch counts of both runs are kept
    def window_of(v):
        start = first if first >= 0 else max(len(v) + first, 0)
        return start, v[start:start + count]
    (start, sel_f), (_, sel_w) = window_of(all_f), window_of(all_w)
    if 2 * min(len(sel_f), len(sel_w)) < count:
        raise SystemExit(f"found {len(sel_f)} / {len(sel_w)} dispatches of {LEG_KERNEL[leg]}")
    fk, wk = sum(sel_f) / len(sel_f), sum(sel_w) / len(sel_w)
    out = {"leg": leg, "kernel": LEG_KERNEL[leg], "kernel_sha": sources_sha(LEG_SRCS[leg]),
           "window": window, "dispatches": [start, count, len(all_f)],
           "dispatches_used": [len(sel_f), len(sel_w)], "dispatches_recorded": [len(all_f), len(all_w)],
           "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
           "fetch_factor": fetch_factor, "write_factor": write_factor,
           "bytes_per_launch": 1024.0 * (fk * fetch_factor + wk * write_factor),
           "commands": commands,
           "calibration": "FETCH_SIZE of a 1 GiB torch sum and WRITE_SIZE of a 1 GiB torch fill "
                          "in the same process; factor = true KiB / counted KiB"}
    with open(os.path.join(PROFILES, f"traffic_{leg}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def trace_summary(trace_glob: str, out_md: str, command: str):
    """A markdown summary of a rocprofv3 --kernel-trace run of the benchmark:
    per (kernel, grid) calls and durations, and the headline window (the
    4096^2 step kernel's dispatches ADVANCE + W .. ADVANCE + W + K - 1 of the
    default run, the headline leg being the first to launch it)."""
    rows = _counter_rows(trace_glob)
    by = {}
    for r in rows:
        key = (r["Kernel_Name"], int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0))
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        by.setdefault(key, []).append((int(r["Dispatch_Id"]), d))
    lines = [f"Kernel trace of `{command}`", "",
             "| kernel | grid (threads) | calls | average ns | min ns | max ns |", "|---|---|---|---|---|---|"]
    for (name, grid), v in sorted(by.items(), key=lambda kv: -sum(d for _, d in kv[1]))[:25]:
        ds = [d for _, d in v]
        lines.append(f"| `{name[:110]}` | {grid} | {len(ds)} | {sum(ds) / len(ds):.0f} | {min(ds)} | {max(ds)} |")
    head = [(i, d) for (name, grid), v in by.items() if LEG_KERNEL["headline"] in name and grid == 4096 * 4096
            for (i, d) in v]
    head.sort()
    return lines, head


# ---- main ------------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["headline", "full", "early", "evolve", "dft", "ring",
                                       "batched", "small", "ratio"], default=None,
                    help="run one leg (for profiling) and print its JSON")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a 1 GiB fill and a 1 GiB sum (reference kernels for the "
                         "HBM byte counters)")
    ap.add_argument("--summarize", nargs=3, metavar=("LEG", "FETCH_GLOB", "WRITE_GLOB"),
                    help="write profiles/traffic_LEG.json from two counter runs (no GPU)")
    ap.add_argument("--command", action="append", default=[],
                    help="with --summarize: the profiling commands, recorded in the file")
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_GLOB", "OUT_MD"),
                    help="markdown summary of a rocprofv3 kernel trace of the default run (no GPU)")
    ap.add_argument("--counter-summary", nargs=3, metavar=("LEG", "CSV_GLOB", "OUT_JSON"),
                    help="per-counter averages over the leg's timed window (no GPU)")
    args = ap.parse_args()
    if args.trace_summary:
        tg, out_md = args.trace_summary
        lines, head = trace_summary(tg, out_md, " ".join(args.command) or "python3 bench.py")
        K, W = args.steps, args.warmup
        win = head[ADVANCE + W:ADVANCE + W + K]
        if len(win) == K:
            avg = sum(d for _, d in win) / K
            lines += ["", f"Headline window: the 4096^2 step kernel's dispatches {ADVANCE + W} to "
                          f"{ADVANCE + W + K - 1} (of {len(head)}): average {avg:.0f} ns."]
        with open(out_md, "w") as fh:
            fh.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return
    if args.counter_summary:
        leg, cg, out_json = args.counter_summary
        K, W = args.steps, args.warmup
        first, count = {"headline": (ADVANCE + W, K), "ring": (RING_ADVANCE + W, K),
                        "dft_f16": (2, 20), "dft_f16_step": (-20, 20), "batched": (-500, 500)}[leg]
        rows = _counter_rows(cg)
        names = sorted({r["Counter_Name"] for r in rows})
        res = {"leg": leg, "kernel": LEG_KERNEL[leg], "counters": {}}
        for cn in names:
            per = _per_dispatch(rows, cn)
            vals = [v for k, (n, v) in sorted(per.items()) if LEG_KERNEL[leg] in n]
            start = first if first >= 0 else len(vals) + first
            sel = vals[start:start + count]
            res["counters"][cn] = sum(sel) / max(len(sel), 1)
            res["dispatches"] = [start, len(sel), len(vals)]
        with open(out_json, "w") as fh:
            json.dump(res, fh, indent=1)
        print(json.dumps(res))
        return
    if args.summarize:
        leg, fg, wg = args.summarize
        K, W = args.steps, args.warmup
        # (window, index of the first timed dispatch of the leg's kernel, count)
        windows = {"headline": ({"advance": ADVANCE, "warmup": W, "steps": K}, ADVANCE + W, K),
                   "ring": ({"advance": RING_ADVANCE, "warmup": W, "steps": K}, RING_ADVANCE + W, K),
                   "batched": ({"steps": 500}, -500, 500),
                   "dft_f16": ({"reps": 20}, 2, 20),
                   "dft_f16_step": ({"warmup": W, "steps": K}, -20, 20)}
        window, first, count = windows[leg]
        summarize(leg, fg, wg, window, first, count, args.command)
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (--gpus {args.gpus} requested); "
              "the path shards by domain decomposition, which is designed but not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_05639_amd import inputs, lenia
    with_cpu = not args.no_cpu_baseline

    if args.calibrate:
        # reference kernels of known size for the HBM byte counters: a 1 GiB
        # fill (writes) and a 1 GiB sum (reads)
        src = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        print(f"calibration sum {float(src.sum()):.0f}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        del src
    only = args.only
    if only == "ratio":
        print(json.dumps({f"bwd_fwd_ratio_{c}": backward_forward_ratio(conv=c) for c in (1, 2, 3)}),
              flush=True)
        return
    if only == "batched":
        print(json.dumps({"batched": batched_throughput(with_cpu=False)}), flush=True)
        return
    if only == "small":
        print(json.dumps({"small_worlds": small_worlds()}), flush=True)
        return
    if only == "ring":
        print(json.dumps({"ring_form": ring_form(args.steps, args.warmup, with_cpu=False)}),
              flush=True)
        return
    world = inputs.config3()
    if only == "full":
        print(json.dumps({"full_run": full_run(world)}), flush=True)
        return
    if only == "early":
        print(json.dumps({"early_phase": early_phase(world)}), flush=True)
        return

    t0 = time.perf_counter()
    h, st = headline(world, args.steps, args.warmup)
    wall = time.perf_counter() - t0
    cells = world.H * world.W
    if only in ("evolve", "dft"):
        if only == "evolve":
            print(json.dumps({"evolve": evolve_form(world, st.A, st.P, with_cpu=False)}), flush=True)
        else:
            print(json.dumps({"dft_split_f16": dft_form(world, st.A, st.P, lenia.CONV_DFT_SPLIT_F16)}),
                  flush=True)
        return
    out = {
        "metric": "cell-updates/s (cells x steps / s) at 4096^2, 3 channels, 15 kernels",
        "value": h["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lenia-3ch15k-4096x4096-localized-genes-2000-blobs, sustained phase "
                               f"(timed steps {ADVANCE + args.warmup}..{ADVANCE + args.warmup + args.steps} "
                               f"of the {FULL_RUN_STEPS}-step run)",
                   "world": [world.H, world.W], "channels": 3, "kernels": 15, "R": world.R,
                   "dt": world.dt, "tile": h["tile"], "conv": "direct_f32", "advance": ADVANCE,
                   "alive_frac": h["alive_frac"], "wall_s": wall},
        "roofline": hbm_roofline(BYTES_PER_CELL * cells, h["ms_per_step"], "headline", h["window"],
                                 "step_kernel<Table3x15, 12, 8, 32>"),
    }
    if only == "headline":
        print(json.dumps(out), flush=True)
        return
    A_state, P_state = st.A, st.P
    out["evolve"] = evolve_form(world, A_state, P_state, with_cpu=with_cpu)
    out["dft_split_f16"] = dft_form(world, A_state, P_state, lenia.CONV_DFT_SPLIT_F16)
    out["dft_split_bf16"] = dft_form(world, A_state, P_state, lenia.CONV_DFT_SPLIT_BF16)
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline(A_state.cpu().numpy(), P_state.cpu().numpy(), world)
    del st, A_state, P_state
    torch.cuda.empty_cache()
    out["early_phase"] = early_phase(world)
    out["full_run"] = full_run(world)
    torch.cuda.empty_cache()
    out["small_worlds"] = small_worlds()
    out["batched"] = batched_throughput(with_cpu=with_cpu)
    torch.cuda.empty_cache()
    out["ring_form"] = ring_form(args.steps, args.warmup, with_cpu=with_cpu)
    torch.cuda.empty_cache()
    for c, key in ((1, "bwd_fwd_ratio"), (2, "bwd_fwd_ratio_dft_bf16"), (3, "bwd_fwd_ratio_dft_f16")):
        out[key] = backward_forward_ratio(conv=c)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
