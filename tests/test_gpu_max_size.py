"""Worlds at the largest sizes the library accepts, where byte offsets within a
plane pass 2^31:

* 32767 x 32767 cells, one channel, global genes: H * W just below 2^30 (the
  limit), so byte offsets within the plane reach 2^32 - 4;
* 23201 x 23203 cells, 3 channels, 15 kernels, localized genes: just above
  2^29 cells, so every one of the 48 planes has byte offsets past 2^31
  (about 210 GB on the device with the plan's workspace).

Both sizes have ragged tails in both directions.  Inputs are drawn on the
device (a checkerboard of empty and random 1024 x 1024 squares, a band where
one gene plane is 0), the step or the operators' iteration runs in place, and
windows are checked cell by cell against the oracle run on the window plus its
halo.  The windows sit at the first cells, across both seams, around the cell
whose byte offset is 2^31, at the last cells, across the boundaries of the
empty squares and of the dead gene band, and at two random places."""
import numpy as np
import pytest

from paper_2304_05639_amd import inputs

from gpu_helpers import (AMB_TAU_DFT, MAX_EXCLUDED_WINDOW, TOL_STATE, TOL_STATE_DFT, compare_evolve,
                         compare_step, device_window)

pytestmark = pytest.mark.gpu

BLOCK = 1024
HW_WIN = 40


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_05639_amd import lenia
    lenia.lib()
    return lenia


def _starts(H, W, seed):
    c = (1 << 31) // 4                   # the cell whose byte offset is 2^31
    h = HW_WIN // 2
    rng = np.random.default_rng(seed)
    s = [(0, 0), (H - h, W - h), (c // W - h, c % W - h), (H - HW_WIN, W - HW_WIN),
         (BLOCK - h, BLOCK - h), (BLOCK - h, 100), (BLOCK - h, BLOCK + 100)]
    s += [(int(rng.integers(H)), int(rng.integers(W))) for _ in range(2)]
    return s


def _free(torch, *plans):
    for p in plans:
        p.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("conv", ["direct", "dft_bf16"])
def test_single_channel_largest_plane(L, oracle, conv):
    import torch
    H = W = 32767
    assert H * W < (1 << 30) and 4 * H * W > (3 << 30) and H % 8 and W % 32
    w = inputs.large_world(H, W, seed=inputs.SEED_BASE + 21, n_channels=1)
    plan = L.Plan(w, conv=L.CONV_DIRECT_F32 if conv == "direct" else L.CONV_DFT_SPLIT_BF16)
    tol, tau = (TOL_STATE, 1e-5) if conv == "direct" else (TOL_STATE_DFT, AMB_TAU_DFT)
    try:
        A, _ = inputs.device_state(w, seed=inputs.SEED_BASE + 22, block=BLOCK)
        m = w.R + 1
        starts = _starts(H, W, 2101)
        before = [device_window(A, y0 - m, x0 - m, HW_WIN + 2 * m, HW_WIN + 2 * m)
                  for (y0, x0) in starts]
        plan.step(A, None, A_out=A)
        torch.cuda.synchronize()
        after = [device_window(A, y0, x0, HW_WIN, HW_WIN) for (y0, x0) in starts]
        del A
    finally:
        _free(torch, plan)
    n = HW_WIN + 2 * m
    d = oracle.Desc(n, n, 1, 1, w.src, w.dst, w.R, w.n_shells, w.beta, w.dt, 0, 0, w.m, w.s, w.h,
             tau=tau)
    worst = 0.0
    for (y0, x0), Aw, A1 in zip(starts, before, after):
        r = oracle.step(d, Aw)
        inner = (slice(m, m + HW_WIN), slice(m, m + HW_WIN))
        rr = dict(A=r["A"][(slice(None),) + inner], P=None, amb=r["amb"][inner])
        errA, _, _ = compare_step(rr, A1, None, tol=tol, max_excluded=MAX_EXCLUDED_WINDOW)
        worst = max(worst, errA)
        print(f"{H}x{W} {conv} window at ({y0}, {x0}): A' err {errA:.2e}", flush=True)
    print(f"{H}x{W} {conv}: worst {worst:.2e}")


@pytest.mark.parametrize("conv", ["direct", "dft_bf16"])
def test_localized_planes_past_2_31_bytes(L, oracle, conv):
    import torch
    H, W = 23201, 23203
    assert H * W > (1 << 29) and H % 8 and W % 32
    w = inputs.large_world(H, W, seed=inputs.SEED_BASE + 23)
    plan = L.Plan(w, conv=L.CONV_DIRECT_F32 if conv == "direct" else L.CONV_DFT_SPLIT_BF16)
    tol, tau = (TOL_STATE, 1e-5) if conv == "direct" else (TOL_STATE_DFT, AMB_TAU_DFT)
    m = w.R + 1
    starts = _starts(H, W, 2301)
    try:
        A, P = inputs.device_state(w, seed=inputs.SEED_BASE + 24, block=BLOCK)
        win = lambda t, y0, x0, n: device_window(t, y0, x0, n, n)
        before = [(win(A, y0 - m, x0 - m, HW_WIN + 2 * m), win(P, y0 - m, x0 - m, HW_WIN + 2 * m))
                  for (y0, x0) in starts]
        plan.step(A, P, A_out=A, P_out=P)
        torch.cuda.synchronize()
        after = [(win(A, y0, x0, HW_WIN), win(P, y0, x0, HW_WIN)) for (y0, x0) in starts]
        del A, P
    finally:
        _free(torch, plan)
    n = HW_WIN + 2 * m
    d = oracle.Desc(n, n, 3, 15, w.src, w.dst, w.R, w.n_shells, w.beta, w.dt, 1, 1, tau=tau)
    active = 0
    for (y0, x0), (Aw, Pw), (A1, P1) in zip(starts, before, after):
        r = oracle.step(d, Aw, Pw)
        inner = (slice(m, m + HW_WIN), slice(m, m + HW_WIN))
        rr = dict(A=r["A"][(slice(None),) + inner], P=r["P"][(slice(None), slice(None)) + inner],
                  amb=r["amb"][inner])
        errA, errP, n_amb = compare_step(rr, A1, P1, tol=tol,
                                           max_excluded=MAX_EXCLUDED_WINDOW)
        a = int((r["alpha"][inner] == 1).sum())
        active += a
        print(f"{H}x{W} {conv} window at ({y0}, {x0}): A' {errA:.2e} P' {errP:.2e} "
              f"alpha=1 {a} ambiguous {n_amb}", flush=True)
    assert active > 0


def test_operators_planes_past_2_31_bytes(L, oracle):
    """Walls (every 4096th row and column, and the last row and column),
    mutation on a square wrapped across both seams at the last cells, and
    penalization, in one iteration at 23201 x 23203."""
    import torch
    H, W = 23201, 23203
    r_oxy, mut_half = 6, 8
    w = inputs.large_world(H, W, seed=inputs.SEED_BASE + 23)
    plan = L.Plan(w, conv=L.CONV_DIRECT_F32)
    ev = dict(mut_p=1, mut_k=7, mut_delta=float(np.float32(0.004)), mut_y0=H - 5, mut_x0=W - 3,
              pen_p=0, pen_k=3, pen_delta=float(np.float32(0.006)))
    m = w.R + 1 + 2 * r_oxy
    starts = _starts(H, W, 2401)
    n = HW_WIN + 2 * m
    try:
        A, P = inputs.device_state(w, seed=inputs.SEED_BASE + 25, block=BLOCK)
        walls = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
        walls[::4096, :] = 1
        walls[:, ::4096] = 1
        walls[H - 1, :] = 1
        walls[:, W - 1] = 1
        win = lambda t, y0, x0, k: device_window(t, y0, x0, k, k)
        before = [(win(A, y0 - m, x0 - m, n), win(P, y0 - m, x0 - m, n), win(walls, y0 - m, x0 - m, n))
                  for (y0, x0) in starts]
        plan.step_evolve(A, P, A_out=A, P_out=P, walls=walls, gamma_mut=5.0, mut_half=mut_half,
                         gamma_pen=0.2, r_oxy=r_oxy, events=[ev])
        torch.cuda.synchronize()
        after = [(win(A, y0, x0, HW_WIN), win(P, y0, x0, HW_WIN)) for (y0, x0) in starts]
        del A, P, walls
    finally:
        _free(torch, plan)
    d = oracle.Desc(n, n, 3, 15, w.src, w.dst, w.R, w.n_shells, w.beta, w.dt, 1, 1)
    for (y0, x0), (Aw, Pw, Ww), (A1, P1) in zip(starts, before, after):
        # the square's cells, as offsets from the crop's first cell, where they
        # fall inside the crop (the crop's own torus is smaller, so a square
        # elsewhere must not be wrapped into it)
        sy = (np.arange(2 * mut_half) + ev["mut_y0"] - mut_half - (y0 - m)) % H
        sx = (np.arange(2 * mut_half) + ev["mut_x0"] - mut_half - (x0 - m)) % W
        hit = bool((sy < n).any() and (sx < n).any())
        if hit:
            assert (sy < n).all() and (sx < n).all(), "square cut by a crop edge"
        evw = dict(ev, mut_y0=int(sy[0]) + mut_half, mut_x0=int(sx[0]) + mut_half)
        r = oracle.evolve_step(d, Aw, Pw, walls=Ww, gamma_mut=5.0 if hit else 0.0,
                               mut_half=mut_half, gamma_pen=0.2, r_oxy=r_oxy, event=evw)
        inner = (slice(m, m + HW_WIN), slice(m, m + HW_WIN))
        rr = dict(A=r["A"][(slice(None),) + inner], P=r["P"][(slice(None), slice(None)) + inner],
                  amb=r["amb"][inner])
        # windows lie across the edges of the empty squares: the cells within
        # 2 r_oxy of the organic-sum boundary there (a band 25 cells wide) may
        # all be excluded
        eA, eP, n_bad = compare_evolve(rr, A1, P1, r_oxy, TOL_STATE, max_excluded=0.6)
        print(f"{H}x{W} operators window at ({y0}, {x0}): A' {eA:.2e} P' {eP:.2e} "
              f"excluded {n_bad} square {hit}", flush=True)
