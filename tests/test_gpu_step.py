"""GPU parity of the fused step (HIP path through the C ABI) against the FP64
oracle: per-step teacher forcing on identical FP32 inputs, max-abs <= 1e-5 on
A' and P' over cells whose alpha decision is not within 1e-5 of the cutoff."""
import numpy as np
import pytest

from paper_2304_05639_amd import inputs

from gpu_helpers import (MAX_EXCLUDED, MAX_EXCLUDED_WINDOW, TOL_STATE, check_excluded, compare_step, dev,
                         gpu_step, host, window)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_05639_amd import lenia
    lenia.lib()
    return lenia


def _parity(L, oracle, w, **plan_kw):
    d = oracle.Desc.from_world(w)
    plan = L.Plan(w, **plan_kw)
    A1, P1 = gpu_step(plan, w.A, w.P)
    r = oracle.step(d, w.A, w.P)
    return compare_step(r, A1, P1)


def test_global_single_channel_rollout_teacher_forced(L, oracle):
    """64x64, one kernel R=13, global genes: every one of 100 steps."""
    w = inputs.config1()
    d = oracle.Desc.from_world(w)
    plan = L.Plan(w)
    A = w.A.astype(np.float32)
    worst = 0.0
    for t in range(100):
        A1, _ = gpu_step(plan, A, None)
        r = oracle.step(d, A)
        errA, _, _ = compare_step(r, A1, None)
        worst = max(worst, errA)
        A = r["A"].astype(np.float32)       # teacher forcing from the oracle state
    print(f"global 64x64: worst per-step max-abs {worst:.3e} over 100 steps")


@pytest.mark.parametrize("H,W,seed", [(16, 16, 101), (40, 56, 102), (100, 150, 103),
                                      (64, 64, 104), (3, 5, 105), (1, 1, 106), (129, 67, 107),
                                      (24, 200, 108)])
def test_localized_parity_sizes(L, oracle, H, W, seed):
    """Several tiles, ragged tails, tori smaller than the kernel (multi-wrap)."""
    nb = max(1, H * W // 600)
    w = inputs.test_world(H, W, seed=seed, n_blobs=nb)
    errA, errP, n_amb = _parity(L, oracle, w)
    print(f"{H}x{W}: errA {errA:.2e} errP {errP:.2e} ambiguous {n_amb}")


@pytest.mark.parametrize("R,pattern", [(12, (1,)), (12, (2,)), (12, (3,)), (12, (3, 1, 2)), (13, (2, 3))])
def test_shell_counts(L, oracle, R, pattern):
    """The step combines per-shell sums for B = 1, 2 and 3 with each kernel's
    heights: worlds whose kernels all have one shell count, or a fixed mix,
    each a different set of the six sums in use (heights drawn in (0.1, 1),
    some of them 0 to leave a shell empty)."""
    w = inputs.test_world(56, 72, seed=170 + R + len(pattern), n_blobs=6, R=R)
    rng = np.random.default_rng(7 * R + sum(pattern))
    for k in range(w.n_shells.shape[0]):
        b = pattern[k % len(pattern)]
        w.n_shells[k] = b
        w.beta[k, :] = 0.0
        w.beta[k, :b] = rng.uniform(0.1, 1.0, b).astype(np.float32)
        if b > 1 and k % 4 == 1:
            w.beta[k, b - 1] = 0.0          # an empty outer shell
    errA, errP, n_amb = _parity(L, oracle, w)
    print(f"R={R} shells {pattern}: errA {errA:.2e} errP {errP:.2e} ambiguous {n_amb}")


def test_localized_readonly_genes(L, oracle):
    w = inputs.test_world(70, 90, seed=111, n_blobs=6, genotype_update=0)
    _parity(L, oracle, w)


def test_r13_three_channels(L, oracle):
    w = inputs.test_world(48, 80, seed=112, n_blobs=4, R=13)
    _parity(L, oracle, w)


def test_c2_teacher_forced_steps(L, oracle):
    """512x512, 15 kernels, localized genes: steps 0, 1, 2 and 6 teacher-forced."""
    w = inputs.config2()
    d = oracle.Desc.from_world(w)
    plan = L.Plan(w)
    A, P = w.A.astype(np.float64), w.P.astype(np.float64)
    for t in range(7):
        A32, P32 = A.astype(np.float32), P.astype(np.float32)
        r = oracle.step(d, A32, P32)
        if t in (0, 1, 2, 6):
            A1, P1 = gpu_step(plan, A32, P32)
            errA, errP, n_amb = compare_step(r, A1, P1)
            print(f"512^2 step {t}: errA {errA:.2e} errP {errP:.2e} ambiguous {n_amb}")
        A, P = r["A"], r["P"]


def test_zero_world_stays_zero(L):
    w = inputs.test_world(64, 64, seed=113, n_blobs=0)
    plan = L.Plan(w)
    A1, P1 = gpu_step(plan, np.zeros_like(w.A), w.P, n_steps=3)
    assert (A1 == 0).all() and (P1 == 0).all()
    w1 = inputs.config1()
    plan1 = L.Plan(w1)
    A1, _ = gpu_step(plan1, np.zeros_like(w1.A), None, n_steps=100)
    assert (A1 == 0).all()


def test_tiles_agree_bitwise(L):
    """Each cell's arithmetic does not depend on its tile: all tile shapes give
    identical bits."""
    w = inputs.test_world(160, 192, seed=114, n_blobs=8)
    outs = []
    for tile in [(16, 32), (32, 32), (8, 32), (16, 64), (8, 64), (4, 64)]:
        plan = L.Plan(w, tile=tile)
        assert (plan.info().tile_y, plan.info().tile_x) == tile
        outs.append(gpu_step(plan, w.A, w.P))
    for A1, P1 in outs[1:]:
        assert np.array_equal(A1, outs[0][0]) and np.array_equal(P1, outs[0][1])


@pytest.mark.parametrize("tile,dead_genes", [((8, 32), False), ((16, 32), False), ((8, 32), True)])
def test_empty_tile_shortcut_bitwise(L, tile, dead_genes):
    """Tiles where some channel is empty over the whole window (tile + halo),
    or where gene plane 0 is at or below eps on the tile and its ring, have
    alpha = 0 everywhere, so the step skips their convolution.  Asking for the
    saved potentials turns the shortcut off; both must give identical bits, on
    a world with empty and occupied tiles (and, with dead_genes, a band of
    matter whose genes were masked to 0 by an earlier step)."""
    w = inputs.test_world(256, 320, seed=116, n_blobs=4)
    assert (w.A == 0).all(axis=0).mean() > 0.5          # mostly empty space
    if dead_genes:
        w.A[:, 100:180, :] = np.maximum(w.A[:, 100:180, :], 0.3)
        w.P[:, :, 96:184, 40:300] = 0.0
    plan = L.Plan(w, tile=tile)
    a1, p1 = gpu_step(plan, w.A, w.P)
    a2, p2 = gpu_step(plan, w.A, w.P, saved=plan.new_saved())
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)
    assert (p1 != 0).any() and (a1 != 0).any()


def test_translation_bitwise(L):
    w = inputs.test_world(96, 128, seed=115, n_blobs=5)
    plan = L.Plan(w)
    A0, P0 = gpu_step(plan, w.A, w.P)
    sy, sx = 37, -45
    A1, P1 = gpu_step(plan, np.roll(w.A, (sy, sx), (1, 2)), np.roll(w.P, (sy, sx), (2, 3)))
    assert np.array_equal(A1, np.roll(A0, (sy, sx), (1, 2)))
    assert np.array_equal(P1, np.roll(P0, (sy, sx), (2, 3)))


def test_deterministic(L):
    w = inputs.test_world(128, 128, seed=116, n_blobs=6)
    plan = L.Plan(w)
    a = gpu_step(plan, w.A, w.P, n_steps=5)
    b = gpu_step(plan, w.A, w.P, n_steps=5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_multistep_schedules_agree(L):
    """n steps in one call (out of place, in place, odd/even) == n single calls."""
    import torch
    w = inputs.test_world(96, 96, seed=117, n_blobs=5)
    plan = L.Plan(w)
    A, P = dev(w.A), dev(w.P)
    ref = [(A.clone(), P.clone())]
    for _ in range(5):
        a, p = plan.step(ref[-1][0], ref[-1][1])
        ref.append((a, p))
    for n in (0, 1, 2, 3, 4, 5):
        a, p = plan.step(A, P, n_steps=n)                    # out of place
        torch.cuda.synchronize()
        assert torch.equal(a, ref[n][0]) and torch.equal(p, ref[n][1]), n
        a2, p2 = A.clone(), P.clone()
        plan.step(a2, p2, A_out=a2, P_out=p2, n_steps=n)     # in place
        torch.cuda.synchronize()
        assert torch.equal(a2, ref[n][0]) and torch.equal(p2, ref[n][1]), n
    # inputs untouched by out-of-place calls
    assert np.array_equal(host(A), w.A) and np.array_equal(host(P), w.P)


def test_long_call_matches_single_steps(L):
    """40 steps in one call equal 40 single-step calls, bitwise, in and out of
    place, on a sparse world whose tiles go from empty to active and back.
    In a call of more than two steps, a tile that takes the alpha = 0
    shortcut skips rewriting gene planes that its output buffer already holds
    as 0.  The caller's output buffer starts as NaN, so a skipped write that
    the call did not make itself would show."""
    import torch
    w = inputs.test_world(96, 160, seed=118, n_blobs=8)
    plan = L.Plan(w)
    A, P = dev(w.A), dev(w.P)
    a, p = A.clone(), P.clone()
    for _ in range(40):
        a, p = plan.step(a, p)
    A1 = torch.full_like(A, float("nan"))
    P1 = torch.full_like(P, float("nan"))
    plan.step(A, P, A_out=A1, P_out=P1, n_steps=40)
    Ai, Pi = A.clone(), P.clone()
    plan.step(Ai, Pi, A_out=Ai, P_out=Pi, n_steps=39)
    torch.cuda.synchronize()
    assert torch.equal(A1, a) and torch.equal(P1, p)
    b, q = A.clone(), P.clone()
    for _ in range(39):
        b, q = plan.step(b, q)
    torch.cuda.synchronize()
    assert torch.equal(Ai, b) and torch.equal(Pi, q)
    # the trajectory does cross the shortcut: some cells alive, some tiles empty
    alive = float((p[0, 0] > 0).float().mean())
    assert 0.0 < alive < 0.9, alive


def test_saved_potentials_and_alpha(L, oracle):
    w = inputs.test_world(80, 100, seed=118, n_blobs=6)
    d = oracle.Desc.from_world(w)
    plan = L.Plan(w)
    saved = plan.new_saved()
    gpu_step(plan, w.A, w.P, saved=saved)
    u, a = plan.saved_views(saved)
    r = oracle.step(d, w.A, w.P)
    assert np.abs(host(u) - r["U"]).max() <= 2e-6
    ok = (r["amb"] & 1) == 0
    check_excluded(~ok, MAX_EXCLUDED)
    assert np.array_equal(host(a)[ok], r["alpha"][ok])


def test_call_errors(L):
    import torch
    w = inputs.test_world(32, 32, seed=119, n_blobs=1)
    plan = L.Plan(w)
    A, P = dev(w.A), dev(w.P)
    with pytest.raises(L.LeniaError):
        plan.step(A, P, A_out=A, P_out=torch.empty_like(P))     # mixed in/out of place
    with pytest.raises(L.LeniaError):
        plan.step(A, P, n_steps=2, saved=plan.new_saved())      # saved needs n_steps == 1
    with pytest.raises(ValueError):
        plan.step(A[:2], P)


@pytest.fixture(scope="module")
def c3_world():
    return inputs.config3()


@pytest.mark.parametrize("t0", [0, 100, 1000, 10000])
def test_full_size_sampled_windows(L, oracle, c3_world, t0):
    """4096^2, 2000 blobs with their own genotypes, in the benchmark's launch
    configuration.  The GPU runs t0 steps freely; one more step is then taken
    from that state (teacher forcing: the oracle starts from the same FP32
    snapshot) and sampled windows, including ones across the torus seam, are
    checked cell by cell against the oracle run on the window plus its halo."""
    import torch
    w = c3_world
    plan = L.Plan(w)
    A, P = dev(w.A), dev(w.P)
    for _ in range(t0 // 1000):          # in chunks, each followed by a progress line
        A, P = plan.step(A, P, n_steps=1000)
        torch.cuda.synchronize()
        print(".", end="", flush=True)
    if t0 % 1000:
        A, P = plan.step(A, P, n_steps=t0 % 1000)
    torch.cuda.synchronize()
    A0h, P0h = host(A), host(P)
    A1, P1 = plan.step(A, P)
    torch.cuda.synchronize()
    A1h, P1h = host(A1), host(P1)
    del A, P, A1, P1
    rng = np.random.default_rng(5 + t0)
    m = w.R + 1                          # halo: kernel radius + diffusion radius
    hw = 48
    starts = [(0, 0), (4096 - 20, 4096 - 30), (2048, 17)] + \
             [tuple(rng.integers(0, 4096, 2)) for _ in range(3)]
    # one window centred on the densest matter, so that it is never all empty
    dens = A0h.sum(0)[::64, ::64]
    iy, ix = np.unravel_index(int(dens.argmax()), dens.shape)
    starts.append((iy * 64, ix * 64))
    active = 0
    for (y0, x0) in starts:
        Aw = window(A0h, y0 - m, x0 - m, hw + 2 * m, hw + 2 * m)
        Pw = window(P0h, y0 - m, x0 - m, hw + 2 * m, hw + 2 * m)
        dw = oracle.Desc(hw + 2 * m, hw + 2 * m, 3, 15, w.src, w.dst, w.R, w.n_shells, w.beta,
                         w.dt, 1, 1)
        r = oracle.step(dw, Aw, Pw)
        inner = (slice(m, m + hw), slice(m, m + hw))
        rr = dict(A=r["A"][(slice(None),) + inner], P=r["P"][(slice(None), slice(None)) + inner],
                  amb=r["amb"][inner])
        active += int((r["alpha"][inner] == 1).sum())
        compare_step(rr, window(A1h, y0, x0, hw, hw), window(P1h, y0, x0, hw, hw),
                     max_excluded=MAX_EXCLUDED_WINDOW)
    print(f"4096^2 at t={t0}: {len(starts)} windows, {active} cells with alpha = 1")
    assert active > 0


def test_check_finite_flag(L):
    """LENIA_FLAG_CHECK_FINITE: a plan with the flag steps exactly like one
    without it; a NaN or an infinity in an input buffer returns
    LENIA_ERR_NONFINITE before anything is enqueued (the outputs keep their
    contents)."""
    import torch
    w = inputs.test_world(64, 80, seed=121, n_blobs=4)
    ref = gpu_step(L.Plan(w), w.A, w.P)
    plan = L.Plan(w, check_finite=True)
    got = gpu_step(plan, w.A, w.P)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    for which, val in (("A", np.nan), ("A", np.inf), ("P", -np.inf), ("P", np.nan)):
        A, P = w.A.copy(), w.P.copy()
        (A if which == "A" else P).reshape(-1)[777] = val
        A_out = torch.full(w.A.shape, 7.0, device="cuda")
        P_out = torch.full(w.P.shape, 7.0, device="cuda")
        with pytest.raises(L.LeniaError) as e:
            plan.step(dev(A), dev(P), A_out, P_out)
        torch.cuda.synchronize()
        assert e.value.status == L.ERR_NONFINITE, str(e.value)
        assert (host(A_out) == 7.0).all() and (host(P_out) == 7.0).all()
    A = w.A.copy()
    A[1, 5, 6] = np.nan
    with pytest.raises(L.LeniaError) as e:
        plan.potentials(dev(A))
    assert e.value.status == L.ERR_NONFINITE
    # the adjoint checks its cotangents too
    saved = plan.new_saved()
    At, Pt = dev(w.A), dev(w.P)
    plan.step(At, Pt, saved=saved)
    gA1 = np.zeros(w.A.shape, np.float32)
    gA1[2, 3, 4] = np.inf
    with pytest.raises(L.LeniaError) as e:
        plan.backward(At, Pt, saved, dev(gA1), dev(np.zeros(w.P.shape, np.float32)))
    assert e.value.status == L.ERR_NONFINITE
    torch.cuda.synchronize()
