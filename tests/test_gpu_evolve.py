"""GPU parity of the operators around a step (lenia_step_evolve through the C
ABI: walls, mutation, penalization; Algorithm 2, Sections 2.5-2.7) against the
oracle's evolve step on identical FP32 inputs and identical random draws.

Cells whose alpha decision is ambiguous are excluded as for the plain step.
Where the organic-matter sum is within tau of eps the penalizing area may
differ within 2 r_oxy of it, so those neighbourhoods are excluded too."""
import numpy as np
import pytest

from paper_2304_05639_amd import inputs

from gpu_helpers import (MAX_EXCLUDED_WINDOW, TOL_STATE, compare_evolve as _compare, dev, host,
                         window)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_05639_amd import lenia
    lenia.lib()
    return lenia


def _events(rng, n, H, W, nk=15):
    return [dict(mut_p=int(rng.integers(3)), mut_k=int(rng.integers(nk)),
                 mut_delta=float(np.float32(rng.uniform(-0.01, 0.01))), mut_y0=int(rng.integers(H)),
                 mut_x0=int(rng.integers(W)), pen_p=(p := int(rng.integers(2))),
                 pen_k=int(rng.integers(nk)),
                 pen_delta=float(np.float32((1 if p == 0 else -1) * rng.uniform(0, 0.01))))
            for _ in range(n)]


def _walls(H, W):
    walls = np.zeros((H, W), np.uint8)
    walls[H // 2: H // 2 + 2, :] = 1            # a horizontal wall two cells thick
    walls[:, W // 3] = 1                         # and a vertical one
    return walls


@pytest.mark.parametrize("conv,tol", [(1, TOL_STATE), (2, 5e-4), (3, TOL_STATE)])
def test_evolve_teacher_forced(L, oracle, conv, tol):
    import torch
    H, W, r_oxy = 96, 128, 4
    w = inputs.test_world(H, W, seed=801, n_blobs=24)
    d = oracle.Desc.from_world(w, tau=2e-5 if conv == 2 else 1e-5)
    plan = L.Plan(w, conv=conv)
    walls = _walls(H, W)
    wt = torch.tensor(walls, device="cuda")
    rng = np.random.default_rng(801)
    evs = _events(rng, 4, H, W)
    A, P = w.A.astype(np.float64), w.P.astype(np.float64)
    for t in range(4):
        A32, P32 = A.astype(np.float32), P.astype(np.float32)
        At, Pt = dev(A32), dev(P32)
        A1, P1 = plan.step_evolve(At, Pt, walls=wt, gamma_mut=5.0, mut_half=6, gamma_pen=0.2,
                                  r_oxy=r_oxy, events=[evs[t]])
        torch.cuda.synchronize()
        # the wall cells of the input were zeroed in place
        assert (host(At)[:, walls == 1] == 0).all() and (host(Pt)[:, :, walls == 1] == 0).all()
        r = oracle.evolve_step(d, A32, P32, walls=walls, gamma_mut=5.0, mut_half=6, gamma_pen=0.2,
                               r_oxy=r_oxy, event=evs[t])
        eA, eP, n_bad = _compare(r, host(A1), host(P1), r_oxy, tol)
        print(f"evolve conv={conv} t={t}: errA {eA:.2e} errP {eP:.2e} excluded {n_bad} "
              f"E_pen {int(r['epen'].sum())} alpha {int((r['flags'] & 1).sum())}", flush=True)
        A, P = r["A"], r["P"]


def test_evolve_without_operators_is_the_step(L):
    import torch
    w = inputs.test_world(80, 100, seed=802, n_blobs=12)
    plan = L.Plan(w)
    A, P = dev(w.A), dev(w.P)
    A1, P1 = plan.step(A, P, n_steps=3)
    A2, P2 = plan.step_evolve(A.clone(), P.clone(), n_steps=3)
    torch.cuda.synchronize()
    assert torch.equal(A1, A2) and torch.equal(P1, P2)


def test_evolve_mutation_square_across_the_seam(L):
    import torch
    H, W, half = 40, 48, 7
    w = inputs.test_world(H, W, seed=803, n_blobs=0)
    A = np.broadcast_to(np.float32([0.3, 0.25, 0.35])[:, None, None], (3, H, W)).copy()
    P = np.empty((3, 15, H, W), np.float32)
    P[0], P[1], P[2] = 0.28, 0.06, 0.4
    plan = L.Plan(w)
    ev = dict(mut_p=2, mut_k=11, mut_delta=0.02, mut_y0=1, mut_x0=W - 2)
    _, P1 = plan.step_evolve(dev(A), dev(P), gamma_mut=3.0, mut_half=half, events=[ev])
    torch.cuda.synchronize()
    P1 = host(P1)
    _, P0 = plan.step(dev(A), dev(P))
    want = host(P0).copy()
    ys = (1 - half + np.arange(2 * half)) % H
    xs = (W - 2 - half + np.arange(2 * half)) % W
    want[2, 11][np.ix_(ys, xs)] += np.float32(3.0 * np.float32(0.02))
    assert np.array_equal(P1, want)


@pytest.mark.parametrize("H,W,r_oxy,seed,world", [
    (96, 192, 14, 821, "band"),
    (96, 192, 16, 822, "band"),     # the largest radius
    (96, 90, 16, 823, "band"),      # torus narrower than the disk test's tile + halo (wrap by modulo)
    (100, 150, 13, 825, "band"),    # ragged in both directions
    (96, 128, 0, 811, "blobs"),     # the disk is the cell itself
    (33, 70, 2, 814, "blobs"),
])
def test_evolve_penalizing_area_radii(L, oracle, H, W, r_oxy, seed, world):
    """One iteration with penalization and mutation against the oracle's evolve
    step, at the edge radii of the penalizing area and on tori where the disk
    test's tiles wrap or are ragged.  The band worlds have a thin band of
    matter, whose organic region holds no disk of radius r_oxy, and a thick
    block that does, so the penalizing area covers some alpha cells and not
    others and its shape decides the result."""
    import torch
    if world == "band":
        w = inputs.band_and_block_world(H, W, seed)
    else:
        w = inputs.test_world(H, W, seed=seed, n_blobs=max(1, H * W // 400))
    d = oracle.Desc.from_world(w)
    plan = L.Plan(w)
    ev = _events(np.random.default_rng(seed), 1, H, W)[0]
    mut_half = min(6, H // 2, W // 2)
    A32, P32 = w.A.astype(np.float32), w.P.astype(np.float32)
    A1, P1 = plan.step_evolve(dev(A32), dev(P32), gamma_mut=5.0, mut_half=mut_half, gamma_pen=0.2,
                              r_oxy=r_oxy, events=[ev])
    torch.cuda.synchronize()
    r = oracle.evolve_step(d, A32, P32, gamma_mut=5.0, mut_half=mut_half, gamma_pen=0.2,
                           r_oxy=r_oxy, event=ev)
    alpha = (r["flags"] & 1) != 0
    pen = int(((r["epen"] != 0) & alpha).sum())
    eA, eP, n_bad = _compare(r, host(A1), host(P1), r_oxy, TOL_STATE)
    print(f"{world} {H}x{W} r_oxy={r_oxy}: errA {eA:.2e} errP {eP:.2e} excluded {n_bad} "
          f"penalized {pen} of {int(alpha.sum())} alpha cells", flush=True)
    assert pen > 0
    if world == "band":
        assert pen < int(alpha.sum())


def test_evolve_rejects(L):
    import torch
    w = inputs.test_world(32, 32, seed=804, n_blobs=1)
    plan = L.Plan(w)
    A, P = dev(w.A), dev(w.P)
    for kw in (dict(r_oxy=17, gamma_pen=0.2, events=[dict(pen_p=0)]),
               dict(gamma_mut=1.0, mut_half=17, events=[dict(mut_p=0)]),
               dict(gamma_pen=0.2, events=[dict(pen_p=2)]),
               dict(gamma_mut=1.0, events=[dict(mut_k=15)]),
               dict(gamma_mut=1.0)):
        with pytest.raises(L.LeniaError):
            plan.step_evolve(A, P, **kw)
    rw = inputs.ring_test_world(32, 32, seed=805, n_blobs=1)
    with pytest.raises(L.LeniaError):
        L.Plan(rw).step_evolve(dev(rw.A), dev(rw.P))


def test_evolve_full_size_sampled_windows(L, oracle):
    """4096^2 benchmark world, walls every 512 rows and columns, both rates on:
    one iteration, checked on windows against the oracle run on the window
    plus a halo of R + 1 + 2 r_oxy (the reach of the penalizing area)."""
    import torch
    w = inputs.config3()
    H = W = 4096
    r_oxy = 6
    walls = np.zeros((H, W), np.uint8)
    walls[::512, :] = 1
    walls[:, ::512] = 1
    rng = np.random.default_rng(806)
    ev = _events(rng, 1, H, W)[0]
    ev["mut_y0"], ev["mut_x0"] = 2060, 40
    plan = L.Plan(w)
    A, P = dev(w.A), dev(w.P)
    A1, P1 = plan.step_evolve(A, P, walls=torch.tensor(walls, device="cuda"), gamma_mut=5.0,
                              mut_half=8, gamma_pen=0.2, r_oxy=r_oxy, events=[ev])
    torch.cuda.synchronize()
    A1h, P1h = host(A1), host(P1)
    del A, P, A1, P1
    m = w.R + 1 + 2 * r_oxy
    hw = 40
    square = np.zeros((H, W), bool)
    square[np.ix_((ev["mut_y0"] - 8 + np.arange(16)) % H, (ev["mut_x0"] - 8 + np.arange(16)) % W)] = True
    starts = [(2048, 17), (4096 - 20, 4096 - 30), (500, 500)]
    dens = w.A.sum(0)[::64, ::64]
    iy, ix = np.unravel_index(int(dens.argmax()), dens.shape)
    starts.append((iy * 64, ix * 64))
    for (y0, x0) in starts:
        sl = lambda a: window(a, y0 - m, x0 - m, hw + 2 * m, hw + 2 * m)
        dw = oracle.Desc(hw + 2 * m, hw + 2 * m, 3, 15, w.src, w.dst, w.R, w.n_shells, w.beta,
                         w.dt, 1, 1)
        # the square, where it meets the crop, lies inside it (the crop's own
        # torus is smaller, so a square elsewhere must not be wrapped into it)
        hit = bool(sl(square).any())
        evw = dict(ev, mut_y0=ev["mut_y0"] - (y0 - m), mut_x0=ev["mut_x0"] - (x0 - m))
        r = oracle.evolve_step(dw, sl(w.A), sl(w.P), walls=sl(walls), gamma_mut=5.0 if hit else 0.0,
                               mut_half=8,
                               gamma_pen=0.2, r_oxy=r_oxy, event=evw)
        inner = (slice(m, m + hw), slice(m, m + hw))
        rr = dict(A=r["A"][(slice(None),) + inner], P=r["P"][(slice(None), slice(None)) + inner],
                  amb=r["amb"][inner])
        _compare(rr, window(A1h, y0, x0, hw, hw), window(P1h, y0, x0, hw, hw), r_oxy, TOL_STATE,
                 max_excluded=MAX_EXCLUDED_WINDOW)


def test_evolve_long_call_matches_single_iterations(L):
    """12 iterations with walls, mutation and penalization in one call equal 12
    single calls, bitwise, with the caller's output buffers starting as NaN
    (the zero-gene tile flags act from the third step of a call)."""
    import torch
    H, W = 80, 128
    w = inputs.test_world(H, W, seed=808, n_blobs=6)
    plan = L.Plan(w)
    walls = torch.tensor(_walls(H, W), device="cuda")
    evs = _events(np.random.default_rng(808), 12, H, W)
    kw = dict(walls=walls, gamma_mut=5.0, mut_half=6, gamma_pen=0.2, r_oxy=3)
    A, P = dev(w.A), dev(w.P)
    B, Q = A.clone(), P.clone()
    for t in range(12):
        B, Q = plan.step_evolve(B, Q, events=[evs[t]], **kw)
    A1 = torch.full_like(A, float("nan"))
    P1 = torch.full_like(P, float("nan"))
    plan.step_evolve(A.clone(), P.clone(), A1, P1, n_steps=12, events=evs, **kw)
    torch.cuda.synchronize()
    assert torch.equal(A1, B) and torch.equal(P1, Q)


def test_evolve_multi_step_call_matches_single_steps(L):
    """n iterations in one call (ping-pong buffers, in place and out of place)
    equal one call per iteration with the same events, bitwise."""
    import torch
    H, W = 72, 96
    w = inputs.test_world(H, W, seed=807, n_blobs=14)
    plan = L.Plan(w)
    walls = torch.tensor(_walls(H, W), device="cuda")
    evs = _events(np.random.default_rng(807), 3, H, W)
    kw = dict(walls=walls, gamma_mut=5.0, mut_half=6, gamma_pen=0.2, r_oxy=3)
    A, P = dev(w.A), dev(w.P)
    B, Q = A.clone(), P.clone()
    for t in range(3):
        B, Q = plan.step_evolve(B, Q, events=[evs[t]], **kw)
    A3, P3 = plan.step_evolve(A.clone(), P.clone(), n_steps=3, events=evs, **kw)
    Ai, Pi = A.clone(), P.clone()
    plan.step_evolve(Ai, Pi, Ai, Pi, n_steps=3, events=evs, **kw)
    torch.cuda.synchronize()
    assert torch.equal(A3, B) and torch.equal(P3, Q)
    assert torch.equal(Ai, B) and torch.equal(Pi, Q)
