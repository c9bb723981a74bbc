"""GPU parity of the adjoint (lenia_backward through the C ABI) against the FP64
oracle's vector-Jacobian product on identical FP32 inputs.

Where a thresholded decision (alpha, a clip) is within 1e-5 of its cutoff in
the oracle, either side is correct and the gradient differs locally, so
gradients are compared only where no such cell can reach them: gA at cells
farther than R from any ambiguous cell, gP farther than 1.  A "smooth" world
(every decision far from its cutoff) checks everything, shell heights included,
over the whole torus."""
import numpy as np
import pytest

from paper_2304_05639_amd import inputs

from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

TOL_REL = 2e-5      # relative max-abs error of each gradient
# Under the split-bf16 DFT form the saved potentials carry an absolute error of
# up to TOL_U = 2e-5.  The u-derivative of the growth, -2h e x / s with
# x = (u - m)/s, peaks at 1.21 h / s, and its own u-derivative is bounded by
# 2h / s^2, so a potential error du moves it by at most 1.65 du / s relative to
# its peak: 1.1e-3 at the smallest s of the smooth world (0.03).  The gene and
# shell-height gradients inherit the same factor.
TOL_REL_DFT = 2e-3
# The same bound for the scaled fp16 form, whose potentials are within 1e-6:
# 1.65 * 1e-6 / 0.03 = 5.5e-5, plus the FP32 form's own 2e-5.
TOL_REL_DFT_F16 = 8e-5


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_05639_amd import lenia
    lenia.lib()
    return lenia


def _dilate(mask, r):
    H, W = mask.shape
    out = np.zeros_like(mask)
    ys, xs = np.nonzero(mask)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dy * dy + dx * dx <= r * r:
                out[(ys + dy) % H, (xs + dx) % W] = True
    return out


def _gpu_vjp(L, w, gA1, gP1, conv=1):
    import torch
    plan = L.Plan(w, conv=conv)
    A, P = dev(w.A), dev(w.P)
    saved = plan.new_saved()
    plan.step(A, P, saved=saved)
    gA, gP, gb = plan.backward(A, P, saved, dev(gA1), dev(gP1))
    torch.cuda.synchronize()
    return host(gA), host(gP), host(gb)


def _rel(a, b, mask=None):
    d = np.abs(a - b)
    if mask is not None:
        d = d[..., mask]
        b = b[..., mask]
    assert d.size > 0, "no entry left to compare"
    scale = max(np.abs(b).max(), 1e-30)
    return float(d.max() / scale)


def smooth_world(H, W, seed, genotype_update=1):
    """Every potential and gene well above the cutoff, no clip active."""
    rng = np.random.default_rng(seed)
    w = inputs.test_world(H, W, seed=seed, n_blobs=0, genotype_update=genotype_update, dt=0.02)
    w.A = rng.uniform(0.3, 0.6, (3, H, W)).astype(np.float32)
    P = np.empty((3, 15, H, W), np.float32)
    P[0] = rng.uniform(0.1, 0.4, (15, H, W))
    P[1] = rng.uniform(0.03, 0.1, (15, H, W))
    P[2] = rng.uniform(0.1, 1.0, (15, H, W))
    w.P = P
    return w


@pytest.mark.parametrize("H,W,seed,upd", [(40, 56, 201, 1), (48, 64, 202, 0), (33, 70, 203, 1)])
def test_vjp_smooth_world(L, oracle, H, W, seed, upd):
    w = smooth_world(H, W, seed, genotype_update=upd)
    d = oracle.Desc.from_world(w)
    r = oracle.step(d, w.A, w.P)
    assert (r["amb"] == 0).all() and (r["alpha"] == 1).all()
    rng = np.random.default_rng(seed)
    gA1 = rng.standard_normal(w.A.shape).astype(np.float32)
    gP1 = rng.standard_normal(w.P.shape).astype(np.float32)
    gA, gP, gb = _gpu_vjp(L, w, gA1, gP1)
    g = oracle.step_vjp(d, w.A, w.P, gA1, gP1)
    eA, eP, eb = _rel(gA, g["gA"]), _rel(gP, g["gP"]), _rel(gb, g["gbeta"])
    print(f"smooth {H}x{W} upd={upd}: rel err gA {eA:.2e} gP {eP:.2e} gbeta {eb:.2e}")
    assert eA <= TOL_REL and eP <= TOL_REL and eb <= 1e-4


@pytest.mark.parametrize("H,W,seed", [(64, 64, 211), (100, 150, 212), (16, 16, 213)])
def test_vjp_blob_world(L, oracle, H, W, seed):
    """Creatures in empty space: alpha and clips active."""
    w = inputs.test_world(H, W, seed=seed, n_blobs=max(1, H * W // 600))
    d = oracle.Desc.from_world(w)
    rng = np.random.default_rng(seed)
    gA1 = rng.standard_normal(w.A.shape).astype(np.float32)
    gP1 = rng.standard_normal(w.P.shape).astype(np.float32)
    gA, gP, gb = _gpu_vjp(L, w, gA1, gP1)
    g = oracle.step_vjp(d, w.A, w.P, gA1, gP1)
    amb = g["amb"] != 0
    okA = ~_dilate(amb, w.R)
    okP = ~_dilate(amb, 1)
    eA, eP = _rel(gA, g["gA"], okA), _rel(gP, g["gP"], okP)
    print(f"blobs {H}x{W}: ambiguous {int(amb.sum())}, rel err gA {eA:.2e} gP {eP:.2e}")
    assert okA.sum() > 0 and eA <= TOL_REL and eP <= TOL_REL
    if not amb.any():
        assert _rel(gb, g["gbeta"]) <= 1e-4


@pytest.mark.parametrize("conv", [2, 3])
@pytest.mark.parametrize("H,W,seed", [(64, 64, 204), (100, 150, 205)])
def test_vjp_dft_form(L, oracle, H, W, seed, conv):
    """The adjoint of a step whose potentials came from the split-bf16 DFT
    form (the transpose itself is the direct gather), on a smooth world."""
    w = smooth_world(H, W, seed)
    d = oracle.Desc.from_world(w)
    r = oracle.step(d, w.A, w.P)
    assert (r["amb"] == 0).all() and (r["alpha"] == 1).all()
    rng = np.random.default_rng(seed)
    gA1 = rng.standard_normal(w.A.shape).astype(np.float32)
    gP1 = rng.standard_normal(w.P.shape).astype(np.float32)
    gA, gP, gb = _gpu_vjp(L, w, gA1, gP1, conv=conv)
    g = oracle.step_vjp(d, w.A, w.P, gA1, gP1)
    eA, eP, eb = _rel(gA, g["gA"]), _rel(gP, g["gP"]), _rel(gb, g["gbeta"])
    print(f"DFT form {conv} smooth {H}x{W}: rel err gA {eA:.2e} gP {eP:.2e} gbeta {eb:.2e}")
    tol = TOL_REL_DFT if conv == 2 else TOL_REL_DFT_F16
    assert eA <= tol and eP <= tol and eb <= tol


@pytest.mark.parametrize("seed", [231, 232])
def test_vjp_large_world_patch(L, oracle, seed):
    """A 1024^2 world, large enough for the gather's wide tiles (one thread per
    vertical cell pair), with cotangents on a 48 x 48 patch only.  The exact
    gradients then depend only on the state within 2R + 2 of the patch: on a
    torus cropped to the patch +- (2R + 2) the oracle's VJP equals the full
    world's on the patch +- R (gA) and +- 1 (gP), and the shell-height
    gradients are sums over the patch.  Outside the patch +- R the GPU's gA
    and gP must be exactly 0."""
    import dataclasses
    from scipy.ndimage import uniform_filter
    H = W = 1024
    NP = 48
    w = inputs.test_world(H, W, seed=seed, n_blobs=H * W // 600)
    R = w.R
    M = 2 * R + 2
    # the patch on the most matter
    dens = uniform_filter(w.A.sum(0).astype(np.float64), size=NP, mode="wrap")
    cy, cx = np.unravel_index(int(np.argmax(dens)), dens.shape)
    py, px = (cy - NP // 2) % H, (cx - NP // 2) % W
    rng = np.random.default_rng(seed)
    rows_p = (py + np.arange(NP)) % H
    cols_p = (px + np.arange(NP)) % W
    gA1 = np.zeros_like(w.A)
    gP1 = np.zeros_like(w.P)
    gA1[np.ix_(range(3), rows_p, cols_p)] = rng.standard_normal((3, NP, NP))
    gP1[np.ix_(range(3), range(15), rows_p, cols_p)] = rng.standard_normal((3, 15, NP, NP))
    gA, gP, gb = _gpu_vjp(L, w, gA1, gP1)

    # oracle on the cropped torus
    n = NP + 2 * M
    rows = (py - M + np.arange(n)) % H
    cols = (px - M + np.arange(n)) % W
    wc = dataclasses.replace(w, H=n, W=n, A=np.ascontiguousarray(w.A[:, rows][:, :, cols]),
                             P=np.ascontiguousarray(w.P[:, :, rows][:, :, :, cols]))
    d = oracle.Desc.from_world(wc)
    g = oracle.step_vjp(d, wc.A, wc.P, np.ascontiguousarray(gA1[:, rows][:, :, cols]),
                        np.ascontiguousarray(gP1[:, :, rows][:, :, :, cols]))
    amb = g["amb"] != 0
    inner = np.zeros((n, n), bool)
    inner[M:M + NP, M:M + NP] = True
    amb &= inner                       # ambiguity outside the patch does not reach it
    boxA = np.zeros((n, n), bool)
    boxA[M - R:M + NP + R, M - R:M + NP + R] = True
    boxP = np.zeros((n, n), bool)
    boxP[M - 1:M + NP + 1, M - 1:M + NP + 1] = True
    okA = boxA & ~_dilate(amb, R)
    okP = boxP & ~_dilate(amb, 1)
    gA_c = gA[:, rows][:, :, cols]
    gP_c = gP[:, :, rows][:, :, :, cols]
    eA, eP = _rel(gA_c, g["gA"], okA), _rel(gP_c, g["gP"], okP)
    print(f"1024^2 patch at ({py},{px}) seed {seed}: ambiguous {int(amb.sum())}, "
          f"rel err gA {eA:.2e} gP {eP:.2e}")
    assert okA.sum() > 0 and eA <= TOL_REL and eP <= TOL_REL
    if not amb.any():
        eb = _rel(gb, g["gbeta"])
        print(f"  gbeta rel err {eb:.2e}")
        assert eb <= 1e-4
    # nothing outside the reach of the patch
    far = np.ones((H, W), bool)
    far[np.ix_((py - R + np.arange(NP + 2 * R)) % H, (px - R + np.arange(NP + 2 * R)) % W)] = False
    assert (gA[:, far] == 0).all() and (gP[:, :, far] == 0).all()


def test_vjp_gbeta_accumulates(L):
    import torch
    w = smooth_world(32, 32, 221)
    plan = L.Plan(w)
    A, P = dev(w.A), dev(w.P)
    saved = plan.new_saved()
    plan.step(A, P, saved=saved)
    gA1 = torch.randn_like(A)
    _, _, gb1 = plan.backward(A, P, saved, gA1, None)
    gb2 = gb1.clone()
    plan.backward(A, P, saved, gA1, None, gbeta=gb2)
    torch.cuda.synchronize()
    assert torch.allclose(gb2, 2 * gb1, rtol=1e-6, atol=0)
    # entries beyond each kernel's shell count stay untouched
    for k in range(15):
        assert (host(gb1)[k, w.n_shells[k]:] == 0).all()


def test_vjp_deterministic(L):
    w = inputs.test_world(96, 96, seed=222, n_blobs=8)
    rng = np.random.default_rng(1)
    gA1 = rng.standard_normal(w.A.shape).astype(np.float32)
    gP1 = rng.standard_normal(w.P.shape).astype(np.float32)
    a = _gpu_vjp(L, w, gA1, gP1)
    b = _gpu_vjp(L, w, gA1, gP1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_backward_errors(L):
    import torch
    w = inputs.test_world(32, 32, seed=223, n_blobs=1)
    plan = L.Plan(w)
    A, P = dev(w.A), dev(w.P)
    saved = plan.new_saved()
    plan.step(A, P, saved=saved)
    gA1 = torch.zeros_like(A)
    with pytest.raises(L.LeniaError):
        plan.backward(A, P, saved, gA1, None, gA_t=A)        # output aliases an input
    wg = inputs.config1()
    pg = L.Plan(wg)
    Ag = dev(wg.A)
    sv = pg.new_saved()
    pg.step(Ag, None, saved=sv)
    import ctypes
    st = L.lib().lenia_backward(pg.handle, Ag.data_ptr(), Ag.data_ptr(), sv.data_ptr(),
                                Ag.data_ptr(), None, torch.empty_like(Ag).data_ptr(),
                                torch.empty_like(Ag).data_ptr(),
                                torch.zeros(3, device="cuda").data_ptr(), None)
    assert st == L.ERR_UNSUPPORTED


def _oracle_rollout_vjp(oracle, w, T, gAT):
    d = oracle.Desc.from_world(w)
    states = [(w.A.astype(np.float64), w.P.astype(np.float64))]
    for _ in range(T):
        r = oracle.step(d, *states[-1])
        states.append((r["A"], r["P"]))
    gA, gP = gAT.astype(np.float64), np.zeros_like(states[0][1])
    gbeta = np.zeros((15, 3))
    for t in reversed(range(T)):
        g = oracle.step_vjp(d, states[t][0], states[t][1], gA, gP)
        gA, gP = g["gA"], g["gP"]
        gbeta += g["gbeta"]
    return gA, gP, gbeta


@pytest.mark.parametrize("conv,tol", [(1, 1e-4), (2, 6 * TOL_REL_DFT), (3, 6 * TOL_REL_DFT_F16)])
def test_checkpointed_rollout_matches_oracle(L, oracle, conv, tol):
    """T = 6 steps with checkpoints every 4 (an uneven last segment) on a
    smooth world: autograd through LeniaRollout vs the chained FP64 VJP, for
    the direct form and the DFT form (whose per-step bound adds up over the
    six steps)."""
    import torch
    from paper_2304_05639_amd.autograd import rollout
    w = smooth_world(40, 48, 231)
    plan = L.Plan(w, conv=conv)
    A0 = dev(w.A).requires_grad_(True)
    P0 = dev(w.P).requires_grad_(True)
    beta = torch.tensor(w.beta, dtype=torch.float32, device="cuda", requires_grad=True)
    AT, PT = rollout(A0, P0, beta, plan, T=6, ckpt=4)
    rng = np.random.default_rng(3)
    gAT = rng.standard_normal(w.A.shape).astype(np.float32)
    (AT * dev(gAT)).sum().backward()
    gA, gP, gb = _oracle_rollout_vjp(oracle, w, 6, gAT)
    eA, eP, eb = _rel(host(A0.grad), gA), _rel(host(P0.grad), gP), _rel(host(beta.grad), gb)
    print(f"rollout T=6 conv={conv}: rel err gA0 {eA:.2e} gP0 {eP:.2e} gbeta {eb:.2e}")
    assert eA <= tol and eP <= tol and eb <= tol


@pytest.mark.parametrize("T,ckpt", [(8, 4), (3, 8), (5, 1)])
def test_rollout_segment_layouts(L, oracle, T, ckpt):
    """The rollout keeps its last segment from the forward (with the saved
    buffers) and recomputes the others: segments that divide T evenly, a
    single segment (nothing recomputed) and one-step segments all give the
    chained FP64 VJP."""
    import torch
    from paper_2304_05639_amd.autograd import rollout
    w = smooth_world(32, 40, 233)
    plan = L.Plan(w)
    A0 = dev(w.A).requires_grad_(True)
    P0 = dev(w.P).requires_grad_(True)
    beta = torch.tensor(w.beta, dtype=torch.float32, device="cuda", requires_grad=True)
    AT, PT = rollout(A0, P0, beta, plan, T=T, ckpt=ckpt)
    rng = np.random.default_rng(T * 10 + ckpt)
    gAT = rng.standard_normal(w.A.shape).astype(np.float32)
    (AT * dev(gAT)).sum().backward()
    gA, gP, gb = _oracle_rollout_vjp(oracle, w, T, gAT)
    eA, eP, eb = _rel(host(A0.grad), gA), _rel(host(P0.grad), gP), _rel(host(beta.grad), gb)
    print(f"rollout T={T} ckpt={ckpt}: rel err gA0 {eA:.2e} gP0 {eP:.2e} gbeta {eb:.2e}")
    assert eA <= 1e-4 and eP <= 1e-4 and eb <= 1e-4


def test_rollout_forward_same_with_and_without_grad(L):
    """With a gradient wanted, the forward runs its last segment one step at a
    time with the saved buffers; without, as one multi-step call.  The states
    are bitwise the same either way, and a second backward-free rollout too."""
    import torch
    from paper_2304_05639_amd.autograd import rollout
    w = inputs.test_world(64, 80, seed=234, n_blobs=5)
    plan = L.Plan(w)
    beta = torch.tensor(w.beta, dtype=torch.float32, device="cuda")
    A0, P0 = dev(w.A), dev(w.P)
    with torch.no_grad():
        A1, P1 = rollout(A0, P0, beta, plan, T=10, ckpt=4)
    A0g, P0g = dev(w.A).requires_grad_(True), dev(w.P).requires_grad_(True)
    A2, P2 = rollout(A0g, P0g, beta, plan, T=10, ckpt=4)
    assert torch.equal(A1, A2.detach()) and torch.equal(P1, P2.detach())


def _rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def test_c5_gradient_error_report(L, oracle):
    """256^2 world with creatures, T = 64 with checkpoints every 8, MSE loss to
    a random target: relative L2 error of each gradient input (A0, the m and s
    gene planes, the shell heights) against the chained FP64 VJP, for both
    convolution forms.  Over 64 chaotic steps with thresholds (alpha, clips)
    the two trajectories may take different sides of a cutoff, so this is a
    report (printed), held only to being finite."""
    import torch
    from paper_2304_05639_amd.autograd import rollout
    w = inputs.config5()
    T, ckpt = 64, 8
    d = oracle.Desc.from_world(w)
    states = [(w.A.astype(np.float64), w.P.astype(np.float64))]
    for _ in range(T):
        r = oracle.step(d, *states[-1])
        states.append((r["A"], r["P"]))
    n = w.A.size
    gA = 2.0 * (states[-1][0] - w.target.astype(np.float64)) / n
    gP = np.zeros_like(states[0][1])
    gbeta = np.zeros((15, 3))
    for t in reversed(range(T)):
        g = oracle.step_vjp(d, states[t][0], states[t][1], gA, gP)
        gA, gP = g["gA"], g["gP"]
        gbeta += g["gbeta"]
    for conv in (1, 2, 3):
        plan = L.Plan(w, conv=conv)
        A0 = dev(w.A).requires_grad_(True)
        P0 = dev(w.P).requires_grad_(True)
        beta = torch.tensor(w.beta, dtype=torch.float32, device="cuda", requires_grad=True)
        AT, _ = rollout(A0, P0, beta, plan, T, ckpt)
        loss = ((AT - dev(w.target)) ** 2).mean()
        loss.backward()
        torch.cuda.synchronize()
        gpA, gpP, gpb = host(A0.grad), host(P0.grad), host(beta.grad)
        errs = dict(A0=_rel_l2(gpA, gA), m=_rel_l2(gpP[0], gP[0]), s=_rel_l2(gpP[1], gP[1]),
                    beta=_rel_l2(gpb, gbeta))
        print(f"C5 gradients conv={conv}: rel L2 " +
              " ".join(f"{k} {v:.2e}" for k, v in errs.items()))
        assert all(np.isfinite(v) for v in errs.values())


def test_backward_allocation_failure_then_retry(L):
    """The adjoint's three workspaces are allocated on the first call, all or
    none: when the first, second or third allocation fails the call returns
    out-of-memory and leaves the plan as it was, and the next call allocates
    again and gives the same bits as a plan whose first call succeeded."""
    import torch
    w = inputs.test_world(64, 64, seed=231, n_blobs=6)
    rng = np.random.default_rng(231)
    gA1 = rng.standard_normal(w.A.shape).astype(np.float32)
    gP1 = rng.standard_normal(w.P.shape).astype(np.float32)
    ref = _gpu_vjp(L, w, gA1, gP1)
    plan = L.Plan(w)
    A, P = dev(w.A), dev(w.P)
    saved = plan.new_saved()
    plan.step(A, P, saved=saved)
    torch.cuda.synchronize()
    for after in (0, 1, 2):
        L.debug_fail_alloc(after, 1)
        try:
            with pytest.raises(L.LeniaError) as e:
                plan.backward(A, P, saved, dev(gA1), dev(gP1))
            assert e.value.status == L.ERR_OUT_OF_MEMORY
        finally:
            L.debug_fail_alloc(0, 0)
    gA, gP, gb = plan.backward(A, P, saved, dev(gA1), dev(gP1))
    torch.cuda.synchronize()
    for a, b in zip((host(gA), host(gP), host(gb)), ref):
        assert np.array_equal(a, b)
