"""GPU parity of the MFMA DFT-as-GEMM forms (split bf16 or fp16 operands,
FP32 accumulation) against the FP64 oracle.  The potentials carry the form's
rounding (about 16 significant bits per product, four transform stages), so
they are compared with TOL_U; the state after the growth mapping, which can
amplify a potential error by up to dt * max|G'| (24 at s = 0.01, dt = 0.2), is
compared with TOL_STATE_DFT over cells whose alpha decision is not within
the alpha-ambiguity band of the cutoff."""
import numpy as np
import pytest

from paper_2304_05639_amd import inputs

from gpu_helpers import AMB_TAU_DFT, MAX_EXCLUDED, TOL_STATE, TOL_STATE_DFT, check_excluded, dev, host

pytestmark = pytest.mark.gpu

TOL_U = 2e-5
AMB_TAU = AMB_TAU_DFT
# The fp16 split with power-of-two scaled operands keeps about 22 bits per
# product: each operand within 2^-22 of itself, the dropped lo*lo term within
# 2^-22 of the product, so each of the four chained matrix products adds up
# to about 3 * 2^-22 = 7e-7 of the magnitude of its terms, which on a tile of
# unit-scale values is of the order of the potentials themselves: potentials
# within 1e-6 (measured up to 6.3e-7 on a dense 512^2 world).  The state and
# the ambiguity band are the FP32 form's (measured state error up to 5.7e-6).
TOL_U_F16 = 1e-6
TOL_STATE_F16 = TOL_STATE
AMB_TAU_F16 = 1e-5
TOLS = {2: (TOL_U, TOL_STATE_DFT, AMB_TAU), 3: (TOL_U_F16, TOL_STATE_F16, AMB_TAU_F16)}


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_05639_amd import lenia
    lenia.lib()
    return lenia


FORMS = [2, 3]       # CONV_DFT_SPLIT_BF16, CONV_DFT_SPLIT_F16


def _run(L, w, n_steps=1, conv=2):
    import torch
    plan = L.Plan(w, conv=conv)
    assert plan.info().conv == conv
    saved = plan.new_saved() if n_steps == 1 else None
    A1, P1 = plan.step(dev(w.A), dev(w.P) if w.P is not None else None, n_steps=n_steps,
                       saved=saved)
    torch.cuda.synchronize()
    u = host(plan.saved_views(saved)[0]) if saved is not None else None
    return host(A1), (host(P1) if P1 is not None else None), u


@pytest.mark.parametrize("conv", FORMS)
@pytest.mark.parametrize("H,W,seed,R", [(64, 64, 401, 12), (100, 150, 402, 12), (16, 16, 403, 12),
                                        (81, 120, 404, 13), (512, 512, 405, 12)])
def test_dft_potentials_and_state(L, oracle, H, W, seed, R, conv):
    w = inputs.test_world(H, W, seed=seed, n_blobs=max(1, H * W // 600), R=R)
    tol_u, tol_state, tau = TOLS[conv]
    d = oracle.Desc(w.H, w.W, 3, 15, w.src, w.dst, w.R, w.n_shells, w.beta, w.dt, 1, 1,
                    tau=tau)
    A1, P1, u = _run(L, w, conv=conv)
    r = oracle.step(d, w.A, w.P)
    eu = float(np.abs(u - r["U"]).max())
    ok = (r["amb"] & 1) == 0
    check_excluded(~ok, MAX_EXCLUDED)
    eA = float(np.abs(A1 - r["A"])[:, ok].max())
    eP = float(np.abs(P1 - r["P"])[:, :, ok].max())
    print(f"DFT conv={conv} {H}x{W} R={R}: u err {eu:.2e}  A' err {eA:.2e}  P' err {eP:.2e}  "
          f"ambiguous {int((~ok).sum())}")
    assert eu <= tol_u
    assert eA <= tol_state and eP <= tol_state


@pytest.mark.parametrize("conv", FORMS)
def test_dft_global_single_channel(L, oracle, conv):
    w = inputs.config1()
    d = oracle.Desc.from_world(w)
    A1, _, u = _run(L, w, conv=conv)
    r = oracle.step(d, w.A)
    eu = float(np.abs(u - r["U"]).max())
    eA = float(np.abs(A1 - r["A"]).max())
    print(f"DFT conv={conv} global 64x64 R=13: u err {eu:.2e}  A' err {eA:.2e}")
    assert eu <= TOLS[conv][0] and eA <= TOLS[conv][1]


@pytest.mark.parametrize("conv", FORMS)
def test_dft_deterministic_and_multistep(L, conv):
    w = inputs.test_world(128, 96, seed=406, n_blobs=6)
    a = _run(L, w, n_steps=3, conv=conv)
    b = _run(L, w, n_steps=3, conv=conv)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("conv", FORMS)
def test_dft_close_to_direct_form(L, conv):
    """The forms compute the same convolution: the potentials after one step
    differ by the DFT form's rounding only."""
    import torch
    w = inputs.test_world(200, 256, seed=407, n_blobs=20)
    pd = L.Plan(w)
    pf = L.Plan(w, conv=conv)
    sd, sf = pd.new_saved(), pf.new_saved()
    pd.step(dev(w.A), dev(w.P), saved=sd)
    pf.step(dev(w.A), dev(w.P), saved=sf)
    torch.cuda.synchronize()
    ud, uf = host(pd.saved_views(sd)[0]), host(pf.saved_views(sf)[0])
    # each within its own bound of the exact potentials (the direct form's: 2e-6)
    assert np.abs(ud - uf).max() <= TOLS[conv][0] + 2e-6


def test_potentials_entry_point(L, oracle):
    """lenia_potentials: u_k for every kernel, both forms, against the oracle."""
    import torch
    w = inputs.test_world(96, 160, seed=408, n_blobs=10)
    r = oracle.step(oracle.Desc.from_world(w), w.A, w.P)
    for conv, tol in ((L.CONV_DIRECT_F32, 2e-6), (L.CONV_DFT_SPLIT_BF16, TOL_U),
                      (L.CONV_DFT_SPLIT_F16, TOL_U_F16)):
        plan = L.Plan(w, conv=conv)
        U = plan.potentials(dev(w.A))
        torch.cuda.synchronize()
        err = float(np.abs(host(U) - r["U"]).max())
        print(f"potentials conv={conv}: max err {err:.2e}")
        assert err <= tol
    A = dev(w.A)
    assert L.lib().lenia_potentials(plan.handle, A.data_ptr(), A.data_ptr(), None) == \
        L.ERR_INVALID_ARG                      # U must not alias A


# kernel order of the fused step: per source channel, that channel's kernels
KIDX = [0, 1, 2, 9, 10, 3, 4, 5, 11, 12, 6, 7, 8, 13, 14]


@pytest.mark.parametrize("conv", FORMS)
@pytest.mark.parametrize("H,W,seed,R,steps", [(64, 64, 411, 12, 1), (100, 150, 412, 12, 2),
                                              (16, 16, 413, 12, 1), (81, 120, 414, 13, 3),
                                              (512, 512, 415, 12, 1), (40, 200, 416, 12, 4)])
def test_dft_fused_step_matches_two_kernel_step(L, H, W, seed, R, steps, conv):
    """The one-kernel step (no saved buffers) and the two-kernel step
    (potentials through HBM, then the per-cell epilogue; taken when the
    potentials are saved) give identical bits, step after step, on worlds
    whose tiles are ragged, smaller than the window, or wrap several times.
    The worlds hold cells whose alpha fails at a later kernel than the first,
    which the fused step handles by clearing genes it already wrote."""
    import torch
    w = inputs.test_world(H, W, seed=seed, n_blobs=max(1, H * W // 600), R=R)
    pu = L.Plan(w, conv=conv)
    pf = L.Plan(w, conv=conv, dft_fused=True)
    A_u, P_u = dev(w.A), dev(w.P)
    A_f, P_f = dev(w.A), dev(w.P)
    late = 0
    for t in range(steps):
        sv = pu.new_saved()
        A_u, P_u = pu.step(A_u, P_u, saved=sv)
        A_f, P_f = pf.step(A_f, P_f)
        torch.cuda.synchronize()
        for name, x, y in (("A'", host(A_u), host(A_f)), ("P'", host(P_u), host(P_f))):
            diff = x != y
            assert not diff.any(), (f"{name} differs at step {t} in {int(diff.sum())} values "
                                    f"(largest {float(np.abs(x - y).max()):.3g})")
        u = host(pu.saved_views(sv)[0])[KIDX]
        above = u > w.eps
        # cells whose first potential at or below eps is not the first kernel
        first_fail = np.argmin(above, axis=0)
        late += int(((~above).any(axis=0) & (first_fail > 0)).sum())
    print(f"fused vs two-kernel conv={conv} {H}x{W} R={R}: {steps} step(s) identical, "
          f"{late} cell-steps whose alpha fails after the first kernel")
    if H * W >= 64 * 64:        # the 16 x 16 world is one blob, uniformly alive or dead
        assert late > 0


@pytest.mark.parametrize("conv", FORMS)
def test_dft_fused_multistep_against_oracle(L, oracle, conv):
    """Three fused steps in one call against three oracle steps, each oracle
    step starting from the GPU's previous state (teacher forcing), cells of
    ambiguous alpha excluded."""
    import torch
    w = inputs.test_world(120, 136, seed=417, n_blobs=24)
    tol_u, tol_state, tau = TOLS[conv]
    d = oracle.Desc(w.H, w.W, 3, 15, w.src, w.dst, w.R, w.n_shells, w.beta, w.dt, 1, 1, tau=tau)
    plan = L.Plan(w, conv=conv, dft_fused=True)
    A, P = w.A, w.P
    for t in range(3):
        A1, P1 = plan.step(dev(A), dev(P))
        torch.cuda.synchronize()
        A1, P1 = host(A1), host(P1)
        r = oracle.step(d, A, P)
        ok = (r["amb"] & 1) == 0
        check_excluded(~ok, MAX_EXCLUDED)
        eA = float(np.abs(A1 - r["A"])[:, ok].max())
        eP = float(np.abs(P1 - r["P"])[:, :, ok].max())
        print(f"fused conv={conv} t={t}: A' err {eA:.2e}  P' err {eP:.2e}")
        assert eA <= tol_state and eP <= tol_state
        A, P = A1, P1
