"""Shared helpers of the GPU parity tests (GPU path through the C ABI vs the
FP64 oracle on identical FP32 inputs)."""
import numpy as np

TOL_STATE = 1e-5      # per-step max-abs on A' and P' over non-ambiguous cells
# split-bf16 DFT form: the state after the growth mapping (a potential error of
# 2e-5 amplified by up to dt max|G'| = 24), and the alpha-ambiguity band (above
# the form's potential error)
TOL_STATE_DFT = 5e-4
AMB_TAU_DFT = 2e-5
# A comparison must compare something: at most this fraction of the cells may
# be left out as ambiguous.  On the test worlds the oracle flags at most 0.7%
# of the cells at tau = 1e-5 and 1.1% at tau = 2e-5 (bit 0, and for the
# operators the 2 r_oxy neighbourhood of bit 2); a 48 x 48 window of a large
# world may hold more of them locally.
MAX_EXCLUDED = 0.02
MAX_EXCLUDED_WINDOW = 0.05


def dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x, np.float32), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def gpu_step(plan, A, P, n_steps=1, saved=None):
    """One call of lenia_step from host FP32 arrays; returns host arrays."""
    import torch
    At = dev(A)
    Pt = dev(P) if P is not None else None
    A1, P1 = plan.step(At, Pt, n_steps=n_steps, saved=saved)
    torch.cuda.synchronize()
    return host(A1), (host(P1) if P1 is not None else None)


def check_excluded(excluded, max_excluded):
    """At least one cell is compared, and at most max_excluded of them left out."""
    n, n_ex = excluded.size, int(excluded.sum())
    assert n_ex < n, f"every one of the {n} cells is excluded: nothing compared"
    assert n_ex <= max_excluded * n, \
        f"{n_ex} of {n} cells excluded as ambiguous (bound {max_excluded:.0%})"


def compare_step(oracle_res, A1, P1, tol=TOL_STATE, max_excluded=MAX_EXCLUDED):
    """Max-abs errors over cells whose alpha decision is not ambiguous."""
    ok = (oracle_res["amb"] & 1) == 0
    check_excluded(~ok, max_excluded)
    errA = float(np.abs(A1.astype(np.float64) - oracle_res["A"])[:, ok].max())
    errP = 0.0
    if P1 is not None and oracle_res["P"] is not None:
        errP = float(np.abs(P1.astype(np.float64) - oracle_res["P"])[:, :, ok].max())
    n_amb = int((~ok).sum())
    assert errA <= tol, f"A' max-abs error {errA:.3e} > {tol} ({n_amb} ambiguous cells)"
    assert errP <= tol, f"P' max-abs error {errP:.3e} > {tol} ({n_amb} ambiguous cells)"
    return errA, errP, n_amb


def window(arr, y0, x0, h, w):
    """arr[..., y0:y0+h, x0:x0+w] with wrap-around on the last two axes."""
    H, W = arr.shape[-2:]
    ys = (y0 + np.arange(h)) % H
    xs = (x0 + np.arange(w)) % W
    return np.take(np.take(arr, ys, axis=-2), xs, axis=-1)


def dilate(mask, r):
    """Cells within distance r (disk, on the torus) of a True cell."""
    H, W = mask.shape
    out = np.zeros_like(mask)
    ys, xs = np.nonzero(mask)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dy * dy + dx * dx <= r * r:
                out[(ys + dy) % H, (xs + dx) % W] = True
    return out


def compare_evolve(r, A1, P1, r_oxy, tol, max_excluded=MAX_EXCLUDED):
    """Max-abs errors of an operators iteration, over cells whose alpha decision
    is not ambiguous and that lie farther than 2 r_oxy from a cell whose
    organic-matter sum is within tau of eps (the penalizing area may differ
    there)."""
    amb = r["amb"]
    bad = ((amb & 1) != 0) | dilate((amb & 4) != 0, 2 * r_oxy)
    ok = ~bad
    check_excluded(bad, max_excluded)
    eA = float(np.abs(A1.astype(np.float64) - r["A"])[:, ok].max())
    eP = float(np.abs(P1.astype(np.float64) - r["P"])[:, :, ok].max())
    assert eA <= tol and eP <= tol, (eA, eP, int(bad.sum()))
    return eA, eP, int(bad.sum())


def device_window(t, y0, x0, h, w):
    """Host copy of t[..., y0:y0+h, x0:x0+w] of a device tensor, with
    wrap-around on the last two axes (gathered on the device)."""
    import torch
    H, W = t.shape[-2:]
    ys = torch.arange(y0, y0 + h, device=t.device) % H
    xs = torch.arange(x0, x0 + w, device=t.device) % W
    return t.index_select(t.dim() - 2, ys).index_select(t.dim() - 1, xs).cpu().numpy()
