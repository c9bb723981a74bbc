"""Shared helpers of the GPU parity tests (GPU path through the C ABI vs the
FP64 oracle on identical FP32 inputs)."""
import numpy as np

TOL_STATE = 1e-5      # per-step max-abs on A' and P' over non-ambiguous cells


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


def compare_step(oracle_res, A1, P1, tol=TOL_STATE):
    """Max-abs errors over cells whose alpha decision is not ambiguous."""
    ok = (oracle_res["amb"] & 1) == 0
    eA = np.abs(A1.astype(np.float64) - oracle_res["A"])[:, ok]
    errA = float(eA.max()) if eA.size else 0.0
    errP = 0.0
    if P1 is not None and oracle_res["P"] is not None:
        eP = np.abs(P1.astype(np.float64) - oracle_res["P"])[:, :, ok]
        errP = float(eP.max()) if eP.size else 0.0
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
