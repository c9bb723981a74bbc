"""Second, independent FP64 oracle written with plain PyTorch CPU ops.

TEST INFRASTRUCTURE ONLY.  It shares no code with ``lenia_oracle.c`` (or the
HIP library): the kernel is built with tensor ops (differentiable in the shell
heights), convolutions are ``conv2d`` on circularly padded inputs, and
gradients come from autograd.  The two oracles cross-check each other.

Definitions: Section 2.1 (normalized kernels, clipped update), Section 2.2
(alpha mask from the potentials and the genes, strict cutoff eps), Section 2.3
(disk diffusion of the genes divided by the count of above-cutoff neighbours,
clipped), Section 2.4 (localized m, s, h), in the order of Algorithm 2; growth
h*(2*exp(-(u-m)^2/(2 s^2)) - 1) and a time step dt.
"""
from __future__ import annotations

import torch
import torch.nn.functional as F

DT = torch.float64


def kernel_t(R: int, n_shells: int, beta: torch.Tensor) -> torch.Tensor:
    """Normalized ring-shell kernel [(2R+1), (2R+1)], differentiable in beta."""
    ax = torch.arange(-R, R + 1, dtype=DT)
    dy, dx = torch.meshgrid(ax, ax, indexing="ij")
    d2 = dy * dy + dx * dx
    inside = d2 < R * R
    BD = n_shells * torch.sqrt(d2) / R
    shell = torch.floor(BD)
    r = BD - shell
    ok = inside & (r > 0) & (r < 1) & (shell < n_shells)
    rs = torch.where(ok, r, torch.full_like(r, 0.5))
    core = torch.where(ok, torch.exp(4.0 - 1.0 / (rs * (1.0 - rs))), torch.zeros_like(r))
    idx = torch.clamp(shell, 0, n_shells - 1).long()
    heights = beta[:n_shells][idx]
    raw = heights * core
    return raw / raw.sum()


def _circ(x: torch.Tensor, p: int) -> torch.Tensor:
    return F.pad(x, (p, p, p, p), mode="circular")


def step_t(A, P, beta, *, R, n_shells, src, dst, dt, localized, genotype_update,
           m=None, s=None, h=None, eps=0.01, r_diff=1):
    """One step on tensors A [C,H,W], P [3,K,H,W] (float64); returns (A', P')."""
    Cn, H, W = A.shape
    NK = len(src)
    if localized and genotype_update:
        rd = r_diff
        ax = torch.arange(-rd, rd + 1, dtype=DT)
        ddy, ddx = torch.meshgrid(ax, ax, indexing="ij")
        disk = ((ddy * ddy + ddx * ddx) <= rd * rd).to(DT)[None, None]
        flat = P.reshape(3 * NK, 1, H, W)
        num = F.conv2d(_circ(flat, rd), disk)
        cnt = F.conv2d(_circ((flat > eps).to(DT), rd), disk)
        safe = torch.where(cnt > 0, cnt, torch.ones_like(cnt))
        Pd = torch.where(cnt > 0, torch.clamp(num / safe, 0.0, 1.0), torch.zeros_like(num))
        Pd = Pd.reshape(3, NK, H, W)
    else:
        Pd = P
    U = []
    for k in range(NK):
        Kk = kernel_t(R, int(n_shells[k]), beta[k])[None, None]
        a = A[int(src[k])][None, None]
        U.append(F.conv2d(_circ(a, R), Kk)[0, 0])
    U = torch.stack(U)
    if localized and genotype_update:
        alpha = (U > eps).all(0) & (Pd > eps).reshape(3 * NK, H, W).all(0)
    else:
        alpha = torch.ones(H, W, dtype=torch.bool)
    af = alpha.to(DT)
    if localized:
        Pm = Pd * af if genotype_update else Pd
        gm, gs, gh = Pm[0], Pm[1], Pm[2]
    else:
        gm = m[:, None, None].expand(NK, H, W)
        gs = s[:, None, None].expand(NK, H, W)
        gh = h[:, None, None].expand(NK, H, W)
    s_safe = torch.where(alpha[None], gs, torch.ones_like(gs))
    G = gh * (2.0 * torch.exp(-(U - gm) ** 2 / (2.0 * s_safe ** 2)) - 1.0)
    G = torch.where(alpha[None], G, torch.zeros_like(G))
    outs = []
    for c in range(Cn):
        tot = torch.zeros(H, W, dtype=DT)
        for k in range(NK):
            if int(dst[k]) == c:
                tot = tot + G[k]
        outs.append(torch.clamp(A[c] + dt * tot, 0.0, 1.0))
    A1 = torch.stack(outs)
    if localized:
        P1 = Pd * af if genotype_update else P
    else:
        P1 = None
    return A1, P1


def step_np(d, A, P=None):
    """Convenience wrapper taking an oracle ``Desc``-like object and numpy arrays."""
    import numpy as np
    At = torch.tensor(np.asarray(A, np.float64))
    Pt = torch.tensor(np.asarray(P, np.float64)) if P is not None else None
    beta = torch.tensor(np.asarray(d.beta, np.float64))
    kw = _kw(d)
    with torch.no_grad():
        A1, P1 = step_t(At, Pt, beta, **kw)
    return A1.numpy(), (P1.numpy() if P1 is not None else None)


def _kw(d):
    import numpy as np
    kw = dict(R=d.R, n_shells=[int(x) for x in d.n_shells], src=[int(x) for x in d.src],
              dst=[int(x) for x in d.dst], dt=d.dt, localized=d.localized,
              genotype_update=d.genotype_update, eps=d.eps, r_diff=d.r_diff)
    if not d.localized:
        kw.update(m=torch.tensor(np.asarray(d.m, np.float64)),
                  s=torch.tensor(np.asarray(d.s, np.float64)),
                  h=torch.tensor(np.asarray(d.h, np.float64)))
    return kw


def vjp_np(d, A, P, gA_next, gP_next=None):
    """Autograd VJP of one step: returns dict(gA, gP, gbeta[, gm, gs, gh])."""
    import numpy as np
    At = torch.tensor(np.asarray(A, np.float64), requires_grad=True)
    Pt = torch.tensor(np.asarray(P, np.float64), requires_grad=True) if P is not None else None
    beta = torch.tensor(np.asarray(d.beta, np.float64), requires_grad=True)
    kw = _kw(d)
    if not d.localized:
        for key in ("m", "s", "h"):
            kw[key] = kw[key].clone().requires_grad_(True)
    A1, P1 = step_t(At, Pt, beta, **kw)
    loss = (A1 * torch.tensor(np.asarray(gA_next, np.float64))).sum()
    if P1 is not None and gP_next is not None:
        loss = loss + (P1 * torch.tensor(np.asarray(gP_next, np.float64))).sum()
    ins = [At, beta] + ([Pt] if Pt is not None else []) + \
        ([kw["m"], kw["s"], kw["h"]] if not d.localized else [])
    grads = torch.autograd.grad(loss, ins, allow_unused=True)
    z = lambda g, ref: (g if g is not None else torch.zeros_like(ref)).numpy()
    out = dict(gA=z(grads[0], At), gbeta=z(grads[1], beta))
    if Pt is not None:
        out["gP"] = z(grads[2], Pt)
    else:
        out["gm"], out["gs"], out["gh"] = (z(grads[2], kw["m"]), z(grads[3], kw["s"]),
                                           z(grads[4], kw["h"]))
    return out
