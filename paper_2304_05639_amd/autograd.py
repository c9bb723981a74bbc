"""Differentiable Lenia rollouts: a torch.autograd.Function over lenia_step /
lenia_backward with step checkpointing.

Forward runs T steps, keeping (A, P) every `ckpt` steps.  Backward walks the
segments in reverse: it recomputes a segment from its checkpoint while saving
each step's potentials and alpha mask (lenia_step with a `saved` buffer), then
applies lenia_backward step by step.  The last segment is not recomputed:
when a gradient is wanted, the forward runs it step by step with the saved
buffers already, and keeps its states for the backward (the memory the
backward's recomputation of that segment would hold anyway).  Gradients flow to the initial state A0,
the initial gene planes P0 and the kernels' shell heights beta.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lenia


class LeniaRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A0, P0, beta, plan, T: int, ckpt: int = 8):
        if T < 1 or ckpt < 1:
            raise ValueError("T and ckpt must be >= 1")
        want = np.asarray(plan.world.beta, np.float64).reshape(plan.NK, 3)
        have = beta.detach().double().cpu().numpy().reshape(plan.NK, 3)
        if not np.array_equal(want.astype(np.float32), have.astype(np.float32)):
            raise ValueError("beta must equal the shell heights the plan was built with")
        A, P = A0.contiguous(), P0.contiguous()
        ckpts = [(A, P)]
        steps = []
        keep_last = any(ctx.needs_input_grad[:3])
        ctx.last = None
        t = 0
        while t < T:
            n = min(ckpt, T - t)
            if keep_last and t + n >= T:
                # the last segment: each step keeps its potentials and alpha
                states, saved = [(A, P)], [plan.new_saved() for _ in range(n)]
                for i in range(n):
                    A, P = plan.step(A, P, saved=saved[i])
                    states.append((A, P))
                ctx.last = (states, saved)
            else:
                A, P = plan.step(A, P, n_steps=n)
            steps.append(n)
            t += n
            if t < T:
                ckpts.append((A, P))
        ctx.plan = plan
        ctx.steps = steps
        ctx.save_for_backward(*[x for pair in ckpts for x in pair])
        return A, P

    @staticmethod
    def backward(ctx, gA, gP):
        plan = ctx.plan
        flat = ctx.saved_tensors
        ckpts = [(flat[2 * i], flat[2 * i + 1]) for i in range(len(flat) // 2)]
        A_ref = ckpts[0][0]
        gA = torch.zeros_like(A_ref) if gA is None else gA.contiguous()
        gP = torch.zeros_like(ckpts[0][1]) if gP is None else gP.contiguous()
        gbeta = torch.zeros(plan.NK, 3, dtype=torch.float32, device=A_ref.device)
        saved_last = ctx.last[1] if ctx.last is not None else []
        saved = saved_last + [plan.new_saved() for _ in range(max(ctx.steps) - len(saved_last))]
        # two cotangent buffers, used alternately (an output must not alias an input)
        bufs = [(torch.empty_like(gA), torch.empty_like(gP)) for _ in range(2)]
        nb = 0
        for seg in reversed(range(len(ctx.steps))):
            if seg == len(ctx.steps) - 1 and ctx.last is not None:
                states = ctx.last[0]       # kept by the forward, with its saved buffers
            else:
                A, P = ckpts[seg]
                states = [(A, P)]
                for i in range(ctx.steps[seg]):
                    A, P = plan.step(A, P, saved=saved[i])
                    states.append((A, P))
            for i in reversed(range(ctx.steps[seg])):
                oA, oP = bufs[nb]
                nb ^= 1
                gA, gP, _ = plan.backward(states[i][0], states[i][1], saved[i], gA, gP,
                                          gA_t=oA, gP_t=oP, gbeta=gbeta)
        ctx.last = None
        return gA, gP, gbeta.to(ctx.saved_tensors[0].dtype), None, None, None


def rollout(A0, P0, beta, plan, T: int, ckpt: int = 8):
    """(A_T, P_T) after T steps, differentiable in A0, P0 and beta."""
    return LeniaRollout.apply(A0, P0, beta, plan, T, ckpt)
