"""Python front end of the FP64 CPU oracle (``lenia_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the HIP library or its binding.  Takes
plain numpy arrays (any float dtype; promoted to float64) and returns float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lenia_oracle.c")
LIB = os.path.join(HERE, "liblenia_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        up = C.POINTER(C.c_uint8)
        L.oracle_shell_basis.restype = C.c_double
        L.oracle_shell_basis.argtypes = [C.c_int] * 5
        L.oracle_kernel.restype = C.c_double
        L.oracle_kernel.argtypes = [C.c_int, C.c_int, dp, dp]
        common = [C.c_int, C.c_int, C.c_int, C.c_int, ip, ip, C.c_int, dp, C.c_double,
                  C.c_int, dp, dp, dp, C.c_int, C.c_double, C.c_int, C.c_double, dp, dp]
        L.oracle_step.restype = C.c_int
        L.oracle_step.argtypes = common + [dp, dp, dp, up, up]
        L.oracle_step_vjp.restype = C.c_int
        L.oracle_step_vjp.argtypes = common + [dp, dp, dp, dp, dp, dp, dp, dp, up]
        L.oracle_beta_grad.restype = C.c_int
        L.oracle_beta_grad.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_ring_of.restype = C.c_int
        L.oracle_ring_of.argtypes = [C.c_int] * 4
        L.oracle_ring_sizes.restype = None
        L.oracle_ring_sizes.argtypes = [C.c_int, C.c_int, dp]
        L.oracle_evolve_step.restype = C.c_int
        L.oracle_evolve_step.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, ip, ip, C.c_int, dp,
                                         C.c_double, C.c_double, C.c_int, C.c_double, up,
                                         C.c_double, C.c_int, C.c_double, C.c_int, C.c_int,
                                         C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.c_double, dp, dp, up, up, up]
        L.oracle_cast_potentials.restype = C.c_int
        L.oracle_cast_potentials.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, ip, C.c_int,
                                             C.c_double, C.c_int, dp, dp, dp]
        L.oracle_ring_step.restype = C.c_int
        L.oracle_ring_step.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, ip, ip, C.c_int, C.c_int,
                                       C.c_double, C.c_double, C.c_int, C.c_double, dp, dp, dp, dp,
                                       dp, up, up]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def shell_basis(R: int, B: int, i: int, dy: int, dx: int) -> float:
    return lib().oracle_shell_basis(R, B, i, dy, dx)


def kernel(R: int, n_shells: int, beta: Sequence[float]):
    """Normalized kernel on the (2R+1)^2 offset grid and its raw sum Z."""
    S = 2 * R + 1
    K = np.zeros((S, S), np.float64)
    b = _d(np.asarray(beta, np.float64)[:n_shells] if len(beta) else [0.0])
    Z = lib().oracle_kernel(R, n_shells, _p(b), _p(K))
    return K, Z


def kernels(R: int, n_shells, beta) -> np.ndarray:
    """Stack of normalized kernels [k][2R+1][2R+1]."""
    return np.stack([kernel(R, int(n_shells[k]), beta[k])[0] for k in range(len(n_shells))])


class Desc:
    """Plain parameter bundle for the oracle (mirrors a world's descriptor)."""

    def __init__(self, H, W, n_channels, n_kernels, src, dst, R, n_shells, beta, dt,
                 localized, genotype_update, m=None, s=None, h=None, eps=0.01,
                 r_diff=1, tau=1e-5, n_ring=0):
        self.H, self.W, self.C, self.NK = int(H), int(W), int(n_channels), int(n_kernels)
        self.src = np.ascontiguousarray(src, np.int32)
        self.dst = np.ascontiguousarray(dst, np.int32)
        self.R = int(R)
        self.n_shells = np.asarray(n_shells, np.int32)
        self.beta = np.asarray(beta, np.float64)
        self.dt = float(dt)
        self.localized = int(localized)
        self.genotype_update = int(genotype_update)
        z = np.zeros(self.NK)
        self.m = _d(m if m is not None else z)
        self.s = _d(s if s is not None else z)
        self.h = _d(h if h is not None else z)
        self.eps, self.r_diff, self.tau = float(eps), int(r_diff), float(tau)
        self.n_ring = int(n_ring)   # > 0: ring-decomposed kernels from the genes (ring_step)
        self.K = _d(kernels(self.R, self.n_shells, self.beta))

    @classmethod
    def from_world(cls, w, tau=1e-5):
        return cls(w.H, w.W, w.n_channels, w.n_kernels, w.src, w.dst, w.R, w.n_shells,
                   w.beta, w.dt, w.localized, w.genotype_update, w.m, w.s, w.h,
                   w.eps, w.r_diff, tau, getattr(w, "n_ring", 0))

    def _args(self):
        return [self.H, self.W, self.C, self.NK, _p(self.src, C.c_int), _p(self.dst, C.c_int),
                self.R, _p(self.K), self.dt, self.localized, _p(self.m), _p(self.s),
                _p(self.h), self.genotype_update, self.eps, self.r_diff, self.tau]


def step(d: Desc, A, P=None):
    """One step.  Returns dict(A, P, U, alpha, amb) as float64 / uint8 arrays."""
    A = _d(A).reshape(d.C, d.H, d.W)
    Pin = _d(P).reshape(3, d.NK, d.H, d.W) if d.localized else None
    A1 = np.empty_like(A)
    P1 = np.empty_like(Pin) if d.localized else None
    U = np.empty((d.NK, d.H, d.W))
    alpha = np.empty((d.H, d.W), np.uint8)
    amb = np.empty((d.H, d.W), np.uint8)
    rc = lib().oracle_step(*d._args(), _p(A), _p(Pin), _p(A1), _p(P1), _p(U),
                           _p(alpha, C.c_uint8), _p(amb, C.c_uint8))
    if rc != 0:
        raise MemoryError("oracle_step failed")
    return dict(A=A1, P=P1, U=U, alpha=alpha, amb=amb)


def rollout(d: Desc, A, P=None, steps: int = 1):
    A = _d(A)
    P = _d(P) if P is not None else None
    for _ in range(steps):
        r = step(d, A, P)
        A, P = r["A"], r["P"]
    return A, P


def step_vjp(d: Desc, A, P, gA_next, gP_next=None):
    """VJP of one step; returns dict(gA, gP, gK, gm, gs, gh, gbeta, amb)."""
    A = _d(A).reshape(d.C, d.H, d.W)
    Pin = _d(P).reshape(3, d.NK, d.H, d.W) if d.localized else None
    gAn = _d(gA_next).reshape(d.C, d.H, d.W)
    gPn = (_d(gP_next).reshape(3, d.NK, d.H, d.W) if gP_next is not None
           else np.zeros((3, d.NK, d.H, d.W))) if d.localized else None
    gA = np.empty_like(A)
    gP = np.empty_like(Pin) if d.localized else None
    S = 2 * d.R + 1
    gK = np.empty((d.NK, S, S))
    gm = np.zeros(d.NK); gs = np.zeros(d.NK); gh = np.zeros(d.NK)
    amb = np.empty((d.H, d.W), np.uint8)
    rc = lib().oracle_step_vjp(*d._args(), _p(A), _p(Pin), _p(gAn), _p(gPn), _p(gA), _p(gP),
                               _p(gK), _p(gm), _p(gs), _p(gh), _p(amb, C.c_uint8))
    if rc != 0:
        raise MemoryError("oracle_step_vjp failed")
    gbeta = np.zeros((d.NK, 3))
    for k in range(d.NK):
        gbeta[k, :d.n_shells[k]] = beta_grad(d.R, int(d.n_shells[k]), d.beta[k], gK[k])
    return dict(gA=gA, gP=gP, gK=gK, gm=gm, gs=gs, gh=gh, gbeta=gbeta, amb=amb)


def beta_grad(R: int, B: int, beta, gK) -> np.ndarray:
    out = np.zeros(B)
    b = _d(np.asarray(beta, np.float64)[:B])
    g = _d(gK)
    rc = lib().oracle_beta_grad(R, B, _p(b), _p(g), _p(out))
    if rc != 0:
        raise MemoryError("oracle_beta_grad failed")
    return out


def ring_of(R: int, n_ring: int, dy: int, dx: int) -> int:
    """Ring index of an offset (Section 2.4), -1 outside |d| < R."""
    return lib().oracle_ring_of(R, n_ring, dy, dx)


def ring_sizes(R: int, n_ring: int) -> np.ndarray:
    """Number of lattice offsets in each ring."""
    out = np.zeros(n_ring)
    lib().oracle_ring_sizes(R, n_ring, _p(out))
    return out


def ring_step(d: Desc, A, P):
    """One step with ring-decomposed localized kernels (Section 2.4): genes
    P[9][NK][H][W] in the order r1, w1, b1, r2, w2, b2, m, s, h.  Returns
    dict(A, P, U, alpha, amb) as float64 / uint8 arrays."""
    if d.n_ring <= 0:
        raise ValueError("ring_step needs n_ring > 0")
    A = _d(A).reshape(d.C, d.H, d.W)
    Pin = _d(P).reshape(9, d.NK, d.H, d.W)
    A1 = np.empty_like(A)
    P1 = np.empty_like(Pin)
    U = np.empty((d.NK, d.H, d.W))
    alpha = np.empty((d.H, d.W), np.uint8)
    amb = np.empty((d.H, d.W), np.uint8)
    rc = lib().oracle_ring_step(d.H, d.W, d.C, d.NK, _p(d.src, C.c_int), _p(d.dst, C.c_int), d.R,
                                d.n_ring, d.dt, d.eps, d.r_diff, d.tau, _p(A), _p(Pin), _p(A1),
                                _p(P1), _p(U), _p(alpha, C.c_uint8), _p(amb, C.c_uint8))
    if rc != 0:
        raise MemoryError("oracle_ring_step failed")
    return dict(A=A1, P=P1, U=U, alpha=alpha, amb=amb)


def cast_potentials(d: Desc, A, P):
    """The cast form of the localized kernels (Section 2.4): each cell's
    two-bump kernel function evaluated at every offset's own radius,
    normalized over the disk, summed directly.  P[9][NK][H][W] as for
    ring_step.  Returns U[NK][H][W]."""
    A = _d(A).reshape(d.C, d.H, d.W)
    Pin = _d(P).reshape(9, d.NK, d.H, d.W)
    U = np.empty((d.NK, d.H, d.W))
    rc = lib().oracle_cast_potentials(d.H, d.W, d.C, d.NK, _p(d.src, C.c_int), d.R, d.eps,
                                      d.r_diff, _p(A), _p(Pin), _p(U))
    if rc != 0:
        raise MemoryError("oracle_cast_potentials failed")
    return U


def evolve_step(d: Desc, A, P, walls=None, gamma_mut=0.0, mut_half=8, gamma_pen=0.0, r_oxy=6,
                event=None):
    """One iteration of Algorithm 2 with its operators (Sections 2.5-2.7) around
    the shell-form step: walls on the input, the step, the penalizing area,
    mutation, penalization.  `event` holds the iteration's random draws:
    mut_p, mut_k, mut_delta, mut_y0, mut_x0, pen_p, pen_k, pen_delta.
    Returns dict(A, P, flags, epen, amb) (flags: bit 0 alpha, bit 1 organic)."""
    ev = dict(mut_p=0, mut_k=0, mut_delta=0.0, mut_y0=0, mut_x0=0, pen_p=0, pen_k=0,
              pen_delta=0.0)
    if event:
        ev.update(event)
    A = _d(A).reshape(d.C, d.H, d.W).copy()
    P = _d(P).reshape(3, d.NK, d.H, d.W).copy()
    w = None if walls is None else np.ascontiguousarray(walls, np.uint8)
    flags = np.empty((d.H, d.W), np.uint8)
    epen = np.empty((d.H, d.W), np.uint8)
    amb = np.empty((d.H, d.W), np.uint8)
    rc = lib().oracle_evolve_step(d.H, d.W, d.C, d.NK, _p(d.src, C.c_int), _p(d.dst, C.c_int), d.R,
                                  _p(d.K), d.dt, d.eps, d.r_diff, d.tau, _p(w, C.c_uint8),
                                  float(gamma_mut), int(mut_half), float(gamma_pen), int(r_oxy),
                                  int(ev["mut_p"]), int(ev["mut_k"]), float(ev["mut_delta"]),
                                  int(ev["mut_y0"]), int(ev["mut_x0"]), int(ev["pen_p"]),
                                  int(ev["pen_k"]), float(ev["pen_delta"]), _p(A), _p(P),
                                  _p(flags, C.c_uint8), _p(epen, C.c_uint8), _p(amb, C.c_uint8))
    if rc != 0:
        raise MemoryError("oracle_evolve_step failed")
    return dict(A=A, P=P, flags=flags, epen=epen, amb=amb)


def ring_rollout(d: Desc, A, P, steps: int):
    A = _d(A)
    P = _d(P)
    for _ in range(steps):
        r = ring_step(d, A, P)
        A, P = r["A"], r["P"]
    return A, P


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (0 leaves them)."""
    lib().oracle_set_threads(int(n))


def threads() -> int:
    n = os.environ.get("OMP_NUM_THREADS")
    return int(n) if n else len(os.sched_getaffinity(0))
