"""ctypes binding of liblenia.so (include/lenia.h).

Argument marshalling only: descriptors are packed into ``lenia_desc``, torch
tensors are passed as device pointers, the current torch stream as the HIP
stream.  Every step of the computation runs in the library's HIP kernels; if
the library is missing the first call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblenia.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_OUT_OF_MEMORY, ERR_HIP, ERR_STATE, ERR_NONFINITE = range(7)
CONV_AUTO, CONV_DIRECT_F32, CONV_DFT_SPLIT_BF16, CONV_DFT_SPLIT_F16 = range(4)
FLAG_AUTOTUNE = 1
FLAG_CHECK_FINITE = 2
FLAG_DFT_FUSED = 4

API = ("lenia_desc_validate", "lenia_kernel_taps", "lenia_plan", "lenia_plan_batched",
       "lenia_step", "lenia_step_batched", "lenia_potentials", "lenia_saved_bytes", "lenia_backward",
       "lenia_step_evolve", "lenia_plan_get_info", "lenia_plan_destroy", "lenia_status_str",
       "lenia_last_error", "lenia_debug_fail_alloc", "lenia_backward_noalloc")


class LeniaError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {_status_name(status)}: {detail}")
        self.status = status


class Desc(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("n_channels", C.c_int32),
                ("n_kernels", C.c_int32), ("src", C.POINTER(C.c_int32)),
                ("dst", C.POINTER(C.c_int32)), ("R", C.c_int32),
                ("n_shells", C.POINTER(C.c_int32)), ("beta", C.POINTER(C.c_double)),
                ("dt", C.c_double), ("localized", C.c_int32), ("genotype_update", C.c_int32),
                ("m", C.POINTER(C.c_double)), ("s", C.POINTER(C.c_double)),
                ("h", C.POINTER(C.c_double)), ("eps", C.c_double), ("r_diff", C.c_int32),
                ("conv", C.c_int32), ("tile_y", C.c_int32), ("tile_x", C.c_int32),
                ("flags", C.c_uint32), ("n_ring", C.c_int32)]


class Evolution(C.Structure):
    _fields_ = [("walls", C.c_void_p), ("gamma_mut", C.c_double), ("mut_half", C.c_int32),
                ("gamma_pen", C.c_double), ("r_oxy", C.c_int32)]


class Event(C.Structure):
    _fields_ = [("mut_p", C.c_int32), ("mut_k", C.c_int32), ("mut_delta", C.c_float),
                ("mut_y0", C.c_int32), ("mut_x0", C.c_int32), ("pen_p", C.c_int32),
                ("pen_k", C.c_int32), ("pen_delta", C.c_float)]


class PlanInfo(C.Structure):
    _fields_ = [("conv", C.c_int32), ("tile_y", C.c_int32), ("tile_x", C.c_int32),
                ("n_worlds", C.c_int32), ("cells", C.c_int64), ("workspace_bytes", C.c_size_t),
                ("saved_bytes", C.c_size_t)]


_lib = None


def library_loaded() -> bool:
    return _lib is not None


def lib():
    """Loads liblenia.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.lenia_desc_validate.argtypes = [C.POINTER(Desc)]
        L.lenia_kernel_taps.argtypes = [C.POINTER(Desc), C.c_int32, C.POINTER(C.c_double)]
        L.lenia_plan.argtypes = [C.POINTER(Desc), vp, C.POINTER(vp)]
        L.lenia_plan_batched.argtypes = [C.POINTER(Desc), C.c_int32, vp, C.POINTER(vp)]
        L.lenia_step.argtypes = [vp, vp, vp, vp, vp, C.c_int32, vp, vp]
        L.lenia_step_batched.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.c_int32, vp]
        L.lenia_potentials.argtypes = [vp, vp, vp, vp]
        L.lenia_saved_bytes.argtypes = [vp]
        L.lenia_saved_bytes.restype = C.c_size_t
        L.lenia_backward.argtypes = [vp] + [vp] * 8 + [vp]
        L.lenia_backward_noalloc.argtypes = [vp] + [vp] * 8 + [vp]
        L.lenia_plan_get_info.argtypes = [vp, C.POINTER(PlanInfo)]
        L.lenia_step_evolve.argtypes = [vp, vp, vp, vp, vp, C.c_int32, C.POINTER(Evolution),
                                        C.POINTER(Event), vp]
        L.lenia_plan_destroy.argtypes = [vp]
        L.lenia_status_str.argtypes = [C.c_int]
        L.lenia_status_str.restype = C.c_char_p
        L.lenia_last_error.restype = C.c_char_p
        L.lenia_debug_fail_alloc.argtypes = [C.c_int32, C.c_int32]
        L.lenia_debug_fail_alloc.restype = None
        for name in ("lenia_desc_validate", "lenia_kernel_taps", "lenia_plan",
                     "lenia_plan_batched", "lenia_step", "lenia_step_batched",
                     "lenia_potentials", "lenia_backward", "lenia_backward_noalloc",
                     "lenia_plan_get_info",
                     "lenia_plan_destroy"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def debug_fail_alloc(after: int, count: int) -> None:
    """Test hook: let `after` device allocations of the library through, then
    fail `count` of them (count <= 0: off)."""
    lib().lenia_debug_fail_alloc(int(after), int(count))


def _status_name(s: int) -> str:
    try:
        return lib().lenia_status_str(s).decode()
    except Exception:
        return str(s)


def _check(status: int, where: str) -> None:
    if status != OK:
        raise LeniaError(status, where, lib().lenia_last_error().decode())


class DescBuilder:
    """Packs a world (inputs.World or any object with the same fields) into a
    lenia_desc and keeps the host arrays alive."""

    def __init__(self, w, conv: int = CONV_AUTO, tile: Optional[Sequence[int]] = None,
                 autotune: bool = False, check_finite: bool = False, dft_fused: bool = False):
        nk = int(w.n_kernels)
        self._src = np.ascontiguousarray(w.src, np.int32)
        self._dst = np.ascontiguousarray(w.dst, np.int32)
        self._nsh = np.ascontiguousarray(w.n_shells, np.int32)
        self._beta = np.ascontiguousarray(np.asarray(w.beta, np.float64).reshape(nk, 3))
        z = np.zeros(nk)
        self._m = np.ascontiguousarray(w.m if w.m is not None else z, np.float64)
        self._s = np.ascontiguousarray(w.s if w.s is not None else z, np.float64)
        self._h = np.ascontiguousarray(w.h if w.h is not None else z, np.float64)
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        ty, tx = (tile if tile else (0, 0))
        self.desc = Desc(int(w.H), int(w.W), int(w.n_channels), nk, ip(self._src), ip(self._dst),
                         int(w.R), ip(self._nsh), dp(self._beta), float(w.dt), int(w.localized),
                         int(w.genotype_update), dp(self._m), dp(self._s), dp(self._h),
                         float(w.eps), int(w.r_diff), int(conv), int(ty), int(tx),
                         (FLAG_AUTOTUNE if autotune else 0) |
                         (FLAG_CHECK_FINITE if check_finite else 0) |
                         (FLAG_DFT_FUSED if dft_fused else 0), int(getattr(w, "n_ring", 0)))


def validate(w, **kw) -> int:
    """Host-only descriptor check; returns the lenia_status code."""
    b = DescBuilder(w, **kw)
    return lib().lenia_desc_validate(C.byref(b.desc))


def last_error() -> str:
    return lib().lenia_last_error().decode()


def kernel_taps(w, k: int) -> np.ndarray:
    """The FP64 normalized kernel K~_k the library builds for world w."""
    b = DescBuilder(w)
    S = 2 * int(w.R) + 1
    out = np.zeros((S, S), np.float64)
    _check(lib().lenia_kernel_taps(C.byref(b.desc), int(k), out.ctypes.data_as(C.POINTER(C.c_double))),
           "lenia_kernel_taps")
    return out


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _check_tensor(t, shape, name):
    import torch
    if t is None:
        raise ValueError(f"{name} is required")
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Plan:
    """A single-world plan (lenia_plan)."""

    def __init__(self, world, conv: int = CONV_AUTO, tile=None, autotune: bool = False,
                 stream=None, check_finite: bool = False, dft_fused: bool = False):
        self.world = world
        self._b = DescBuilder(world, conv, tile, autotune, check_finite, dft_fused)
        h = C.c_void_p()
        _check(lib().lenia_plan(C.byref(self._b.desc), C.c_void_p(_stream(stream)), C.byref(h)),
               "lenia_plan")
        self._h = h
        self.C, self.NK, self.H, self.W = (int(world.n_channels), int(world.n_kernels),
                                           int(world.H), int(world.W))
        self.localized = int(world.localized)
        self.update = int(world.genotype_update)
        # gene types per kernel: m, s, h, or the ring form's 9
        self.gene_types = 9 if int(getattr(world, "n_ring", 0)) > 0 else 3

    @property
    def handle(self):
        return self._h

    def info(self) -> PlanInfo:
        i = PlanInfo()
        _check(lib().lenia_plan_get_info(self._h, C.byref(i)), "lenia_plan_get_info")
        return i

    @property
    def saved_bytes(self) -> int:
        return int(lib().lenia_saved_bytes(self._h))

    def new_saved(self):
        import torch
        return torch.empty(self.saved_bytes, dtype=torch.uint8, device="cuda")

    def saved_views(self, saved):
        """(u [NK,H,W] float32, alpha [H,W] uint8) views of a saved buffer."""
        import torch
        n = self.NK * self.H * self.W
        u = saved[: 4 * n].view(torch.float32).view(self.NK, self.H, self.W)
        a = saved[4 * n: 4 * n + self.H * self.W].view(self.H, self.W)
        return u, a

    def step(self, A, P=None, A_out=None, P_out=None, n_steps: int = 1, saved=None, stream=None):
        """Advances n_steps; returns (A_out, P_out) (new tensors unless given)."""
        import torch
        _check_tensor(A, (self.C, self.H, self.W), "A")
        if self.localized:
            _check_tensor(P, (self.gene_types, self.NK, self.H, self.W), "P")
        if A_out is None:
            A_out = torch.empty_like(A)
        if self.update and P_out is None:
            P_out = torch.empty_like(P)
        _check_tensor(A_out, A.shape, "A_out")
        if self.update:
            _check_tensor(P_out, P.shape, "P_out")
        if saved is not None:
            if saved.dtype != torch.uint8 or not saved.is_cuda or saved.numel() < self.saved_bytes:
                raise ValueError("saved must be a CUDA uint8 buffer of saved_bytes bytes")
        _check(lib().lenia_step(self._h, _ptr(A), _ptr(P) if self.localized else None, _ptr(A_out),
                                _ptr(P_out) if self.update else None, int(n_steps),
                                _ptr(saved), C.c_void_p(_stream(stream))), "lenia_step")
        return A_out, (P_out if self.update else P)

    def step_evolve(self, A, P, A_out=None, P_out=None, n_steps: int = 1, walls=None,
                    gamma_mut: float = 0.0, mut_half: int = 8, gamma_pen: float = 0.0,
                    r_oxy: int = 6, events=None, stream=None):
        """n_steps iterations of Algorithm 2 with walls, mutation and penalization
        (lenia_step_evolve); the wall cells of (A, P) are zeroed in place.
        `walls`: uint8 CUDA tensor [H, W] or None; `events`: one dict per step
        (mut_p, mut_k, mut_delta, mut_y0, mut_x0, pen_p, pen_k, pen_delta)."""
        import torch
        _check_tensor(A, (self.C, self.H, self.W), "A")
        _check_tensor(P, (self.gene_types, self.NK, self.H, self.W), "P")
        if A_out is None:
            A_out = torch.empty_like(A)
        if P_out is None:
            P_out = torch.empty_like(P)
        _check_tensor(A_out, A.shape, "A_out")
        _check_tensor(P_out, P.shape, "P_out")
        if walls is not None and (walls.dtype != torch.uint8 or not walls.is_cuda or
                                  not walls.is_contiguous() or tuple(walls.shape) != (self.H, self.W)):
            raise ValueError("walls must be a contiguous uint8 CUDA tensor [H, W]")
        evo = Evolution(_ptr(walls), float(gamma_mut), int(mut_half), float(gamma_pen), int(r_oxy))
        evs = None
        if events is not None:
            evs = (Event * max(1, len(events)))()
            for i, e in enumerate(events):
                for k, v in e.items():
                    setattr(evs[i], k, v)
        _check(lib().lenia_step_evolve(self._h, _ptr(A), _ptr(P), _ptr(A_out), _ptr(P_out),
                                       int(n_steps), C.byref(evo), evs, C.c_void_p(_stream(stream))),
               "lenia_step_evolve")
        return A_out, P_out

    def potentials(self, A, U=None, stream=None):
        """u_k = K~_k * A_src(k) for every kernel: tensor [NK, H, W]."""
        import torch
        _check_tensor(A, (self.C, self.H, self.W), "A")
        if U is None:
            U = torch.empty(self.NK, self.H, self.W, dtype=torch.float32, device=A.device)
        _check_tensor(U, (self.NK, self.H, self.W), "U")
        _check(lib().lenia_potentials(self._h, _ptr(A), _ptr(U), C.c_void_p(_stream(stream))),
               "lenia_potentials")
        return U

    def backward(self, A_t, P_t, saved, gA_next, gP_next, gA_t=None, gP_t=None, gbeta=None,
                 stream=None, noalloc=False):
        """VJP of one step; returns (gA_t, gP_t, gbeta) (gbeta accumulated).
        noalloc: lenia_backward_noalloc (static workspace, no allocation)."""
        import torch
        _check_tensor(A_t, (self.C, self.H, self.W), "A_t")
        _check_tensor(P_t, (3, self.NK, self.H, self.W), "P_t")
        _check_tensor(gA_next, (self.C, self.H, self.W), "gA_next")
        if gP_next is not None:
            _check_tensor(gP_next, (3, self.NK, self.H, self.W), "gP_next")
        if gA_t is None:
            gA_t = torch.empty_like(A_t)
        if gP_t is None:
            gP_t = torch.empty_like(P_t)
        if gbeta is None:
            gbeta = torch.zeros(self.NK, 3, dtype=torch.float32, device=A_t.device)
        _check_tensor(gbeta, (self.NK, 3), "gbeta")
        fn = lib().lenia_backward_noalloc if noalloc else lib().lenia_backward
        _check(fn(self._h, _ptr(A_t), _ptr(P_t), _ptr(saved), _ptr(gA_next), _ptr(gP_next),
                  _ptr(gA_t), _ptr(gP_t), _ptr(gbeta), C.c_void_p(_stream(stream))),
               "lenia_backward_noalloc" if noalloc else "lenia_backward")
        return gA_t, gP_t, gbeta

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lenia_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedPlan:
    """Many independent worlds stepped together (lenia_plan_batched)."""

    def __init__(self, worlds, tile=None, autotune: bool = False, stream=None):
        self.worlds = list(worlds)
        self._bs = [DescBuilder(w, CONV_AUTO, tile, autotune) for w in self.worlds]
        arr = (Desc * len(self._bs))(*[b.desc for b in self._bs])
        self._arr = arr
        h = C.c_void_p()
        _check(lib().lenia_plan_batched(arr, len(self._bs), C.c_void_p(_stream(stream)), C.byref(h)),
               "lenia_plan_batched")
        self._h = h

    def info(self) -> PlanInfo:
        i = PlanInfo()
        _check(lib().lenia_plan_get_info(self._h, C.byref(i)), "lenia_plan_get_info")
        return i

    def step(self, As, Ps, n_steps: int = 1, stream=None):
        """Advances every world in place by n_steps."""
        n = len(self.worlds)
        if len(As) != n or (Ps is not None and len(Ps) != n):
            raise ValueError("one A (and P) tensor per world")
        for w, A, P in zip(self.worlds, As, Ps if Ps is not None else [None] * n):
            _check_tensor(A, (w.n_channels, w.H, w.W), "A")
            if w.localized:
                _check_tensor(P, (3, w.n_kernels, w.H, w.W), "P")
        pa = (C.c_void_p * n)(*[_ptr(a) for a in As])
        pp = (C.c_void_p * n)(*[_ptr(p) for p in Ps]) if Ps is not None else None
        _check(lib().lenia_step_batched(self._h, pa, pp, int(n_steps), C.c_void_p(_stream(stream))),
               "lenia_step_batched")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lenia_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
