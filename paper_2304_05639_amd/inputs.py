"""Seeded synthetic worlds for the multi-channel Lenia step.

This module only draws inputs: cell states, gene fields, shell heights and the
kernel table of the 3-channel / 15-kernel system of Section 2.1 (three
self-kernels per channel, two cross-kernels per channel pair).  It holds none
of the method's arithmetic (no kernel construction, convolution, growth or
update); both the CPU oracle and the HIP library consume its arrays.

The paper names a seed creature whose cell values are not published, so the
worlds here are random blobs with the paper's shapes (3 channels, 15 kernels,
radius 12, localized m/s/h genes).  Draw order within one world is fixed:

  1. per kernel: number of shells B = integers(1, 4), then heights random(B);
  2. gene fields: for p in (m, s, h), for k in 0..14, one smoothed field;
  3. blobs: for each blob y0 = integers(H), x0 = integers(W),
     then values random((3, 24, 24)), stamped with wrap-around, later blobs
     overwriting earlier ones;
  4. (large world only) per-blob genes: for each blob 15 m, 15 s, 15 h,
     stamped into the 48x48 square centred on the blob;
  5. (rollout workload only) the loss target random((3, H, W)).

A smoothed field is i.i.d. N(0,1) noise, blurred on the torus by a Gaussian of
standard deviation 16 cells (side/8 on tori smaller than 128; FP64, FFT), divided by its empirical standard
deviation, mapped through the normal CDF to a uniform marginal and affinely to
[lo, hi], then rounded to float32.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np
import scipy.fft as sfft
from scipy.special import ndtr

SEED_BASE = 2304056390

# Kernel table: k = 0..8 self kernels (source = target = k // 3); k = 9..14 one
# cross kernel per ordered channel pair.
KERNEL_SRC_3CH = (0, 0, 0, 1, 1, 1, 2, 2, 2, 0, 0, 1, 1, 2, 2)
KERNEL_DST_3CH = (0, 0, 0, 1, 1, 1, 2, 2, 2, 1, 2, 0, 2, 0, 1)

GENE_RANGES = {"m": (0.1, 0.4), "s": (0.01, 0.1), "h": (0.0, 1.0)}
# Kernel-function genes of the ring form (two bumps per kernel; the paper gives
# no ranges): an inner and an outer bump, heights above the cutoff.
RING_GENE_RANGES = {"r1": (0.15, 0.45), "w1": (0.05, 0.15), "b1": (0.3, 1.0),
                    "r2": (0.5, 0.85), "w2": (0.05, 0.15), "b2": (0.1, 1.0)}
RING_PARAMS = ("r1", "w1", "b1", "r2", "w2", "b2", "m", "s", "h")
BLOB = 24
C4_SIDES = (128, 192, 256, 384, 512, 768, 1024)


@dataclasses.dataclass
class World:
    """One Lenia world: descriptor fields plus the initial state arrays."""
    H: int
    W: int
    n_channels: int
    n_kernels: int
    src: Tuple[int, ...]
    dst: Tuple[int, ...]
    R: int
    n_shells: np.ndarray          # int32 [k]
    beta: np.ndarray              # float64 [k, 3]; entries >= n_shells are 0
    dt: float
    localized: int
    genotype_update: int
    m: Optional[np.ndarray]       # float64 [k], global mode only
    s: Optional[np.ndarray]
    h: Optional[np.ndarray]
    eps: float
    r_diff: int
    A: np.ndarray                 # float32 [c, H, W]
    P: Optional[np.ndarray]       # float32 [3, k, H, W] (m, s, h planes)
    target: Optional[np.ndarray] = None
    name: str = ""
    n_ring: int = 0               # > 0: ring-decomposed kernels whose bump genes
                                  # are localized too; P is then float32
                                  # [9, k, H, W] (r1, w1, b1, r2, w2, b2, m, s, h)

    @property
    def cells(self) -> int:
        return self.H * self.W


def smooth_uniform_field(rng: np.random.Generator, H: int, W: int,
                         lo: float, hi: float, sigma: float = 16.0) -> np.ndarray:
    z = rng.standard_normal((H, W))
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.rfftfreq(W)[None, :]
    g = np.exp(-2.0 * np.pi ** 2 * sigma ** 2 * (fy ** 2 + fx ** 2))
    y = sfft.irfft2(sfft.rfft2(z, workers=-1) * g, s=(H, W), workers=-1)
    sd = y.std()
    if sd > 0:
        y = y / sd
    u = ndtr(y)
    return (lo + (hi - lo) * u).astype(np.float32)


def _draw_shells(rng: np.random.Generator, n_kernels: int):
    n_shells = np.zeros(n_kernels, np.int32)
    beta = np.zeros((n_kernels, 3), np.float64)
    for k in range(n_kernels):
        b = int(rng.integers(1, 4))
        n_shells[k] = b
        # heights are rounded to float32 so that every consumer sees the same value
        beta[k, :b] = rng.random(b).astype(np.float32)
    return n_shells, beta


def _stamp(dst: np.ndarray, vals: np.ndarray, y0: int, x0: int) -> None:
    """dst[..., (y0+i) % H, (x0+j) % W] = vals[..., i, j] (later writes win)."""
    H, W = dst.shape[-2:]
    h, w = vals.shape[-2:]
    ys = (y0 + np.arange(h)) % H
    xs = (x0 + np.arange(w)) % W
    # sequential row assignment so that self-overlap on tiny tori keeps the last write
    for i in range(h):
        dst[..., ys[i], xs] = vals[..., i, :]


def default_sigma(H: int, W: int) -> float:
    """16 cells, reduced to side/8 on small test tori where a 16-cell blur would
    leave an almost constant field (worlds of side >= 128 always get 16)."""
    return min(16.0, min(H, W) / 8.0)


def localized_world(rng: np.random.Generator, H: int, W: int, n_blobs: int,
                    per_blob_genes: bool = False, with_target: bool = False,
                    R: int = 12, dt: float = 0.2, genotype_update: int = 1,
                    name: str = "", sigma: Optional[float] = None) -> World:
    """3-channel, 15-kernel world with smoothed m/s/h fields and uniform blobs."""
    sig = default_sigma(H, W) if sigma is None else sigma
    nk = 15
    n_shells, beta = _draw_shells(rng, nk)
    P = np.empty((3, nk, H, W), np.float32)
    for pi, p in enumerate(("m", "s", "h")):
        lo, hi = GENE_RANGES[p]
        for k in range(nk):
            P[pi, k] = smooth_uniform_field(rng, H, W, lo, hi, sig)
    A = np.zeros((3, H, W), np.float32)
    corners = []
    for _ in range(n_blobs):
        y0 = int(rng.integers(H))
        x0 = int(rng.integers(W))
        vals = rng.random((3, BLOB, BLOB)).astype(np.float32)
        _stamp(A, vals, y0, x0)
        corners.append((y0, x0))
    if per_blob_genes:
        side = 2 * BLOB
        for (y0, x0) in corners:
            genes = np.empty((3, nk), np.float32)
            for pi, p in enumerate(("m", "s", "h")):
                lo, hi = GENE_RANGES[p]
                genes[pi] = (lo + (hi - lo) * rng.random(nk)).astype(np.float32)
            block = np.broadcast_to(genes[:, :, None, None], (3, nk, side, side))
            _stamp(P, block, y0 + BLOB // 2 - side // 2, x0 + BLOB // 2 - side // 2)
    target = rng.random((3, H, W)).astype(np.float32) if with_target else None
    return World(H=H, W=W, n_channels=3, n_kernels=nk, src=KERNEL_SRC_3CH,
                 dst=KERNEL_DST_3CH, R=R, n_shells=n_shells, beta=beta, dt=dt,
                 localized=1, genotype_update=genotype_update, m=None, s=None,
                 h=None, eps=0.01, r_diff=1, A=A, P=P, target=target, name=name)


def ring_world(rng: np.random.Generator, H: int, W: int, n_blobs: int,
               per_blob_genes: bool = False, R: int = 12, n_ring: int = 24,
               dt: float = 0.2, name: str = "", sigma: Optional[float] = None) -> World:
    """3-channel, 15-kernel world with ring-decomposed kernels: every one of
    the 9 gene types (r1, w1, b1, r2, w2, b2, m, s, h) is a smoothed field per
    kernel, drawn in that order, then uniform blobs as in localized_world."""
    sig = default_sigma(H, W) if sigma is None else sigma
    nk = 15
    n_shells, beta = _draw_shells(rng, nk)   # unused by the ring form; drawn to keep the stream layout
    ranges = dict(RING_GENE_RANGES, **GENE_RANGES)
    P = np.empty((9, nk, H, W), np.float32)
    for pi, p in enumerate(RING_PARAMS):
        lo, hi = ranges[p]
        for k in range(nk):
            P[pi, k] = smooth_uniform_field(rng, H, W, lo, hi, sig)
    A = np.zeros((3, H, W), np.float32)
    corners = []
    for _ in range(n_blobs):
        y0 = int(rng.integers(H))
        x0 = int(rng.integers(W))
        vals = rng.random((3, BLOB, BLOB)).astype(np.float32)
        _stamp(A, vals, y0, x0)
        corners.append((y0, x0))
    if per_blob_genes:
        side = 2 * BLOB
        for (y0, x0) in corners:
            genes = np.empty((9, nk), np.float32)
            for pi, p in enumerate(RING_PARAMS):
                lo, hi = ranges[p]
                genes[pi] = (lo + (hi - lo) * rng.random(nk)).astype(np.float32)
            block = np.broadcast_to(genes[:, :, None, None], (9, nk, side, side))
            _stamp(P, block, y0 + BLOB // 2 - side // 2, x0 + BLOB // 2 - side // 2)
    return World(H=H, W=W, n_channels=3, n_kernels=nk, src=KERNEL_SRC_3CH,
                 dst=KERNEL_DST_3CH, R=R, n_shells=n_shells, beta=beta, dt=dt,
                 localized=1, genotype_update=1, m=None, s=None, h=None, eps=0.01,
                 r_diff=1, A=A, P=P, name=name, n_ring=n_ring)


def ring_test_world(H: int, W: int, seed: int, n_blobs: Optional[int] = None) -> World:
    """A small ring-form world for parity tests (blob density of the 512 case)."""
    rng = np.random.default_rng(seed)
    nb = blobs_for_side(int(np.sqrt(H * W))) if n_blobs is None else n_blobs
    return ring_world(rng, H, W, nb, name=f"ring-{H}x{W}-s{seed}")


def config_ring(H: int = 4096, W: int = 4096, n_blobs: int = 2000) -> World:
    """The 4096x4096 workload (2000 blobs with their own genes) with
    ring-decomposed kernels: 24 rings of the R = 12 disk."""
    rng = np.random.default_rng(SEED_BASE + 6)
    return ring_world(rng, H, W, n_blobs, per_blob_genes=True, name=f"lenia-ring-3ch15k-{H}")


def orbium_like_world(seed: Optional[int] = None, H: int = 64, W: int = 64,
                      patch: int = 20, R: int = 13) -> World:
    """Single-channel, single-kernel world with global genes (m=0.15, s=0.015,
    dt=0.1, one shell of height 1) and a centred uniform patch."""
    rng = np.random.default_rng(SEED_BASE + 1 if seed is None else seed)
    A = np.zeros((1, H, W), np.float32)
    y0 = (H - patch) // 2
    x0 = (W - patch) // 2
    A[0, y0:y0 + patch, x0:x0 + patch] = rng.random((patch, patch)).astype(np.float32)
    return World(H=H, W=W, n_channels=1, n_kernels=1, src=(0,), dst=(0,), R=R,
                 n_shells=np.array([1], np.int32),
                 beta=np.array([[1.0, 0.0, 0.0]]), dt=0.1, localized=0,
                 genotype_update=0, m=np.array([0.15]), s=np.array([0.015]),
                 h=np.array([1.0]), eps=0.01, r_diff=1, A=A, P=None,
                 name=f"global-1ch-{H}x{W}")


# ---- the five standard workloads -------------------------------------------

def config1() -> World:
    """64x64 torus, 1 channel, 1 kernel (R=13), global genes, 100 steps."""
    return orbium_like_world()


def config2() -> World:
    """512x512 torus, 3 channels, 15 kernels, localized genes, 40 blobs."""
    rng = np.random.default_rng(SEED_BASE + 2)
    return localized_world(rng, 512, 512, 40, name="lenia-3ch15k-512")


def config3(H: int = 4096, W: int = 4096, n_blobs: int = 2000) -> World:
    """4096x4096 torus, 2000 blobs each with its own genotype."""
    rng = np.random.default_rng(SEED_BASE + 3)
    return localized_world(rng, H, W, n_blobs, per_blob_genes=True,
                           name=f"lenia-3ch15k-{H}")


def blobs_for_side(side: int) -> int:
    return max(1, int(round(40 * side * side / (512 * 512))))


def config4(n_worlds: int = 256) -> List[World]:
    """Independent worlds of uneven square sides, each seeded separately."""
    seqs = np.random.SeedSequence(SEED_BASE + 4).spawn(n_worlds)
    worlds = []
    for i, sq in enumerate(seqs):
        rng = np.random.default_rng(sq)
        side = C4_SIDES[int(rng.integers(len(C4_SIDES)))]
        worlds.append(localized_world(rng, side, side, blobs_for_side(side),
                                      name=f"batch{i}-{side}"))
    return worlds


def config5() -> World:
    """256x256 torus with a random loss target, for differentiable rollouts."""
    rng = np.random.default_rng(SEED_BASE + 5)
    return localized_world(rng, 256, 256, blobs_for_side(256), with_target=True,
                           name="lenia-3ch15k-256-rollout")


def test_world(H: int, W: int, seed: int, n_blobs: Optional[int] = None,
               R: int = 12, genotype_update: int = 1, dt: float = 0.2) -> World:
    """A small localized world for parity tests (blob density of the 512 case
    unless given)."""
    rng = np.random.default_rng(seed)
    nb = blobs_for_side(int(np.sqrt(H * W))) if n_blobs is None else n_blobs
    return localized_world(rng, H, W, nb, R=R, genotype_update=genotype_update,
                           dt=dt, name=f"test-{H}x{W}-s{seed}")


def band_and_block_world(H: int, W: int, seed: int, band_width: int = 4) -> World:
    """A world whose organic matter has a thin and a thick part: uniform random
    matter in a horizontal band of band_width rows (rows [H/5, H/5 +
    band_width), columns [W/20, 11W/20)) and in a block (rows [H/2, 15H/16),
    columns [5W/8, 15W/16)), nothing elsewhere; genes as in localized_world.
    Draw order: localized_world's with no blobs, then random((3, H, W)) of
    which the band and the block are kept."""
    rng = np.random.default_rng(seed)
    w = localized_world(rng, H, W, 0, name=f"band-block-{H}x{W}-s{seed}")
    mask = np.zeros((H, W), bool)
    mask[H // 5:H // 5 + band_width, W // 20:11 * W // 20] = True
    mask[H // 2:15 * H // 16, 5 * W // 8:15 * W // 16] = True
    w.A = (rng.random((3, H, W)).astype(np.float32) * mask).astype(np.float32)
    return w


# ---- worlds too large to draw on the host -----------------------------------

def large_world(H: int, W: int, seed: int, n_channels: int = 3) -> World:
    """Descriptor of a world drawn on the device by device_state (A and P are
    None here).  3 channels: the 15-kernel table, shells drawn as in
    localized_world from default_rng(seed); 1 channel: the global-gene kernel
    of orbium_like_world."""
    if n_channels == 1:
        w = orbium_like_world(seed=seed, H=8, W=8, patch=4)
        return dataclasses.replace(w, H=H, W=W, A=None, name=f"global-1ch-{H}x{W}")
    rng = np.random.default_rng(seed)
    n_shells, beta = _draw_shells(rng, 15)
    return World(H=H, W=W, n_channels=3, n_kernels=15, src=KERNEL_SRC_3CH,
                 dst=KERNEL_DST_3CH, R=12, n_shells=n_shells, beta=beta, dt=0.2,
                 localized=1, genotype_update=1, m=None, s=None, h=None, eps=0.01,
                 r_diff=1, A=None, P=None, name=f"large-3ch15k-{H}x{W}")


def device_state(w: World, seed: int, block: int = 1024, device: str = "cuda"):
    """(A, P) of world w drawn on the device by torch's generator seeded with
    `seed`, in this order: A uniform in [0, 1) (all channels at once), then for
    p in (m, s, h) and k ascending, P[p, k] uniform in GENE_RANGES[p].  The
    block x block squares with (y // block + x // block) odd are emptied in
    every channel, and the m gene of kernel 0 is 0 on rows [0, block), so that
    tiles without matter and tiles with a dead gene plane both occur.  P is
    None for global genes."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    A = torch.rand((w.n_channels, w.H, w.W), generator=g, device=device)
    yb = (torch.arange(w.H, device=device) // block) % 2
    xb = (torch.arange(w.W, device=device) // block) % 2
    A.masked_fill_((yb[:, None] ^ xb[None, :]).bool(), 0.0)
    if not w.localized:
        return A, None
    P = torch.empty((3, w.n_kernels, w.H, w.W), device=device)
    for pi, p in enumerate(("m", "s", "h")):
        lo, hi = GENE_RANGES[p]
        for k in range(w.n_kernels):
            P[pi, k].uniform_(lo, hi, generator=g)
    P[0, 0, :block, :] = 0.0
    return A, P


# ---- the same recipes drawn on the device -------------------------------------
#
# The benchmark's batched and ring-form workloads hold billions of gene values,
# which the numpy recipe above draws in minutes.  These functions follow the
# same recipe on the device with torch's generator: shells from numpy
# default_rng(seed) as in localized_world, then with a torch generator seeded
# with `seed` the gene fields (i.i.d. N(0,1) in FP64, the circular Gaussian
# blur in FP64 by FFT, divided by the empirical standard deviation, the normal
# CDF, affinely to [lo, hi], rounded to float32; same order), blob corners
# and values (later blobs overwrite earlier ones) and, with per_blob_genes,
# the blobs' own genes.  The values differ from the numpy draws (another
# generator); the distributions are the same.  These worlds are not compared
# with the oracle.

def _device_smooth_field(g, H: int, W: int, lo: float, hi: float, sigma: float, device):
    import math
    import torch
    z = torch.randn((H, W), generator=g, device=device, dtype=torch.float64)
    fy = torch.fft.fftfreq(H, device=device, dtype=torch.float64)[:, None]
    fx = torch.fft.rfftfreq(W, device=device, dtype=torch.float64)[None, :]
    tf = torch.exp(-2.0 * math.pi ** 2 * sigma ** 2 * (fy ** 2 + fx ** 2))
    y = torch.fft.irfft2(torch.fft.rfft2(z) * tf, s=(H, W))
    sd = float(y.std(correction=0))
    if sd > 0:
        y = y / sd
    u = torch.special.ndtr(y)
    return (lo + (hi - lo) * u).to(torch.float32)


def device_world(H: int, W: int, n_blobs: int, seed: int, per_blob_genes: bool = False,
                 ring: bool = False, R: int = 12, dt: float = 0.2, n_ring: int = 24,
                 name: str = "", device: str = "cuda"):
    """A localized_world (or, with ring=True, a ring_world) drawn on the device.
    Returns (World with A = P = None, A, P) with A, P float32 device tensors."""
    import torch
    rng = np.random.default_rng(seed)
    nk = 15
    n_shells, beta = _draw_shells(rng, nk)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) % (1 << 63))
    sig = default_sigma(H, W)
    params = RING_PARAMS if ring else ("m", "s", "h")
    ranges = dict(RING_GENE_RANGES, **GENE_RANGES)
    P = torch.empty((len(params), nk, H, W), dtype=torch.float32, device=device)
    for pi, p in enumerate(params):
        lo, hi = ranges[p]
        for k in range(nk):
            P[pi, k] = _device_smooth_field(g, H, W, lo, hi, sig, device)
    A = torch.zeros((3, H, W), dtype=torch.float32, device=device)
    corners = torch.stack([torch.randint(0, H, (n_blobs,), generator=g, device=device),
                           torch.randint(0, W, (n_blobs,), generator=g, device=device)], 1).cpu()
    vals = torch.rand((n_blobs, 3, BLOB, BLOB), generator=g, device=device)
    ar = torch.arange(BLOB, device=device)
    for b in range(n_blobs):
        y0, x0 = int(corners[b, 0]), int(corners[b, 1])
        ys, xs = (y0 + ar) % H, (x0 + ar) % W
        A[:, ys[:, None], xs[None, :]] = vals[b]
    if per_blob_genes:
        side = 2 * BLOB
        sr = torch.arange(side, device=device)
        lo = torch.tensor([ranges[p][0] for p in params], dtype=torch.float32, device=device)
        hi = torch.tensor([ranges[p][1] for p in params], dtype=torch.float32, device=device)
        genes = lo[None, :, None] + (hi - lo)[None, :, None] * torch.rand(
            (n_blobs, len(params), nk), generator=g, device=device)
        for b in range(n_blobs):
            y0 = int(corners[b, 0]) + BLOB // 2 - side // 2
            x0 = int(corners[b, 1]) + BLOB // 2 - side // 2
            ys, xs = (y0 + sr) % H, (x0 + sr) % W
            P[:, :, ys[:, None], xs[None, :]] = genes[b][:, :, None, None]
    w = World(H=H, W=W, n_channels=3, n_kernels=nk, src=KERNEL_SRC_3CH, dst=KERNEL_DST_3CH,
              R=R, n_shells=n_shells, beta=beta, dt=dt, localized=1, genotype_update=1,
              m=None, s=None, h=None, eps=0.01, r_diff=1, A=None, P=None, name=name,
              n_ring=n_ring if ring else 0)
    return w, A, P


def device_config4(n_worlds: int = 256, device: str = "cuda"):
    """The batched workload drawn on the device: sides as in config4 (the same
    per-world numpy streams decide them), each world from device_world seeded
    by its stream's first 63-bit draw.  Returns a list of (World, A, P)."""
    seqs = np.random.SeedSequence(SEED_BASE + 4).spawn(n_worlds)
    out = []
    for i, sq in enumerate(seqs):
        rng = np.random.default_rng(sq)
        side = C4_SIDES[int(rng.integers(len(C4_SIDES)))]
        seed = int(rng.integers(1 << 62))
        out.append(device_world(side, side, blobs_for_side(side), seed, name=f"batch{i}-{side}",
                                device=device))
    return out


def device_config_ring(H: int = 4096, W: int = 4096, n_blobs: int = 2000, device: str = "cuda"):
    """The 4096^2 ring-form workload (2000 blobs with their own 9 x 15 genes)
    drawn on the device."""
    return device_world(H, W, n_blobs, SEED_BASE + 6, per_blob_genes=True, ring=True,
                        name=f"lenia-ring-3ch15k-{H}", device=device)
