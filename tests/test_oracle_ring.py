"""Pins of the oracle's ring-decomposed kernels (Section 2.4) against facts
that do not come from the oracle's own formula: hand-derived ring sizes, the
invariants of a normalized weighted average, reductions to a disk or a single
ring whose offsets are listed by hand, translation equivariance, and a closed
form for a uniform world."""
import os

import numpy as np
import pytest

from oracle import oracle
from paper_2304_05639_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
R, NR = 12, 24


def _desc(w, tau=1e-5):
    return oracle.Desc.from_world(w, tau=tau)


def _genes(H, W, nk=15, r1=0.3, w1=0.1, b1=0.8, r2=0.7, w2=0.1, b2=0.5, m=0.2, s=0.05, h=0.6):
    P = np.empty((9, nk, H, W))
    for i, v in enumerate((r1, w1, b1, r2, w2, b2, m, s, h)):
        P[i] = v
    return P


def test_ring_sizes_match_hand_count():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "ring_sizes_R12_n24.txt"))
            if l.strip() and not l.startswith("#")]
    sizes = oracle.ring_sizes(R, NR)
    for j, n in rows:
        assert sizes[int(j)] == float(n), (j, sizes[int(j)], n)
    # every offset of the open disk |d| < R is in exactly one ring
    disk = sum(1 for y in range(-R, R + 1) for x in range(-R, R + 1) if y * y + x * x < R * R)
    assert sizes.sum() == disk
    assert oracle.ring_of(R, NR, 12, 0) == -1 and oracle.ring_of(R, NR, 0, 11) == 22


def test_constant_world_gives_constant_potential():
    # u_k is a weighted average with non-negative weights: a constant channel
    # gives exactly its value, whatever the (non-uniform) genes
    w = inputs.ring_test_world(40, 36, seed=501, n_blobs=0)
    c = np.array([0.2, 0.55, 0.9])
    A = np.broadcast_to(c[:, None, None], (3, 40, 36)).copy()
    r = oracle.ring_step(_desc(w), A, w.P)
    for k in range(15):
        assert np.abs(r["U"][k] - c[w.src[k]]).max() <= 1e-12


def _narrow(w, j, seed):
    """u for a bump of width 1e-3 centred on j / n_ring (eps lowered to 1e-4 so
    that the diffusion keeps such a width): it weighs ring j by b1 and every
    other ring by exp(-(1/24)^2 / 2e-6) = 0, so u is the mean over ring j (0
    where the ring is empty)."""
    import dataclasses
    w = dataclasses.replace(w, eps=1e-4)
    H, W = w.H, w.W
    rng = np.random.default_rng(seed)
    A = rng.random((3, H, W))
    P = _genes(H, W, r1=j / NR, w1=1e-3, b1=0.7, r2=0.9, w2=1e-3, b2=0.0)
    return A, oracle.ring_step(_desc(w), A, P)


def test_rings_partition_the_disk():
    # sum over rings of (ring size x single-ring mean) is the plain sum of the
    # source channel over the open disk |d| < R: no offset dropped or counted twice
    H, W = 28, 30
    w = inputs.ring_test_world(H, W, seed=502, n_blobs=0)
    sizes = oracle.ring_sizes(R, NR)
    total = None
    for j in range(NR):
        A, r = _narrow(w, j, seed=502)
        part = sizes[j] * r["U"]
        total = part if total is None else total + part
    offs = [(y, x) for y in range(-R, R + 1) for x in range(-R, R + 1) if y * y + x * x < R * R]
    for k in range(15):
        c = w.src[k]
        disk = sum(np.roll(A[c], (-y, -x), axis=(0, 1)) for y, x in offs)
        assert np.abs(total[k] - disk).max() <= 1e-9


# ring members listed by hand: ring 2 = |d| in {1, sqrt 2}, ring 4 = |d| in
# {2, sqrt 5}, ring 5 = |d| = sqrt 8
RING_MEMBERS = {
    2: [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1)],
    4: [(2, 0), (-2, 0), (0, 2), (0, -2), (1, 2), (1, -2), (-1, 2), (-1, -2),
        (2, 1), (2, -1), (-2, 1), (-2, -1)],
    5: [(2, 2), (2, -2), (-2, 2), (-2, -2)],
}


@pytest.mark.parametrize("j", [2, 4, 5])
def test_narrow_bump_selects_one_ring(j):
    w = inputs.ring_test_world(20, 22, seed=503, n_blobs=0)
    A, r = _narrow(w, j, seed=503 + j)
    for k in range(15):
        c = w.src[k]
        mean = sum(np.roll(A[c], (-y, -x), axis=(0, 1)) for y, x in RING_MEMBERS[j]) / len(RING_MEMBERS[j])
        assert np.abs(r["U"][k] - mean).max() <= 1e-12


def test_empty_ring_gives_zero_potential():
    # ring 1 holds no lattice offset: a bump that weighs only it leaves the
    # denominator 0, and u is defined as 0 there
    w = inputs.ring_test_world(20, 22, seed=508, n_blobs=0)
    A, r = _narrow(w, 1, seed=508)
    assert (r["U"] == 0).all()


def test_translation_equivariance():
    w = inputs.ring_test_world(36, 40, seed=504)
    d = _desc(w)
    r0 = oracle.ring_step(d, w.A, w.P)
    sh = (7, -11)
    r1 = oracle.ring_step(d, np.roll(w.A, sh, axis=(1, 2)), np.roll(w.P, sh, axis=(2, 3)))
    assert np.array_equal(np.roll(r0["A"], sh, axis=(1, 2)), r1["A"])
    assert np.array_equal(np.roll(r0["P"], sh, axis=(2, 3)), r1["P"])


def test_empty_world_stays_empty():
    w = inputs.ring_test_world(24, 24, seed=505, n_blobs=0)
    r = oracle.ring_step(_desc(w), np.zeros((3, 24, 24)), w.P)
    assert (r["A"] == 0).all() and (r["P"] == 0).all() and (r["alpha"] == 0).all()


def test_uniform_world_closed_form():
    # constant genes and a constant state: diffusion keeps each gene, u_k is the
    # source value, alpha = 1, and each channel moves by dt times the sum of
    # h (2 exp(-(c - m)^2 / (2 s^2)) - 1) over the kernels writing it
    H, W = 26, 28
    w = inputs.ring_test_world(H, W, seed=506, n_blobs=0)
    c = np.array([0.3, 0.25, 0.35])
    A = np.broadcast_to(c[:, None, None], (3, H, W)).copy()
    m, s, h = 0.28, 0.06, 0.4
    P = _genes(H, W, m=m, s=s, h=h)
    r = oracle.ring_step(_desc(w), A, P)
    assert (r["alpha"] == 1).all()
    assert np.abs(r["P"] - P).max() <= 1e-15
    for ch in range(3):
        g = sum(h * (2 * np.exp(-(c[w.src[k]] - m) ** 2 / (2 * s * s)) - 1)
                for k in range(15) if w.dst[k] == ch)
        want = min(max(c[ch] + w.dt * g, 0.0), 1.0)
        assert np.abs(r["A"][ch] - want).max() <= 1e-15


def test_low_bump_height_closes_alpha():
    # every gene plane takes part in the mask: a bump height at or below eps
    # switches alpha off, so A' = clip01(A) and P' = 0
    H, W = 24, 26
    w = inputs.ring_test_world(H, W, seed=507, n_blobs=0)
    rng = np.random.default_rng(507)
    A = rng.random((3, H, W))
    P = _genes(H, W, b2=0.005)
    r = oracle.ring_step(_desc(w), A, P)
    assert (r["alpha"] == 0).all() and (r["P"] == 0).all()
    assert np.array_equal(r["A"], np.clip(A, 0, 1))


# ---- calibration against the cast kernels (Section 2.4, last paragraph) ------

def _smooth_state(H, W, seed):
    rng = np.random.default_rng(seed)
    return np.stack([inputs.smooth_uniform_field(rng, H, W, 0.0, 1.0, 4.0) for _ in range(3)])


def test_ring_form_converges_to_the_cast_form():
    """The ring form evaluates each kernel function at its ring's inner radius
    j / n_ring instead of at each offset's own radius: an error of first order
    in the ring width.  On smooth states and smooth gene fields the ring
    potentials approach the cast potentials as n_ring grows, by about the
    factor the rings narrow (at least half of it here)."""
    import dataclasses
    H, W = 40, 44
    w = inputs.ring_test_world(H, W, seed=511, n_blobs=0)
    A = _smooth_state(H, W, 512)
    uc = oracle.cast_potentials(_desc(w), A, w.P)
    errs = []
    for n in (24, 96, 384):
        r = oracle.ring_step(_desc(dataclasses.replace(w, n_ring=n)), A, w.P)
        errs.append(float(np.abs(r["U"] - uc).max()))
    assert errs[0] > 1e-6                         # the forms differ at the paper's 24 rings
    assert errs[1] <= errs[0] / 2 and errs[2] <= errs[1] / 2, errs


def _impulse_kernels(w, genes):
    """Normalized kernel of kernel 0 in the ring and the cast form, read back
    from the oracles' potentials of a unit impulse under constant genes: with
    A = delta at x0, u(x) = K(x0 - x).  Returned on the (2R+1)^2 offset grid."""
    H = W = 2 * R + 5
    P = np.broadcast_to(np.asarray(genes, np.float64)[:, None, None, None], (9, 15, H, W)).copy()
    A = np.zeros((3, H, W))
    y0 = x0 = H // 2
    A[w.src[0], y0, x0] = 1.0
    d = oracle.Desc(H, W, 3, 15, w.src, w.dst, R, w.n_shells, w.beta, w.dt, 1, 1, n_ring=NR)
    ur = oracle.ring_step(d, A, P)["U"][0]
    uc = oracle.cast_potentials(d, A, P)[0]
    take = lambda u: np.array([[u[y0 - dy, x0 - dx] for dx in range(-R, R + 1)]
                               for dy in range(-R, R + 1)])
    return take(ur), take(uc)


GENE_SETS = [(0.3, 0.1, 0.8, 0.7, 0.1, 0.5, 0.2, 0.05, 0.6),      # two bumps, wide
             (0.25, 0.05, 1.0, 0.75, 0.05, 0.4, 0.2, 0.05, 0.6),   # narrow bumps
             (0.5, 0.15, 1.0, 0.9, 0.08, 0.2, 0.2, 0.05, 0.6)]     # one wide bump mid-radius


@pytest.mark.parametrize("genes", GENE_SETS)
def test_ring_and_cast_kernels_bound(genes):
    """Both forms are normalized weighted averages over the same disk, so for
    any state u_ring - u_cast = sum_d (Kr(d) - Kc(d)) (A(x + d) - A(x)), at
    most ||Kr - Kc||_1 times the state's spread over the disk.  Checked on a
    smooth state under constant genes, with the two kernels read back from
    the oracles by impulses; both kernels sum to 1 and depend on |d| only."""
    w = inputs.ring_test_world(2 * R + 5, 2 * R + 5, seed=513, n_blobs=0)
    Kr, Kc = _impulse_kernels(w, genes)
    assert abs(Kr.sum() - 1) < 1e-12 and abs(Kc.sum() - 1) < 1e-12
    for K in (Kr, Kc):
        assert np.allclose(K, K.T, atol=1e-15) and np.allclose(K, K[::-1], atol=1e-15)
    l1 = float(np.abs(Kr - Kc).sum())
    H, W = 48, 52
    A = _smooth_state(H, W, 514)
    P = np.broadcast_to(np.asarray(genes, np.float64)[:, None, None, None], (9, 15, H, W)).copy()
    d = oracle.Desc(H, W, 3, 15, w.src, w.dst, R, w.n_shells, w.beta, w.dt, 1, 1, n_ring=NR)
    ur = oracle.ring_step(d, A, P)["U"][0]
    uc = oracle.cast_potentials(d, A, P)[0]
    s = A[w.src[0]]
    spread = np.zeros((H, W))
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            if dy * dy + dx * dx < R * R:
                spread = np.maximum(spread, np.abs(np.roll(s, (-dy, -dx), (0, 1)) - s))
    diff = np.abs(ur - uc)
    assert (diff <= l1 * spread + 1e-12).all()
    print(f"genes {genes[:6]}: ||Kr - Kc||_1 = {l1:.3f}, max |u_ring - u_cast| = {diff.max():.2e} "
          f"(bound {float((l1 * spread).max()):.2e})")


def _anisotropy(K):
    """max over 0 < |k| <= pi/4 of |T(k, 0) - T(k/sqrt2, k/sqrt2)|, T the
    kernel's transfer function sum_d K(d) cos(k . d): how differently plane
    waves of one wavelength (8 cells and longer) along an axis and along a
    diagonal are passed."""
    d = np.arange(-R, R + 1)
    dy, dx = np.meshgrid(d, d, indexing="ij")
    worst = 0.0
    for k in np.linspace(0.01, np.pi / 4, 80):
        ta = float((K * np.cos(k * dx)).sum())
        q = k / np.sqrt(2.0)
        td = float((K * np.cos(q * dx + q * dy)).sum())
        worst = max(worst, abs(ta - td))
    return worst


@pytest.mark.parametrize("genes", GENE_SETS)
def test_ring_form_anisotropy(genes):
    """The anisotropy the ring recombination adds: the axis-against-diagonal
    difference of the transfer function of the ring kernel stays within
    0.02 of the cast kernel's own (the lattice makes both slightly
    anisotropic) at wavelengths of 8 cells and longer."""
    w = inputs.ring_test_world(2 * R + 5, 2 * R + 5, seed=513, n_blobs=0)
    Kr, Kc = _impulse_kernels(w, genes)
    ar, ac = _anisotropy(Kr), _anisotropy(Kc)
    print(f"genes {genes[:6]}: anisotropy ring {ar:.4f}, cast {ac:.4f}")
    assert ar <= ac + 0.02
