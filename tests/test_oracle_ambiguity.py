"""Pins of the oracle's ambiguity mask: the cells a GPU parity comparison may
leave out because either side of a cutoff or clip is a correct result.

Section 2.2 makes alpha a strict `> eps` test of every potential and every
diffused gene; Section 2.3 clips the diffusion quotient to [0, 1] and the
update clips the state to [0, 1].  A quantity within tau of such a boundary
may land on either side in FP32, so the oracle flags it:

  bit 0  a potential u_k or a diffused gene P_d within tau of eps
  bit 1  the pre-clip update z or a diffusion quotient q within tau of 0 or 1
  bit 2  (operators iteration) the organic sum sum_k u_k within tau of eps

Each test places values by hand at boundary +- tau/2 and +- 0.9 tau (inside
the band: the bit must be set on exactly the expected cells) and at boundary
+- 1.1 tau and +- 3 tau (outside: no cell may carry it), through closed forms that do not use the
oracle's arithmetic: a constant world gives u_k = kappa exactly (the kernel
sums to 1), a constant gene patch diffuses to itself in its interior, and a
single counted value among uncounted neighbours gives q = their sum.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_2304_05639_amd import inputs

EPS, TAU = 0.01, 1e-5
H, W = 20, 24
DST0 = [k for k in range(15) if inputs.KERNEL_DST_3CH[k] == 0]     # kernels updating channel 0
# inside the band, and outside it; the points at 0.9 and 1.1 tau catch a band
# shrunk or widened by a tenth
INSIDE = (TAU / 2, -TAU / 2, 0.9 * TAU, -0.9 * TAU)
OUTSIDE = (3 * TAU, -3 * TAU, 1.1 * TAU, -1.1 * TAU)


def _desc(w, tau=TAU):
    d = oracle.Desc.from_world(w, tau=tau)
    assert d.eps == EPS and d.tau == tau
    return d


@pytest.fixture(scope="module")
def shell():
    return inputs.test_world(H, W, seed=901, n_blobs=0)


@pytest.fixture(scope="module")
def ring():
    return inputs.ring_test_world(H, W, seed=902, n_blobs=0)


def _const_genes(m=0.3, s=0.05, h=0.5, types=3):
    P = np.empty((types, 15, H, W))
    if types == 9:            # r1, w1, b1, r2, w2, b2: two bumps well above the cutoff
        for i, v in enumerate((0.3, 0.1, 0.8, 0.7, 0.1, 0.5)):
            P[i] = v
    P[types - 3], P[types - 2], P[types - 1] = m, s, h
    return P


def _state(kappa):
    return np.full((3, H, W), kappa)


def _step(form, w, A, P, tau=TAU):
    return (oracle.ring_step if form == "ring" else oracle.step)(_desc(w, tau), A, P)


def _bit(r, b):
    return (r["amb"] >> b) & 1


# ---- bit 0 from the potentials ----------------------------------------------

@pytest.mark.parametrize("form", ["shell", "ring"])
@pytest.mark.parametrize("delta", INSIDE + OUTSIDE)
def test_potential_at_cutoff(shell, ring, form, delta):
    """A constant world kappa = eps + delta: every u_k equals kappa; the genes
    (0.3, 0.05, 0.5) are far from eps and z = kappa + dt sum h G is far from
    the clip bounds."""
    w = ring if form == "ring" else shell
    r = _step(form, w, _state(EPS + delta), _const_genes(types=9 if form == "ring" else 3))
    assert np.abs(r["U"] - (EPS + delta)).max() <= 1e-15
    assert (_bit(r, 0) == (1 if abs(delta) <= TAU else 0)).all()
    assert (_bit(r, 1) == 0).all()
    assert (r["alpha"] == (1 if delta > 0 else 0)).all()       # strict > eps


# ---- bit 0 from a diffused gene ----------------------------------------------

def _patch(value, base, types=3, p=1, k=4):
    """Gene plane (p, k) = `base` with the block rows 5..12, cols 6..15 set to
    `value`; the block's 5-point interior is rows 6..11, cols 7..14."""
    P = _const_genes(types=types)
    P[types - 3 + p, k] = base
    P[types - 3 + p, k, 5:13, 6:16] = value
    interior = np.zeros((H, W), bool)
    interior[6:12, 7:15] = True
    return P, interior


@pytest.mark.parametrize("form", ["shell", "ring"])
@pytest.mark.parametrize("delta", (TAU / 2, 0.9 * TAU, 1.1 * TAU, 3 * TAU))
def test_gene_patch_above_cutoff(shell, ring, form, delta):
    """Inside the patch every disk value is eps + delta, so P_d = eps + delta;
    a cell with j < 5 patch values in its disk averages them with the 0.05
    background: P_d >= 0.05 - far from eps."""
    w = ring if form == "ring" else shell
    P, interior = _patch(EPS + delta, 0.05, types=9 if form == "ring" else 3)
    r = _step(form, w, _state(0.3), P)
    want = interior if delta <= TAU else np.zeros_like(interior)
    assert np.array_equal(_bit(r, 0).astype(bool), want)
    assert (r["alpha"] == 1).all()


@pytest.mark.parametrize("form", ["shell", "ring"])
def test_gene_patch_below_cutoff_is_not_ambiguous(shell, ring, form):
    """A patch at eps - tau/2: no disk value inside counts, so the interior's
    diffused gene is 0 (alpha closes there, unambiguously); border cells
    average only the counted background."""
    w = ring if form == "ring" else shell
    P, interior = _patch(EPS - TAU / 2, 0.05, types=9 if form == "ring" else 3)
    r = _step(form, w, _state(0.3), P)
    assert (_bit(r, 0) == 0).all()
    assert np.array_equal(r["alpha"] == 0, interior)


def _single(a, b, types=3, p=0, k=9, y=9, x=11):
    """Gene plane (p, k) = 0 except a at (y, x) and b at its four neighbours.
    Only a exceeds eps (b <= eps), so at (y, x) the count is 1 and the quotient
    is a + 4 b; a neighbour's disk holds a, b and zeros: q = a + b; every other
    cell counts nothing (P_d = 0, no quotient)."""
    P = _const_genes(types=types)
    pi = types - 3 + p
    P[pi, k] = 0.0
    P[pi, k, y, x] = a
    for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        P[pi, k, y + dy, x + dx] = b
    return P, (y, x)


@pytest.mark.parametrize("form", ["shell", "ring"])
@pytest.mark.parametrize("delta", INSIDE + OUTSIDE)
def test_gene_quotient_at_cutoff_from_mixed_disk(shell, ring, form, delta):
    """q = a + 4 b = eps + delta at one cell, from above and from below."""
    a = 0.05
    b = (EPS + delta - a) / 4
    w = ring if form == "ring" else shell
    P, (y, x) = _single(a, b, types=9 if form == "ring" else 3)
    r = _step(form, w, _state(0.3), P)
    want = np.zeros((H, W), np.uint8)
    if abs(delta) <= TAU:
        want[y, x] = 1
    assert np.array_equal(_bit(r, 0), want)
    assert (_bit(r, 1) == 0).all()


# ---- bit 1 from the diffusion quotient ----------------------------------------

@pytest.mark.parametrize("form", ["shell", "ring"])
@pytest.mark.parametrize("delta", INSIDE + OUTSIDE)
def test_gene_quotient_at_upper_clip(shell, ring, form, delta):
    """A patch of h genes at 1 + delta: the interior's quotient is 1 + delta;
    border quotients average it with the 0.5 background (<= 0.9)."""
    w = ring if form == "ring" else shell
    P, interior = _patch(1.0 + delta, 0.5, types=9 if form == "ring" else 3, p=2, k=7)
    r = _step(form, w, _state(0.3), P)
    want = interior if abs(delta) <= TAU else np.zeros_like(interior)
    assert np.array_equal(_bit(r, 1).astype(bool), want)
    assert (_bit(r, 0) == 0).all()


@pytest.mark.parametrize("form", ["shell", "ring"])
@pytest.mark.parametrize("delta", INSIDE + OUTSIDE)
def test_gene_quotient_at_lower_clip(shell, ring, form, delta):
    """q = a + 4 b = delta at one cell: within tau of the lower clip bound 0
    (and 0.01 away from eps, so bit 0 stays clear)."""
    a = 0.05
    b = (delta - a) / 4
    w = ring if form == "ring" else shell
    P, (y, x) = _single(a, b, types=9 if form == "ring" else 3)
    r = _step(form, w, _state(0.3), P)
    want = np.zeros((H, W), np.uint8)
    if abs(delta) <= TAU:
        want[y, x] = 1
    assert np.array_equal(_bit(r, 1), want)
    assert (_bit(r, 0) == 0).all()


# ---- bit 1 from the pre-clip update --------------------------------------------

@pytest.mark.parametrize("form", ["shell", "ring"])
@pytest.mark.parametrize("bound", [0.0, 1.0])
@pytest.mark.parametrize("delta", INSIDE + OUTSIDE)
def test_update_at_clip_bound(shell, ring, form, bound, delta):
    """Constant world 0.5 (u_k = 0.5 exactly), dt = 0.2, five kernels per
    target channel.  Upper bound: m = 0.5 gives G = h exactly, and h = 0.5 +
    delta on channel 0's kernels gives z_0 = 0.5 + 0.2 * 5 h = 1 + delta.
    Lower bound: m = 0.1, s = 0.02 gives exp(-200) < 2^-53, so G = -h exactly,
    and h = 0.5 - delta gives z_0 = delta.  The other channels' kernels have
    h = 0.3 (z = 0.8 or 0.2)."""
    w = ring if form == "ring" else shell
    assert w.dt == 0.2
    types = 9 if form == "ring" else 3
    if bound == 1.0:
        P = _const_genes(m=0.5, s=0.05, h=0.3, types=types)
        h0 = 0.5 + delta
    else:
        P = _const_genes(m=0.1, s=0.02, h=0.3, types=types)
        h0 = 0.5 - delta
    P[types - 1, DST0] = h0
    r = _step(form, w, _state(0.5), P)
    z = (1.0 + delta) if bound == 1.0 else delta
    assert np.abs(r["A"][0] - min(max(z, 0.0), 1.0)).max() <= 1e-15
    assert (_bit(r, 1) == (1 if abs(delta) <= TAU else 0)).all()
    assert (_bit(r, 0) == 0).all()
    assert (r["alpha"] == 1).all()


# ---- bit 2: the organic sum of the operators iteration ------------------------

@pytest.mark.parametrize("delta", INSIDE + OUTSIDE)
def test_organic_sum_at_cutoff(shell, delta):
    """Constant world kappa = (eps + delta) / 15: the 15 potentials sum to
    eps + delta (each u_k = kappa, far below eps, so bit 0 stays clear)."""
    kappa = (EPS + delta) / 15
    r = oracle.evolve_step(_desc(shell), _state(kappa), _const_genes())
    assert (_bit(r, 2) == (1 if abs(delta) <= TAU else 0)).all()
    assert (_bit(r, 0) == 0).all()
    assert ((r["flags"] >> 1) & 1 == (1 if delta > 0 else 0)).all()


# ---- tau is the band's half-width ------------------------------------------------

def test_band_width_follows_tau(shell):
    """The same eps + 3e-5 world is outside the band at tau = 1e-5 and inside
    at tau = 4e-5, and a cell exactly at eps + tau is inside (inclusive)."""
    P = _const_genes()
    assert (_step("shell", shell, _state(EPS + 3e-5), P, tau=1e-5)["amb"] == 0).all()
    assert (_step("shell", shell, _state(EPS + 3e-5), P, tau=4e-5)["amb"] == 1).all()
    edge = EPS + 2.0 ** -16            # exactly representable offset
    assert (_step("shell", shell, _state(edge), P, tau=2.0 ** -16 * 1.0000001)["amb"] == 1).all()
    assert (_step("shell", shell, _state(edge), P, tau=2.0 ** -16 * 0.999)["amb"] == 0).all()
