"""Pins of the oracle's operators around a step (Algorithm 2; walls Section
2.7, mutation Section 2.5, penalization Section 2.6): closed forms on uniform
worlds, and the penalizing area against binary morphology from scipy."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import oracle
from paper_2304_05639_amd import inputs


def _uniform(H, W, seed, c=(0.3, 0.25, 0.35), m=0.28, s=0.06, h=0.4):
    w = inputs.test_world(H, W, seed=seed, n_blobs=0)
    A = np.broadcast_to(np.asarray(c)[:, None, None], (3, H, W)).copy()
    P = np.empty((3, 15, H, W))
    P[0], P[1], P[2] = m, s, h
    return w, A, P


def test_matter_only_on_walls_vanishes():
    w = inputs.test_world(40, 48, seed=701, n_blobs=4)
    walls = (w.A.sum(0) > 0).astype(np.uint8)        # every cell with matter is a wall
    r = oracle.evolve_step(oracle.Desc.from_world(w), w.A, w.P, walls=walls)
    assert (r["A"] == 0).all() and (r["P"] == 0).all() and (r["flags"] & 1 == 0).all()


def test_no_operators_is_the_plain_step():
    w = inputs.test_world(36, 44, seed=702, n_blobs=4)
    d = oracle.Desc.from_world(w)
    r = oracle.evolve_step(d, w.A, w.P)
    s = oracle.step(d, w.A, w.P)
    assert np.array_equal(r["A"], s["A"]) and np.array_equal(r["P"], s["P"])
    assert np.array_equal(r["flags"] & 1, s["alpha"])


def test_mutation_raises_the_square():
    # uniform living world: alpha = 1 everywhere and the step keeps the genes,
    # so the mutated plane is the old value plus gamma * delta on the 2s x 2s
    # square (here across the torus seam) and unchanged elsewhere
    H, W, half = 30, 34, 5
    w, A, P = _uniform(H, W, 703)
    d = oracle.Desc.from_world(w)
    ev = dict(mut_p=1, mut_k=7, mut_delta=0.03, mut_y0=2, mut_x0=31)
    r = oracle.evolve_step(d, A, P, gamma_mut=2.0, mut_half=half, event=ev)
    assert (r["flags"] & 1 == 1).all()
    want = P.copy()
    ys = (2 - half + np.arange(2 * half)) % H
    xs = (31 - half + np.arange(2 * half)) % W
    want[1, 7][np.ix_(ys, xs)] += 2.0 * 0.03
    assert np.abs(r["P"] - want).max() <= 1e-15


def test_mutation_outside_alpha_does_nothing():
    H, W = 24, 24
    w, _, P = _uniform(H, W, 704)
    A = np.zeros((3, H, W))
    r = oracle.evolve_step(oracle.Desc.from_world(w), A, P, gamma_mut=5.0, mut_half=4,
                           event=dict(mut_p=0, mut_k=3, mut_delta=0.5, mut_y0=10, mut_x0=10))
    assert (r["P"] == 0).all()


def _disk(r):
    y, x = np.mgrid[-r:r + 1, -r:r + 1]
    return (y * y + x * x) <= r * r


def _wrap_morph(mask, r, op):
    pad = r + 1
    big = np.pad(mask, pad, mode="wrap")
    out = op(big, structure=_disk(r))
    return out[pad:-pad, pad:-pad]


@pytest.mark.parametrize("r_oxy", [2, 4, 7])
def test_penalizing_area_is_an_opening(r_oxy):
    # organic = sum_k u_k > eps; E_pen = the organic set eroded, then dilated,
    # by the r_oxy disk (wrapped on the torus)
    w = inputs.test_world(96, 104, seed=705 + r_oxy, n_blobs=4)
    d = oracle.Desc.from_world(w)
    r = oracle.evolve_step(d, w.A, w.P, gamma_pen=0.2, r_oxy=r_oxy)
    s = oracle.step(d, w.A, w.P)
    organic = s["U"].sum(0) > d.eps
    assert np.array_equal((r["flags"] >> 1) & 1, organic.astype(np.uint8))
    eroded = _wrap_morph(organic, r_oxy, ndimage.binary_erosion)
    opened = _wrap_morph(eroded, r_oxy, ndimage.binary_dilation)
    assert np.array_equal(r["epen"], opened.astype(np.uint8))
    assert 0 < opened.sum() < opened.size


def test_penalization_of_an_all_organic_world():
    H, W = 28, 32
    w, A, P = _uniform(H, W, 709)
    r = oracle.evolve_step(oracle.Desc.from_world(w), A, P, gamma_pen=0.2, r_oxy=3,
                           event=dict(pen_p=0, pen_k=4, pen_delta=0.05))
    assert (r["epen"] == 1).all()
    want = P.copy()
    want[0, 4] += 0.2 * 0.05
    assert np.abs(r["P"] - want).max() <= 1e-15
