"""The seeded input generators used by the tests that need special layouts:
deterministic, and with the structure their documentation states."""
import numpy as np
import torch

from paper_2304_05639_amd import inputs


def test_band_and_block_world_layout():
    H, W = 96, 192
    a = inputs.band_and_block_world(H, W, seed=821)
    b = inputs.band_and_block_world(H, W, seed=821)
    assert np.array_equal(a.A, b.A) and np.array_equal(a.P, b.P)
    mask = np.zeros((H, W), bool)
    mask[H // 5:H // 5 + 4, W // 20:11 * W // 20] = True
    mask[H // 2:15 * H // 16, 5 * W // 8:15 * W // 16] = True
    assert (a.A[:, ~mask] == 0).all()
    assert (a.A[:, mask] > 0).mean() > 0.99
    for pi, p in enumerate(("m", "s", "h")):
        lo, hi = inputs.GENE_RANGES[p]
        assert a.P[pi].min() >= lo and a.P[pi].max() <= hi
    c = inputs.band_and_block_world(H, W, seed=822)
    assert not np.array_equal(a.A, c.A)


def test_large_world_descriptors():
    w3 = inputs.large_world(100, 90, seed=5)
    assert (w3.n_channels, w3.n_kernels, w3.R, w3.localized, w3.genotype_update) == (3, 15, 12, 1, 1)
    assert w3.A is None and w3.P is None
    assert np.array_equal(w3.n_shells, inputs.large_world(7, 9, seed=5).n_shells)
    w1 = inputs.large_world(100, 90, seed=5, n_channels=1)
    assert (w1.n_channels, w1.n_kernels, w1.R, w1.localized) == (1, 1, 13, 0)
    assert (w1.H, w1.W) == (100, 90) and w1.A is None


def test_device_state_layout():
    w = inputs.large_world(48, 40, seed=9)
    A, P = inputs.device_state(w, seed=3, block=16, device="cpu")
    A2, P2 = inputs.device_state(w, seed=3, block=16, device="cpu")
    assert torch.equal(A, A2) and torch.equal(P, P2)
    y = torch.arange(48)[:, None] // 16
    x = torch.arange(40)[None, :] // 16
    empty = ((y + x) % 2 == 1)
    assert (A[:, empty] == 0).all() and (A[:, ~empty] > 0).float().mean() > 0.99
    assert (P[0, 0, :16] == 0).all() and (P[0, 0, 16:] > 0).all()
    for pi, p in enumerate(("m", "s", "h")):
        lo, hi = inputs.GENE_RANGES[p]
        rows = slice(16, None) if pi == 0 else slice(None)
        assert P[pi, :, rows].min() >= lo and P[pi, :, rows].max() <= hi
    w1 = inputs.large_world(32, 32, seed=9, n_channels=1)
    A1, P1 = inputs.device_state(w1, seed=3, block=8, device="cpu")
    assert A1.shape == (1, 32, 32) and P1 is None


def test_device_world_recipe_on_the_cpu():
    """The device-drawn worlds (benchmark only) follow the numpy recipe: gene
    planes uniform in their ranges with a correlation length of about 16
    cells, 24 x 24 blobs of U[0, 1) values in all channels on an empty
    state, per-blob genes constant on 48 x 48 squares; the ring form draws
    its 9 gene types in the paper's order.  Run with torch on the CPU."""
    import torch
    w, A, P = inputs.device_world(128, 160, 6, seed=7, per_blob_genes=True, device="cpu")
    assert A.dtype == torch.float32 and A.shape == (3, 128, 160) and P.shape == (3, 15, 128, 160)
    assert w.A is None and w.P is None and w.n_ring == 0 and w.genotype_update == 1
    for pi, p in enumerate(("m", "s", "h")):
        lo, hi = inputs.GENE_RANGES[p]
        assert float(P[pi].min()) >= lo and float(P[pi].max()) <= hi
    # smooth fields: neighbouring cells nearly equal, cells 64 apart not
    f = P[0, 3]
    f = (f - f.mean()) / f.std()
    c1 = float((f * torch.roll(f, 1, 1)).mean())
    c64 = float((f * torch.roll(f, 64, 1)).mean())
    assert c1 > 0.95 and abs(c64) < 0.5
    occ = (A > 0).any(0)
    assert 6 * 24 * 24 * 0.5 <= int(occ.sum()) <= 6 * 24 * 24
    assert float(A.max()) < 1.0 and float(A.min()) == 0.0
    wr, Ar, Pr = inputs.device_world(64, 64, 2, seed=8, ring=True, device="cpu")
    assert wr.n_ring == 24 and Pr.shape == (9, 15, 64, 64)
    ranges = dict(inputs.RING_GENE_RANGES, **inputs.GENE_RANGES)
    for pi, p in enumerate(inputs.RING_PARAMS):
        lo, hi = ranges[p]
        assert float(Pr[pi].min()) >= lo and float(Pr[pi].max()) <= hi
