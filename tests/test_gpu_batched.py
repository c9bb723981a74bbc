"""Batched worlds of uneven sizes (lenia_plan_batched / lenia_step_batched,
one launch per step over the work list, replayed from a HIP graph): every world of a
batch must equal the same world stepped alone with the same tile, bit for bit,
and one world checked against the FP64 oracle."""
import os

import numpy as np
import pytest

from paper_2304_05639_amd import inputs

from gpu_helpers import compare_step, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_05639_amd import lenia
    lenia.lib()
    return lenia


def _worlds():
    sizes = [(64, 64), (96, 128), (128, 128), (32, 160), (200, 72), (16, 16), (256, 192)]
    return [inputs.test_world(h, w, seed=300 + i, n_blobs=max(1, h * w // 600))
            for i, (h, w) in enumerate(sizes)]


@pytest.mark.parametrize("n_steps", [1, 2, 3, 6])
def test_batched_equals_single(L, n_steps):
    import torch
    worlds = _worlds()
    bp = L.BatchedPlan(worlds)
    tile = (bp.info().tile_y, bp.info().tile_x)
    As = [dev(w.A) for w in worlds]
    Ps = [dev(w.P) for w in worlds]
    bp.step(As, Ps, n_steps=n_steps)
    torch.cuda.synchronize()
    for w, A, P in zip(worlds, As, Ps):
        sp = L.Plan(w, tile=tile)
        a, p = sp.step(dev(w.A), dev(w.P), n_steps=n_steps)
        torch.cuda.synchronize()
        assert torch.equal(a, A) and torch.equal(p, P), (w.name, n_steps)


@pytest.mark.parametrize("n_steps", [19, 20])
def test_batched_long_call_equals_single_steps(L, n_steps):
    """A batched call of many steps equals, for every world, a chain of
    single-step calls (which keep every gene write), bitwise: from the third
    step of a call a tile that takes the alpha = 0 shortcut skips rewriting
    gene planes its output buffer already holds as 0."""
    import torch
    worlds = _worlds()
    bp = L.BatchedPlan(worlds)
    tile = (bp.info().tile_y, bp.info().tile_x)
    As = [dev(w.A) for w in worlds]
    Ps = [dev(w.P) for w in worlds]
    bp.step(As, Ps, n_steps=n_steps)
    torch.cuda.synchronize()
    for w, A, P in zip(worlds, As, Ps):
        sp = L.Plan(w, tile=tile)
        a, p = dev(w.A), dev(w.P)
        for _ in range(n_steps):
            a, p = sp.step(a, p)
        torch.cuda.synchronize()
        assert torch.equal(a, A) and torch.equal(p, P), (w.name, n_steps)


def test_batched_many_tiles_equals_single(L):
    """More than 8 runs of 512 work items, so that blocks map to items through
    the XCD run permutation and its tail: still every world bit for bit."""
    import torch
    sizes = [(512, 512), (512, 512), (512, 512), (512, 512), (200, 264), (96, 64)]
    worlds = [inputs.test_world(h, w, seed=320 + i, n_blobs=max(1, h * w // 2000))
              for i, (h, w) in enumerate(sizes)]
    bp = L.BatchedPlan(worlds, tile=(8, 32))
    assert bp.info().tile_y == 8 and bp.info().tile_x == 32
    As = [dev(w.A) for w in worlds]
    Ps = [dev(w.P) for w in worlds]
    bp.step(As, Ps, n_steps=2)
    torch.cuda.synchronize()
    for w, A, P in zip(worlds, As, Ps):
        a, p = L.Plan(w, tile=(8, 32)).step(dev(w.A), dev(w.P), n_steps=2)
        torch.cuda.synchronize()
        assert torch.equal(a, A) and torch.equal(p, P), w.name


def test_batched_graph_replay_and_pointer_change(L):
    """Repeated calls replay the captured graph; new buffers re-capture it."""
    import torch
    worlds = _worlds()[:4]
    bp = L.BatchedPlan(worlds)
    As = [dev(w.A) for w in worlds]
    Ps = [dev(w.P) for w in worlds]
    for _ in range(3):
        bp.step(As, Ps, n_steps=2)
    As2 = [dev(w.A) for w in worlds]
    Ps2 = [dev(w.P) for w in worlds]
    bp.step(As2, Ps2, n_steps=6)
    torch.cuda.synchronize()
    for A, P, A2, P2 in zip(As, Ps, As2, Ps2):
        assert torch.equal(A, A2) and torch.equal(P, P2)


def test_batched_world_vs_oracle(L, oracle):
    import torch
    worlds = _worlds()
    bp = L.BatchedPlan(worlds)
    As = [dev(w.A) for w in worlds]
    Ps = [dev(w.P) for w in worlds]
    bp.step(As, Ps, n_steps=1)
    torch.cuda.synchronize()
    for i in (0, 4, 5):
        w = worlds[i]
        r = oracle.step(oracle.Desc.from_world(w), w.A, w.P)
        compare_step(r, host(As[i]), host(Ps[i]))


def test_batched_autotune(L, tmp_path, monkeypatch):
    import torch
    monkeypatch.setenv("LENIA_TUNE_CACHE", str(tmp_path / "tune.txt"))
    worlds = _worlds()[:3]
    bp = L.BatchedPlan(worlds, autotune=True)
    t1 = (bp.info().tile_y, bp.info().tile_x)
    assert os.path.exists(tmp_path / "tune.txt")
    bp2 = L.BatchedPlan(worlds, autotune=True)     # served from the cache
    assert (bp2.info().tile_y, bp2.info().tile_x) == t1
    sp = L.Plan(worlds[0], autotune=True)
    assert (sp.info().tile_y, sp.info().tile_x) in [(16, 32), (32, 32), (8, 32), (16, 64), (8, 64),
                                                    (4, 64)]
    As = [dev(w.A) for w in worlds]
    Ps = [dev(w.P) for w in worlds]
    bp.step(As, Ps, n_steps=2)
    torch.cuda.synchronize()
    a, p = L.Plan(worlds[1], tile=t1).step(dev(worlds[1].A), dev(worlds[1].P), n_steps=2)
    torch.cuda.synchronize()
    assert torch.equal(a, As[1]) and torch.equal(p, Ps[1])


def test_batched_errors(L):
    w = _worlds()[:2]
    bp = L.BatchedPlan(w)
    with pytest.raises(ValueError):
        bp.step([dev(w[0].A)], [dev(w[0].P)])
    with pytest.raises(L.LeniaError):
        L.BatchedPlan([w[0], inputs.config1()])       # mixed gene modes / tables
