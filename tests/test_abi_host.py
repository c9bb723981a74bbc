"""Host-only checks of the C ABI (no device call): the library loads, exports
every entry point the header declares, validates descriptors with the right
status codes, and builds the same FP64 kernels as the oracle."""
import os
import re

import numpy as np
import pytest

from paper_2304_05639_amd import inputs
from paper_2304_05639_amd import lenia as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"LENIA_API\s+[\w\s\*]+?\b(lenia_\w+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    names = header_symbols()
    assert len(names) >= 12
    lib = L.lib()
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(L.API) == names


def _ok(w, **kw):
    return L.validate(w, **kw)


def test_standard_workloads_validate():
    for w in (inputs.config1(), inputs.test_world(64, 64, seed=1)):
        assert _ok(w) == L.OK, L.last_error()


def _mut(w, **changes):
    import copy
    w2 = copy.copy(w)
    for k, v in changes.items():
        setattr(w2, k, v)
    return w2


@pytest.mark.parametrize("changes", [
    dict(H=0), dict(W=-3), dict(dt=0.0), dict(dt=float("nan")), dict(eps=1.5),
    dict(eps=-0.1), dict(localized=2), dict(genotype_update=3),
    dict(n_shells=np.array([0] * 15, np.int32)), dict(n_shells=np.array([4] * 15, np.int32)),
    dict(beta=np.zeros((15, 3))), dict(beta=np.full((15, 3), -1.0)),
    dict(src=tuple([5] * 15)), dict(R=0), dict(r_diff=-1), dict(H=65536, W=32768),
    dict(eps=0.0), dict(eps=1e-30),
])
def test_invalid_descriptors(changes):
    w = _mut(inputs.test_world(32, 32, seed=2, n_blobs=1), **changes)
    assert _ok(w) == L.ERR_INVALID_ARG, changes


def test_global_mode_needs_positive_s():
    w = inputs.config1()
    w2 = _mut(w, s=np.array([0.0]))
    assert _ok(w2) == L.ERR_INVALID_ARG
    w3 = _mut(w, genotype_update=1)       # gene update without localized genes
    assert _ok(w3) == L.ERR_INVALID_ARG


@pytest.mark.parametrize("changes", [
    dict(R=7), dict(r_diff=2),
    dict(src=(0, 0, 0, 1, 1, 1, 2, 2, 2, 0, 0, 1, 1, 2, 1)),
])
def test_unsupported_descriptors(changes):
    w = _mut(inputs.test_world(32, 32, seed=2, n_blobs=1), **changes)
    assert _ok(w) == L.ERR_UNSUPPORTED, changes
    assert len(L.last_error()) > 0


def test_convolution_forms_validate():
    w = inputs.test_world(32, 32, seed=2, n_blobs=1)
    for conv in (L.CONV_AUTO, L.CONV_DIRECT_F32, L.CONV_DFT_SPLIT_BF16, L.CONV_DFT_SPLIT_F16):
        assert _ok(w, conv=conv) == L.OK, (conv, L.last_error())
    assert _ok(w, conv=4) == L.ERR_INVALID_ARG


def test_unknown_tile_and_flags():
    w = inputs.test_world(32, 32, seed=2, n_blobs=1)
    assert _ok(w, tile=(24, 24)) == L.ERR_UNSUPPORTED
    assert _ok(w, tile=(16, 32)) == L.OK
    b = L.DescBuilder(w)
    b.desc.flags = 0x80
    import ctypes
    assert L.lib().lenia_desc_validate(ctypes.byref(b.desc)) == L.ERR_INVALID_ARG
    b.desc.flags = 0
    b.desc.tile_y = 32
    assert L.lib().lenia_desc_validate(ctypes.byref(b.desc)) == L.ERR_INVALID_ARG


def test_status_strings():
    lib = L.lib()
    for code, name in [(0, b"LENIA_OK"), (1, b"LENIA_ERR_INVALID_ARG"), (4, b"LENIA_ERR_HIP"),
                       (6, b"LENIA_ERR_NONFINITE")]:
        assert lib.lenia_status_str(code) == name


def test_check_finite_flag_validates():
    import ctypes
    w = inputs.test_world(32, 32, seed=2, n_blobs=1)
    b = L.DescBuilder(w, check_finite=True)
    assert b.desc.flags == L.FLAG_CHECK_FINITE
    assert L.lib().lenia_desc_validate(ctypes.byref(b.desc)) == L.OK
    b.desc.flags = L.FLAG_CHECK_FINITE | L.FLAG_AUTOTUNE
    assert L.lib().lenia_desc_validate(ctypes.byref(b.desc)) == L.OK
    b.desc.flags = L.FLAG_CHECK_FINITE | 8
    assert L.lib().lenia_desc_validate(ctypes.byref(b.desc)) == L.ERR_INVALID_ARG


def test_dft_fused_flag_validates():
    import ctypes
    w = inputs.test_world(32, 32, seed=2, n_blobs=1)
    b = L.DescBuilder(w, conv=L.CONV_DFT_SPLIT_F16, dft_fused=True)
    assert b.desc.flags == L.FLAG_DFT_FUSED
    assert L.lib().lenia_desc_validate(ctypes.byref(b.desc)) == L.OK
    b.desc.flags = L.FLAG_DFT_FUSED | L.FLAG_CHECK_FINITE | L.FLAG_AUTOTUNE
    assert L.lib().lenia_desc_validate(ctypes.byref(b.desc)) == L.OK


def test_null_descriptor_rejected():
    assert L.lib().lenia_desc_validate(None) == L.ERR_INVALID_ARG


def test_null_plan_rejected_by_every_entry_point():
    # validated on the host before anything touches a device
    import ctypes
    lib = L.lib()
    evo = L.Evolution(None, 0.0, 0, 0.0, 0)
    assert lib.lenia_step(None, None, None, None, None, 1, None, None) == L.ERR_INVALID_ARG
    assert lib.lenia_step_evolve(None, None, None, None, None, 1, ctypes.byref(evo), None,
                                 None) == L.ERR_INVALID_ARG
    assert lib.lenia_potentials(None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.lenia_backward(None, *([None] * 9)) == L.ERR_INVALID_ARG
    assert lib.lenia_saved_bytes(None) == 0


@pytest.mark.parametrize("seed", [3, 4])
def test_plan_kernels_match_oracle(oracle, seed):
    w = inputs.test_world(32, 32, seed=seed, n_blobs=1)
    for k in range(15):
        K_lib = L.kernel_taps(w, k)
        K_or, _ = oracle.kernel(w.R, int(w.n_shells[k]), w.beta[k])
        assert np.abs(K_lib - K_or).max() <= 1e-17
    w1 = inputs.config1()
    K_lib = L.kernel_taps(w1, 0)
    K_or, _ = oracle.kernel(13, 1, [1.0])
    assert np.abs(K_lib - K_or).max() <= 1e-17


def test_package_import_does_not_load_library():
    import subprocess
    import sys
    code = ("import paper_2304_05639_amd as p, paper_2304_05639_amd.lenia as L, sys;"
            "sys.exit(0 if not L.library_loaded() else 1)")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT)
    assert r.returncode == 0


def test_missing_library_raises(tmp_path, monkeypatch):
    import importlib
    import paper_2304_05639_amd.lenia as mod
    m2 = importlib.reload(mod)
    try:
        monkeypatch.setattr(m2, "LIB_PATH", str(tmp_path / "nope.so"))
        m2._lib = None
        with pytest.raises(ImportError):
            m2.lib()
    finally:
        importlib.reload(mod)


def test_ring_form_descriptors():
    w = inputs.ring_test_world(32, 32, seed=3, n_blobs=1)
    assert _ok(w) == L.OK, L.last_error()
    # the ring form takes its kernels from the genes: shell tables may be NULL
    b = L.DescBuilder(w)
    b.desc.n_shells = None
    b.desc.beta = None
    import ctypes
    assert L.lib().lenia_desc_validate(ctypes.byref(b.desc)) == L.OK, L.last_error()
    assert _ok(_mut(w, n_ring=-1)) == L.ERR_INVALID_ARG
    assert _ok(_mut(w, genotype_update=0)) == L.ERR_INVALID_ARG
    for changes in (dict(n_ring=12), dict(R=13, n_ring=26)):
        assert _ok(_mut(w, **changes)) == L.ERR_UNSUPPORTED, changes
    assert _ok(w, conv=L.CONV_DFT_SPLIT_BF16) == L.ERR_UNSUPPORTED
    assert _ok(w, autotune=True) == L.ERR_UNSUPPORTED
    assert _ok(w, tile=(16, 32)) == L.ERR_UNSUPPORTED
    assert _ok(w, tile=(8, 32)) == L.OK
