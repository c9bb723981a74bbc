"""Pins of the oracle's kernel construction (Section 2.1: normalized kernels;
ring-shell reading of the kernel core) against properties the mathematics fixes."""
import math

import numpy as np
import pytest


def lattice_count(R):
    """Number of integer offsets with 0 < |d| < R, counted by brute force."""
    return sum(1 for a in range(-R, R + 1) for b in range(-R, R + 1) if 0 < a * a + b * b < R * R)


@pytest.mark.parametrize("R,expected", [(12, 436), (13, 516)])
def test_single_shell_support(oracle, R, expected):
    K, Z = oracle.kernel(R, 1, [1.0])
    assert lattice_count(R) == expected
    assert int((K > 0).sum()) == expected
    assert K[R, R] == 0.0                                   # centre tap (r = 0)
    assert Z > 0


@pytest.mark.parametrize("R,B,beta", [(12, 1, [1.0]), (12, 2, [0.3, 0.9]),
                                      (12, 3, [0.5, 1.0, 0.25]), (13, 1, [1.0]),
                                      (5, 3, [1.0, 0.5, 0.7]), (3, 1, [0.4])])
def test_normalized_sum_and_d4(oracle, R, B, beta):
    K, _ = oracle.kernel(R, B, beta)
    assert abs(K.sum() - 1.0) <= 1e-14
    for T in (K.T, K[::-1], K[:, ::-1], np.rot90(K), np.rot90(K, 2), np.rot90(K, 3), K[::-1].T):
        assert np.array_equal(T, K)
    assert (K >= 0).all()
    # every tap at or beyond the radius is zero
    ax = np.arange(-R, R + 1)
    d2 = ax[:, None] ** 2 + ax[None, :] ** 2
    assert (K[d2 >= R * R] == 0).all()


def test_core_peak_is_one(oracle):
    # The core exp(4 - 1/(r(1-r))) peaks at r = 1/2 with value exp(0) = 1: a
    # single shell of radius 12 has r = 1/2 at distance 6.
    for beta in (1.0, 0.37):
        assert oracle.shell_basis(12, 1, 0, 6, 0) == 1.0
        K, Z = oracle.kernel(12, 1, [beta])
        raw = K * Z
        assert raw[12 + 6, 12] == pytest.approx(beta, rel=1e-15, abs=0)
        assert raw.max() == pytest.approx(beta, rel=1e-15, abs=0)
    # three shells of radius 12: shell width 4, peaks at distances 2, 6, 10
    for i, dist in enumerate((2, 6, 10)):
        assert oracle.shell_basis(12, 3, i, 0, dist) == 1.0


def test_core_shape(oracle):
    # symmetric about the shell middle, rising then falling, zero on the edges
    R = 120
    vals = [oracle.shell_basis(R, 1, 0, 0, d) for d in range(0, R + 1)]
    assert vals[0] == 0.0 and vals[R] == 0.0
    for d in range(1, R // 2):
        assert vals[d] == pytest.approx(vals[R - d], rel=1e-12)
        assert vals[d] < vals[d + 1]
    # at r = 1/5 (and 4/5): exp(4 - 1/(0.16)) = exp(-2.25); distance 24 of 120
    assert vals[24] == pytest.approx(math.exp(-2.25), rel=1e-12)


def test_shell_boundaries_are_zero(oracle):
    # B = 3, R = 12: shell edges at distances 4 and 8 carry no weight
    K, _ = oracle.kernel(12, 3, [1.0, 1.0, 1.0])
    for d in (4, 8):
        assert K[12 + d, 12] == 0.0 and K[12, 12 + d] == 0.0
    # heights scale their own shell only
    K1, Z1 = oracle.kernel(12, 3, [1.0, 2.0, 1.0])
    raw0 = K * oracle.kernel(12, 3, [1.0, 1.0, 1.0])[1]
    raw1 = K1 * Z1
    assert raw1[12, 12 + 6] == pytest.approx(2 * raw0[12, 12 + 6], rel=1e-14)
    assert raw1[12, 12 + 2] == pytest.approx(raw0[12, 12 + 2], rel=1e-14)
