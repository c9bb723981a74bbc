"""The algebra of the DFT forms' tile transform, in float64 on the CPU: the
row DFT restricted to columns 0..32 with columns 0 and 32 packed into one
complex column, the column DFT, the packed spectral product, the inverse
column DFT restricted to the output rows, and the half-spectrum inverse row
DFT restricted to the output columns, against numpy's FFT convolution of the
64 x 64 window (the circular convolution that Section 2.1 computes through the
convolution theorem).  This checks the matrices and the packing the kernel is
built from, written out here from their definitions; the GPU parity tests
check the kernel against the oracle."""
import numpy as np
import pytest

DT = 64


def _half_spectrum_conv(X, kt, R, packed=True):
    V = DT - 2 * R
    n = np.arange(DT)
    C = np.cos(2 * np.pi * np.outer(n, n) / DT)
    S = np.sin(2 * np.pi * np.outer(n, n) / DT)
    F1 = np.empty((DT, DT))                       # [C_0..C_31 | (-1)^j, -S_1..-S_31]
    F1[:, :32] = C[:32].T
    F1[:, 32] = np.cos(np.pi * n)
    F1[:, 33:] = -S[1:32].T
    Y = X @ F1
    T = np.block([[C, S], [-S, C]]) @ np.vstack([Y[:, :32], Y[:, 32:]])
    Tc = T[:DT] + 1j * T[DT:]
    K = np.real(np.fft.fft2(kt)) / DT ** 2
    U = Tc * K[:, :32]
    neg = (-n) % DT
    if packed:
        U[:, 0] = Tc[:, 0] * (K[:, 0] + K[:, 32]) / 2 + np.conj(Tc[neg, 0]) * (K[:, 0] - K[:, 32]) / 2
    idx = np.arange(V) + R
    Cv = np.cos(2 * np.pi * np.outer(idx, n) / DT)
    Sv = np.sin(2 * np.pi * np.outer(idx, n) / DT)
    Z = np.block([[Cv, -Sv], [Sv, Cv]]) @ np.vstack([U.real, U.imag])
    th = 2 * np.pi * np.outer(np.arange(32), idx) / DT
    F4 = np.vstack([2 * np.cos(th), -2 * np.sin(th)])
    F4[0] = 1.0
    F4[32] = np.cos(np.pi * idx)
    return np.hstack([Z[:V], Z[V:]]) @ F4


def _ring_kernel(R, rng):
    kt = np.zeros((DT, DT))
    mu = rng.uniform(0.2, 0.8)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            r = np.hypot(dy, dx)
            if r <= R:
                kt[dy % DT, dx % DT] = np.exp(-((r / R - mu) / 0.15) ** 2)
    return kt / kt.sum()


@pytest.mark.parametrize("R", [12, 13])
def test_half_spectrum_tile_convolution(R):
    rng = np.random.default_rng(2304056)
    V = DT - 2 * R
    for _ in range(3):
        X = rng.random((DT, DT))
        kt = _ring_kernel(R, rng)
        ref = np.real(np.fft.ifft2(np.fft.fft2(X) * np.fft.fft2(kt)))[R:R + V, R:R + V]
        got = _half_spectrum_conv(X, kt, R)
        assert np.abs(got - ref).max() <= 1e-13


def test_packed_column_needs_its_own_product():
    """Treating the packed column as an ordinary one (multiplying it by the
    column-0 spectrum alone) is wrong by far more than rounding: the test
    above would catch a kernel that dropped the packed product."""
    rng = np.random.default_rng(7)
    X = rng.random((DT, DT))
    kt = _ring_kernel(12, rng)
    ref = np.real(np.fft.ifft2(np.fft.fft2(X) * np.fft.fft2(kt)))[12:52, 12:52]
    assert np.abs(_half_spectrum_conv(X, kt, 12) - ref).max() <= 1e-13
    assert np.abs(_half_spectrum_conv(X, kt, 12, packed=False) - ref).max() > 1e-4
