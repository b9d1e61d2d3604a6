"""Pins for oracle.fourier (Sec. 3.4.1 Fourier basis, Sec. 6 padded transforms)."""
import numpy as np
import pytest

from oracle import fourier

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


@pytest.mark.parametrize("M", [1, 2, 5, 8, 12, 33])
def test_dft_matches_numpy_fft(M):
    # A library FFT as a third opinion on tiny sizes.
    rng = np.random.default_rng(M)
    u = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    assert np.allclose(fourier.forward(u), np.fft.fft(u) / M, atol=1e-14)
    assert np.allclose(fourier.backward(u), np.fft.ifft(u) * M, atol=1e-13)
    r = u.real
    assert np.allclose(fourier.rforward(r), np.fft.rfft(r) / M, atol=1e-14)


def test_parseval_and_inverse():
    rng = np.random.default_rng(0)
    M = 30
    u = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    uh = fourier.forward(u)
    assert np.isclose((np.abs(u) ** 2).sum() / M, (np.abs(uh) ** 2).sum(), rtol=1e-13)
    assert np.allclose(fourier.backward(uh), u, atol=1e-13)


def test_delta_and_single_mode():
    M = 16
    d = np.zeros(M)
    d[0] = 1.0
    assert np.allclose(fourier.forward(d), np.full(M, 1.0 / M), atol=1e-16)
    x = 2 * np.pi * np.arange(M) / M
    for l in [-8, -3, 0, 5, 7]:
        uh = fourier.forward(np.exp(1j * l * x))
        expect = np.zeros(M, complex)
        expect[l % M] = 1.0
        assert np.allclose(uh, expect, atol=1e-14)
    assert list(fourier.wavenumbers(8)) == [0, 1, 2, 3, -4, -3, -2, -1]
    assert list(fourier.wavenumbers(5)) == [0, 1, 2, -2, -1]


def test_r2c_round_trip_random_16():
    # The R2CBasis(16) round trip on random data shown in Sec. 3.1.
    rng = np.random.default_rng(16)
    u = rng.random(16)
    assert np.allclose(fourier.rbackward(fourier.rforward(u), 16), u, atol=1e-14)
    u = rng.random(15)
    assert np.allclose(fourier.rbackward(fourier.rforward(u), 15), u, atol=1e-14)


def test_periodic_poisson_cos4x():
    # Sec. 3.4.1: u = cos(4x), f = u'' on N = 32 points; u_hat_l = -f_hat_l / l^2 (l != 0).
    N = 32
    x = 2 * np.pi * np.arange(N) / N
    f = -16 * np.cos(4 * x)
    fh = fourier.forward(f)
    k = fourier.wavenumbers(N).astype(float)
    k[0] = 1.0
    uh = -fh / k**2
    uh[0] = 0
    assert np.allclose(fourier.backward(uh).real, np.cos(4 * x), atol=1e-14)


@pytest.mark.parametrize("N", [6, 7, 8])
def test_padded_transforms_match_zero_padded_fft(N):
    # Independent route: explicit zero-padded spectra through numpy.fft.
    rng = np.random.default_rng(N)
    uh = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    Mp = (3 * N) // 2
    l = fourier.wavenumbers(N)
    pad = np.zeros((Mp, Mp), complex)
    pad[np.ix_(l % Mp, l % Mp)] = uh
    ref = np.fft.ifft2(pad) * Mp * Mp
    up = fourier.padded_backward(uh, Mp)
    assert np.allclose(up, ref, atol=1e-12)
    back = np.fft.fft2(up) / (Mp * Mp)
    assert np.allclose(fourier.padded_forward_truncate(up, N), back[np.ix_(l % Mp, l % Mp)], atol=1e-13)
