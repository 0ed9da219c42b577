"""Pins of the oracle's own DFT and frequency window (Sec. 3.1 eq. frequencies, Sec. 3.2)."""
import numpy as np
import pytest

from oracle.fourier import fft3, ifft3, labels, paper_window, shifted_wavevector


@pytest.mark.parametrize("shape", [(4, 6, 5), (8, 1, 1), (3, 4, 40), (2, 48, 3), (1, 1, 1)])
def test_dft_matches_numpy_fft(shape):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3) + shape) + 1j * rng.standard_normal((2, 3) + shape)
    ref = np.fft.fftn(x, axes=(-3, -2, -1))
    assert np.allclose(fft3(x), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert np.allclose(ifft3(fft3(x)), x, atol=1e-13)


def test_paper_window_lists():
    # even N: k - N/2, odd N: k - (N-1)/2 for k = 0..N-1
    assert list(paper_window(6)) == [-3, -2, -1, 0, 1, 2]
    assert list(paper_window(5)) == [-2, -1, 0, 1, 2]


@pytest.mark.parametrize("N", [1, 2, 5, 6, 16, 40])
def test_labels_at_zero_are_fftfreq(N):
    # Nyquist label is -N/2 (storage index N/2), as numpy's fftfreq
    assert np.array_equal(labels(N, 1.0, 0.0), np.rint(np.fft.fftfreq(N) * N).astype(int))


def test_labels_window_follows_kappa():
    L = 2.0 * np.pi
    N = 6
    # kappa = 1/2 (X point): the paper's window, centred: m + kappa in [-5/2, 5/2]
    m = labels(N, L, 0.5)
    assert sorted(m + 0.5) == [-2.5, -1.5, -0.5, 0.5, 1.5, 2.5]
    # kappa = 0.7 is kappa - 1 = -0.3 with the window shifted by one
    m = labels(N, L, 0.7)
    assert np.allclose(sorted(m + 0.7), sorted(labels(N, L, -0.3) - 0.3))
    # storage index j holds a label congruent to j mod N
    assert np.all(np.mod(m, N) == np.arange(N))


def test_shifted_wavevector_units():
    q = shifted_wavevector((4, 1, 2), (1e-3, 2e-3, 1e-3), (100.0, 0.0, -50.0))
    assert np.allclose(q[0], 2 * np.pi * np.array([0, 1, -2, -1]) / 1e-3 + 100.0)
    assert np.allclose(q[1], [0.0])
    assert np.allclose(q[2], 2 * np.pi * np.array([0, -1]) / 1e-3 - 50.0)
