"""Own discrete Fourier transform and discrete frequencies (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

DFT convention: forward  U^(m) = sum_x u(x) exp(-2 pi i j m / N)  (unnormalized),
inverse u(x) = (1/N) sum_m U^(m) exp(+2 pi i j m / N).  The paper does not fix
the normalization; K = F C F^-1 and M = F rho F^-1 do not depend on it.

Pins: tests/test_oracle_fourier.py checks the DFT against numpy.fft (an
independent implementation) and the frequency window against the paper's
explicit lists for odd and even N.
"""
from __future__ import annotations

import math

import numpy as np

_CACHE: dict = {}


def dft_matrix(N: int, inverse: bool = False) -> np.ndarray:
    """N x N DFT matrix W[j, n] = exp(-+2 pi i j n / N) (inverse scaled by 1/N)."""
    key = (N, inverse)
    if key not in _CACHE:
        j = np.arange(N)
        ph = (np.outer(j, j) % N) / N          # reduce the phase before the exponential
        W = np.exp((2j if inverse else -2j) * np.pi * ph)
        if inverse:
            W = W / N
        _CACHE[key] = W
    return _CACHE[key]


def _along(x: np.ndarray, W: np.ndarray, axis: int) -> np.ndarray:
    """Apply matrix W along one of the last three axes of x (..., N0, N1, N2)."""
    if axis == 2:
        return x @ W.T
    if axis == 1:
        return W @ x
    sh = x.shape
    y = W @ x.reshape(sh[:-3] + (sh[-3], sh[-2] * sh[-1]))
    return y.reshape(sh)


def fft3(x: np.ndarray) -> np.ndarray:
    """Forward 3D DFT over the last three axes."""
    y = x.astype(np.complex128, copy=False)
    for a in range(3):
        y = _along(y, dft_matrix(y.shape[-3 + a]), a)
    return y


def ifft3(x: np.ndarray) -> np.ndarray:
    """Inverse 3D DFT over the last three axes."""
    y = x.astype(np.complex128, copy=False)
    for a in range(3):
        y = _along(y, dft_matrix(y.shape[-3 + a], inverse=True), a)
    return y


def paper_window(N: int) -> np.ndarray:
    """Integer frequency labels listed by the paper for index k = 0..N-1.

    Sec. 3.1 eq. "frequencies": k - (N-1)/2 for odd N, k - N/2 for even N.  This
    is the set of labels; the storage position of label m is m mod N.
    """
    return np.arange(N) - (N - 1) // 2 if N % 2 else np.arange(N) - N // 2


def window_shift(kappa: float) -> int:
    """g = ceil(kappa - 1/2) so that kappa - g lies in (-1/2, 1/2] (1e-9 slack at the edge)."""
    return int(math.ceil(kappa - 0.5 - 1e-9))


def labels(N: int, L: float, k: float) -> np.ndarray:
    """Frequency label m(j) stored at DFT index j = 0..N-1 for Bloch wavenumber k.

    The label set is the paper's window shifted by -g (g from the reduced wave
    number kappa = k L / 2 pi), so that m + kappa is centred; for kappa in
    (-1/2, 1/2] this is exactly the paper's window.  Storage: m = j (mod N).
    """
    kappa = k * L / (2.0 * np.pi)
    lo = int(paper_window(N)[0]) - window_shift(kappa)
    j = np.arange(N)
    return lo + np.mod(j - lo, N)


def snap_wavevector(L, k) -> np.ndarray:
    """k with every component within 1e-9 (in units of 2 pi / L_a) of a whole
    reciprocal vector replaced by that vector, so that xi + k = 0 holds exactly
    on one voxel when k is a reciprocal lattice vector up to rounding."""
    k = np.array(k, dtype=np.float64)
    for a in range(3):
        kappa = k[a] * L[a] / (2.0 * np.pi)
        g = float(np.rint(kappa))
        if abs(kappa - g) <= 1e-9:
            k[a] = 2.0 * np.pi * g / L[a]
    return k


def shifted_wavevector(n, L, k) -> list:
    """Per-axis arrays q_a(j) = 2 pi m_a(j) / L_a + k_a (Sec. 3.2, xi + k)."""
    k = snap_wavevector(L, k)
    return [2.0 * np.pi * labels(n[a], L[a], k[a]) / L[a] + k[a] for a in range(3)]
