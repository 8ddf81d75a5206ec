"""Discrete Fourier transforms for the oracle: a direct DFT and a textbook FFT.

Test infrastructure only (see the package header).

Conventions (the ones the paper's fft2/ifft2 calls use, Sec. 3.1): the forward
transform is unnormalised with kernel exp(-2 pi i n k / L); the inverse has
kernel exp(+2 pi i n k / L) and the factor 1/L per axis.

The FFT is the textbook recursive decimation in time: for a factor p of the
length L = p m, split x into the p subsequences x[r::p], transform each with
length m, and combine as X[k] = sum_r exp(-+2 pi i r k / L) X_r[k mod m].
Factors 2 and 3 are split off; short or other lengths use the direct DFT.

Pinned by tests/test_oracle_dft.py: brute-force agreement with the direct
DFT, the DFT of a unit impulse and of a constant, Parseval's formula, the
inverse property, and agreement with numpy.fft as an outside library.
"""

import numpy as np

DIRECT_MAX = 16


def direct_dft(x, sign=-1):
    """Direct O(L^2) DFT along the last axis with kernel exp(sign 2 pi i n k / L)."""
    x = np.asarray(x, dtype=np.complex128)
    L = x.shape[-1]
    n = np.arange(L)
    kernel = np.exp(sign * 2j * np.pi * np.outer(n, n) / L)
    return x @ kernel.T


def _fft_last(x, sign):
    L = x.shape[-1]
    if L <= DIRECT_MAX:
        return direct_dft(x, sign)
    for p in (2, 3):
        if L % p == 0:
            m = L // p
            parts = [_fft_last(x[..., r::p], sign) for r in range(p)]
            k = np.arange(L)
            out = np.zeros(x.shape, dtype=np.complex128)
            for r in range(p):
                out += np.exp(sign * 2j * np.pi * r * k / L) * parts[r][..., k % m]
            return out
    return direct_dft(x, sign)


def fft(x, axis=-1, sign=-1):
    """Unnormalised DFT along one axis (textbook FFT)."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    return np.moveaxis(_fft_last(x, sign), -1, axis)


def dft2(x):
    """fft2: unnormalised 2-D DFT over the last two axes."""
    return fft(fft(x, axis=-1, sign=-1), axis=-2, sign=-1)


def idft2(X):
    """ifft2: 2-D inverse DFT over the last two axes, with the 1/(M N) factor."""
    M, N = X.shape[-2], X.shape[-1]
    return fft(fft(X, axis=-1, sign=+1), axis=-2, sign=+1) / (M * N)
