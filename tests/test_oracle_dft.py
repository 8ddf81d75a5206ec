"""Pins for the oracle's DFT and textbook FFT."""

import itertools

import numpy as np
import pytest

from oracle.dft import dft2, direct_dft, fft, idft2
from paper_1202_1773_amd.synthetic import gaussian


def test_direct_dft_brute_force_8x8():
    # Config-1 check: an 8x8 Gaussian image, seed 102, against the double sum
    # written out with Python loops.
    x = gaussian(8, 8, seed=102).astype(np.float64)
    X = dft2(x)
    for k2, k1 in itertools.product(range(8), range(8)):
        s = 0j
        for n2, n1 in itertools.product(range(8), range(8)):
            s += x[n2, n1] * np.exp(-2j * np.pi * (n2 * k2 / 8 + n1 * k1 / 8))
        assert abs(X[k2, k1] - s) < 1e-12


@pytest.mark.parametrize("L", list(range(1, 41)) + [48, 64, 96, 128, 192, 243, 256])
def test_fft_equals_direct(L):
    rng = np.random.default_rng(L)
    x = rng.standard_normal((3, L)) + 1j * rng.standard_normal((3, L))
    for sign in (-1, 1):
        ref = direct_dft(x, sign)
        got = fft(x, axis=-1, sign=sign)
        assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_impulse_constant_and_parseval():
    L = 96
    e = np.zeros(L)
    e[0] = 1.0
    np.testing.assert_allclose(fft(e), np.ones(L), atol=1e-14)
    one = np.ones(L)
    expect = np.zeros(L, complex)
    expect[0] = L
    np.testing.assert_allclose(fft(one), expect, atol=1e-12)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((48, 64))
    X = dft2(x)
    assert abs(np.sum(np.abs(X) ** 2) - 48 * 64 * np.sum(x ** 2)) < 1e-9 * np.sum(x ** 2) * 48 * 64


@pytest.mark.parametrize("shape", [(8, 8), (64, 64), (384, 512), (512, 512), (24, 96)])
def test_against_numpy_fft_and_inverse(shape):
    rng = np.random.default_rng(7)
    x = rng.standard_normal(shape)
    X = dft2(x)
    ref = np.fft.fft2(x)  # an outside library, used only here as a cross-check
    assert np.max(np.abs(X - ref)) < 1e-10 * np.max(np.abs(ref))
    np.testing.assert_allclose(idft2(X).real, x, atol=1e-12)
    assert np.max(np.abs(idft2(X).imag)) < 1e-12
