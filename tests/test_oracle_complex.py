"""Pins for the complex (one-sided) shearlet reading of Sec. 3.8.2."""

import numpy as np
import pytest

from oracle.complex_shearlets import adjoint_real, forward, one_sided_spectra, orientation
from oracle.dft import dft2
from oracle.grid import frequencies
from oracle.spectra import index_table, spectra
from oracle.transform import forward as real_forward


@pytest.mark.parametrize("M,N,J", [(64, 64, 2), (32, 48, 2), (63, 65, 2)])
def test_parseval_and_reconstruction(M, N, J):
    rng = np.random.default_rng(M + N)
    f = rng.standard_normal((M, N))
    pp = one_sided_spectra(M, N, J)
    c = forward(f, pp)
    assert abs(np.sum(np.abs(c) ** 2) / np.sum(f ** 2) - 1) < 1e-12
    assert np.max(np.abs(adjoint_real(c, pp) - f)) < 1e-12
    # grid pairs: |Psi+(w)|^2 + |Psi+(-w)|^2 = Psi(w)^2 + Psi(-w)^2
    mir = pp[:, (-np.arange(M)) % M][:, :, (-np.arange(N)) % N]
    psi = spectra(M, N, J)
    pmir = psi[:, (-np.arange(M)) % M][:, :, (-np.arange(N)) % N]
    np.testing.assert_allclose(pp ** 2 + mir ** 2, psi ** 2 + pmir ** 2, atol=1e-14)


def test_coefficient_spectra_are_one_sided():
    M = N = 64
    J = 2
    f = np.random.default_rng(1).standard_normal((M, N))
    pp = one_sided_spectra(M, N, J)
    c = forward(f, pp)
    w1, w2 = frequencies(M, N, J)
    for i, (kind, j, k) in enumerate(index_table(J)):
        d = orientation(kind, j, k)
        if d is None:
            continue
        C = dft2(c[i])
        neg = (w1 * d[0] + w2 * d[1]) < 0
        # negative side is empty except where the mirror pair is not split
        # (Nyquist lines), which the one-sided spectrum keeps as is
        nyq = np.zeros((M, N), bool)
        nyq[M // 2, :] = True
        nyq[:, N // 2] = True
        assert np.max(np.abs(C[neg & ~nyq])) < 1e-9


@pytest.mark.parametrize("p,q", [(3, 9), (9, -3), (5, 0), (0, 7), (6, 6), (7, -7), (-4, 10)])
def test_plane_wave_gives_analytic_signal(p, q):
    # cos(theta) with theta = 2 pi (p r / M + q c / N): for a shearlet whose
    # positive side holds (p, q), c+_i = Psi_i(p, q) / sqrt(2) * exp(i theta).
    M = N = 64
    J = 2
    r, cc = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    theta = 2 * np.pi * (p * r / M + q * cc / N)
    f = np.cos(theta)
    pp = one_sided_spectra(M, N, J)
    psi = spectra(M, N, J)
    c = forward(f, pp)
    w1, w2 = frequencies(M, N, J)
    for i, (kind, j, k) in enumerate(index_table(J)):
        d = orientation(kind, j, k)
        if d is None:
            np.testing.assert_allclose(c[i], psi[i, p % M, q % N] * f, atol=1e-13)
            continue
        side = w1[p % M, q % N] * d[0] + w2[p % M, q % N] * d[1]
        expect = psi[i, p % M, q % N] / np.sqrt(2.0) * np.exp(1j * (theta if side > 0 else -theta))
        np.testing.assert_allclose(c[i], expect, atol=1e-13)


def test_real_part_is_the_real_transform_off_nyquist():
    # Away from the Nyquist lines Re c+_i = c_i / sqrt(2) for i >= 1.
    M = N = 64
    J = 2
    rng = np.random.default_rng(4)
    F = np.fft.fft2(rng.standard_normal((M, N)))
    F[M // 2, :] = 0
    F[:, N // 2] = 0
    f = np.fft.ifft2(F).real
    c = forward(f, one_sided_spectra(M, N, J))
    cr = real_forward(f, spectra(M, N, J))
    np.testing.assert_allclose(c[0].real, cr[0], atol=1e-13)
    np.testing.assert_allclose(c[1:].real, cr[1:] / np.sqrt(2.0), atol=1e-13)
