"""Pins for the oracle's forward / adjoint / inverse transform (Sec. 3.1-3.3,
Sec. 3.6, Sec. 3.8.1)."""

import numpy as np
import pytest

from oracle.spectra import spectra
from oracle.transform import adjoint, forward, inverse
from paper_1202_1773_amd.synthetic import cartoon, config1_image, gaussian


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_config1_reconstruction_and_energy(golden):
    # 64x64 cartoon, J = 2 (13 spectra). The paper measures about 2e-15 for
    # the transform exactness (Sec. 3.6); the bound here is 1e-13.
    f = config1_image().astype(np.float64)
    psi = spectra(64, 64, 2)
    assert psi.shape[0] == 13
    c = forward(f, psi)
    assert np.max(np.abs(inverse(c, psi) - f)) < 1e-13 * np.max(np.abs(f))
    assert float(golden("paper_tables.txt")["transform_exactness"]) < 1e-13
    # energy: Parseval frame, sum_i ||c_i||^2 = ||f||^2
    assert abs(np.sum(c ** 2) - np.sum(f ** 2)) < 1e-12 * np.sum(f ** 2)


def test_frame_matrix_8x8():
    # eq. (shearlet_transform_as_matrix): rows of U are the frame elements;
    # Parseval frame <=> U^T U = I (and U U^T != I: not a basis).
    M = N = 8
    psi = spectra(M, N, 1)
    eye = np.eye(M * N).reshape(M * N, M, N)
    U = forward(eye, psi).reshape(M * N, -1).T   # (eta * M * N, M * N)
    assert U.shape == (5 * 64, 64)
    assert np.max(np.abs(U.T @ U - np.eye(64))) < 1e-13
    assert np.max(np.abs(U @ U.T - np.eye(5 * 64))) > 0.1


def test_adjoint_dot_product():
    rng = np.random.default_rng(3)
    M, N, J = 48, 64, 2
    psi = spectra(M, N, J)
    f = rng.standard_normal((M, N))
    c = rng.standard_normal((psi.shape[0], M, N))
    lhs = np.sum(forward(f, psi) * c)
    rhs = np.sum(f * adjoint(c, psi))
    assert abs(lhs - rhs) < 1e-12 * np.sqrt(np.sum(f ** 2) * np.sum(c ** 2))


@pytest.mark.parametrize("p,q", [(0, 0), (3, 5), (7, 0), (0, 11), (16, 16), (32, 5),
                                 (5, 32), (32, 32), (-3, 9), (20, -27)])
def test_plane_wave(p, q):
    # f = cos(2 pi (p r / M + q c / N)) has its spectrum on (p, q) and (-p, -q);
    # every spectrum is even on the grid, so c_i = Psi_i[p, q] * f. This fixes
    # the pairing rows <-> omega_2, columns <-> omega_1 and the 1/(MN) factor.
    M = N = 64
    psi = spectra(M, N, 2)
    r, cc = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    f = np.cos(2 * np.pi * (p * r / M + q * cc / N))
    c = forward(f, psi)
    for i in range(psi.shape[0]):
        np.testing.assert_allclose(c[i], psi[i, p % M, q % N] * f, atol=1e-13)


def test_constant_image():
    # phi-hat(0) = 1 and every shearlet vanishes at the origin.
    psi = spectra(32, 32, 2)
    c = forward(np.full((32, 32), 2.5), psi)
    np.testing.assert_allclose(c[0], 2.5, atol=1e-14)
    assert np.max(np.abs(c[1:])) < 1e-14


def test_shift_equivariance():
    # Translation invariance: t_m = m on the full grid (Sec. 3.1).
    rng = np.random.default_rng(5)
    f = rng.standard_normal((32, 48))
    psi = spectra(32, 48, 2)
    c = forward(f, psi)
    cs = forward(np.roll(f, (3, -7), axis=(0, 1)), psi)
    np.testing.assert_allclose(cs, np.roll(c, (3, -7), axis=(1, 2)), atol=1e-13)


def test_realness_with_and_without_fix():
    # Sec. 3.8.1: with the Nyquist fix the coefficients are real; without it
    # the finest-scale planes of an even-sized image pick up imaginary parts.
    f = gaussian(64, 64, seed=9).astype(np.float64)
    fixed = forward(f, spectra(64, 64, 2), return_complex=True)
    assert np.max(np.abs(fixed.imag)) < 1e-12 * np.max(np.abs(f))
    raw = forward(f, spectra(64, 64, 2, real_real=False), return_complex=True)
    assert np.max(np.abs(raw.imag)) > 1e-3


def test_odd_sizes_need_no_fix():
    # Remark in Sec. 3.8.1: odd sizes keep the symmetry without the fix.
    f = gaussian(63, 65, seed=4).astype(np.float64)
    raw = forward(f, spectra(63, 65, 2, real_real=False), return_complex=True)
    assert np.max(np.abs(raw.imag)) < 1e-12 * np.max(np.abs(f))


def test_streamed_planes_match_stack():
    f = cartoon(32, 32, 3, 2, 0.1, seed=1).astype(np.float64)
    psi = spectra(32, 32, 2)
    full = forward(f, psi)
    part = forward(f, lambda i: psi[i], planes=[0, 4, 12])
    np.testing.assert_array_equal(part, full[[0, 4, 12]])
