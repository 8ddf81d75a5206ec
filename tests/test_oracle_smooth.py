"""Pins for the smooth-shearlet variant (Sec. 3.4)."""

import numpy as np
import pytest

from oracle.grid import frequencies, grid_spacing, signed_index
from oracle.smooth import corona, smooth_spectrum, tensor_lowpass
from oracle.spectra import index_table, spectra
from oracle.transform import adjoint, forward
from oracle.windows import varphi


def test_corona_support_and_telescoping():
    # Sec. 3.4: Psi1 is supported in the Cartesian corona [-4,4]^2 \ [-1/2,1/2]^2
    # and Phi^2(w) + sum_j Psi1^2(4^-j w) = 1.
    g = np.linspace(-6, 6, 481)
    w1, w2 = np.meshgrid(g, g, indexing="ij")
    c = corona(w1, w2)
    inner = (np.abs(w1) <= 0.5) & (np.abs(w2) <= 0.5)
    outer = (np.abs(w1) >= 4.0) | (np.abs(w2) >= 4.0)
    assert np.all(c[inner] == 0.0) and np.all(c[outer] < 1e-7)
    total = tensor_lowpass(w1, w2) ** 2 + sum(corona(w1 / 4.0 ** j, w2 / 4.0 ** j) ** 2 for j in range(12))
    assert np.max(np.abs(total - 1.0)) < 1e-14
    # tensor low-pass is the product of the one-dimensional ones (eq. Phi)
    assert tensor_lowpass(0.75, 0.75) == pytest.approx(varphi(0.75) ** 2)


@pytest.mark.parametrize("M,N,J", [(64, 64, 2), (256, 256, 3), (128, 256, 3), (63, 65, 2)])
def test_smooth_parseval_on_grid(M, N, J):
    psi = spectra(M, N, J, shearlet="smooth")
    assert np.max(np.abs((psi ** 2).sum(0) - 1.0)) < 1e-13


def test_smooth_direction_pins():
    # On a shearlet's centre ray in its flat band the corona is 1 (the inner
    # tensor low-pass vanishes, the outer one is 1) and psi2 is 1 only for that
    # shearlet, as in the Meyer case.
    M = N = 256
    J = 3
    d = grid_spacing(M, N, J)
    tab = index_table(J)
    w1, w2 = frequencies(M, N, J)
    for i, (kind, j, k) in enumerate(tab):
        if kind == "lowpass":
            continue
        P = 2 ** j
        q = int(np.ceil(4 ** j / d))
        q += (-q) % P
        along, across = q, -k * q // P
        q1, q2 = (across, along) if kind == "v" else (along, across)
        r, c = q2 % M, q1 % N
        col = np.array([smooth_spectrum(kk, jj, ss, w1[r:r + 1, c:c + 1], w2[r:r + 1, c:c + 1])[0, 0]
                        for (kk, jj, ss) in tab])
        assert col[i] == pytest.approx(1.0, abs=1e-15)
        assert np.all(np.abs(np.delete(col, i)) < 1e-15)


def test_smooth_transform_is_parseval():
    rng = np.random.default_rng(11)
    f = rng.standard_normal((64, 64))
    psi = spectra(64, 64, 2, shearlet="smooth")
    c = forward(f, psi, return_complex=True)
    assert np.max(np.abs(c.imag)) < 1e-12
    assert abs(np.sum(c.real ** 2) / np.sum(f ** 2) - 1) < 1e-12
    assert np.max(np.abs(adjoint(c.real, psi) - f)) < 1e-12


def test_smooth_lowpass_is_the_tensor_one():
    # cone low-pass varphi(max |w_i|) (eq. phi) vs tensor varphi(w1) varphi(w2)
    # (eq. Phi): equal on the axes, different at (3/4, 3/4)
    M = N = 256
    J = 3   # Delta = 1/4
    a = spectra(M, N, J)[0]
    b = spectra(M, N, J, shearlet="smooth")[0]
    assert np.allclose(a[0, :], b[0, :]) and np.allclose(a[:, 0], b[:, 0])
    assert a[3, 3] == pytest.approx(varphi(0.75)) and b[3, 3] == pytest.approx(varphi(0.75) ** 2)
