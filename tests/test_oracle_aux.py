"""Pins for the alternative auxiliary functions v (Remark on the construction
of v, Sec. 3.4): the C^k polynomials with v'(x) = c x^k (x - 1)^k and the
C-infinity function built from s(x) = exp(-(1/(1+x)^2 + 1/(1-x)^2)).

Checked against what the mathematics fixes: end values, the point symmetry
v(x) + v(1 - x) = 1 the frame needs, the derivative against the Beta-function
normalisation c = (-1)^k (2k+1)! / (k!)^2, order of flatness at the ends, the
k = 3 case against the printed eq. (v), and the partitions of unity and the
frame identity with each choice."""

from math import factorial

import numpy as np
import pytest

from oracle import windows as ow
from oracle.complex_shearlets import one_sided_spectra
from oracle.spectra import spectra
from oracle.transform import adjoint, forward

AUX = [1, 2, 3, 5, 8, "inf"]


@pytest.mark.parametrize("aux", AUX)
def test_ends_midpoint_symmetry_monotone(aux):
    assert ow.v(0.0, aux) == 0.0
    assert abs(ow.v(1.0, aux) - 1.0) < 1e-13
    assert abs(ow.v(0.5, aux) - 0.5) < 1e-13
    x = np.linspace(-0.5, 1.5, 4001)
    assert np.max(np.abs(ow.v(x, aux) + ow.v(1.0 - x, aux) - 1.0)) < 1e-12
    t = np.linspace(0.0, 1.0, 2001)
    assert np.all(np.diff(ow.v(t, aux)) >= -1e-15)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6, 8])
def test_polynomial_derivative_and_flatness(k):
    c = (-1) ** k * factorial(2 * k + 1) / factorial(k) ** 2
    x = np.linspace(0.02, 0.98, 49)
    h = 1e-6
    fd = (ow.v(x + h, k) - ow.v(x - h, k)) / (2 * h)
    exact = c * x**k * (x - 1.0) ** k
    assert np.max(np.abs(fd - exact)) < 1e-6 * max(1.0, np.max(np.abs(exact)))
    # v(t) = c' t^(k+1) + O(t^(k+2)) near 0 with c' = |c| / (k + 1)
    t = 1e-3
    assert abs(ow.v(t, k) / t ** (k + 1) - abs(c) / (k + 1)) < 0.05 * abs(c) / (k + 1) + 1e-6


def test_k3_is_the_printed_polynomial():
    t = np.linspace(0.0, 1.0, 1001)
    printed = 35 * t**4 - 84 * t**5 + 70 * t**6 - 20 * t**7
    # the printed monomial form loses ~100 ulp to cancellation near t = 1
    assert np.max(np.abs(ow._v_poly(t, 3) - printed)) < 1e-13


def test_cinf_is_flat_at_both_ends():
    t = np.array([0.01, 0.02, 0.03, 0.05])
    assert np.all(ow.v(t, "inf") < t ** 12)
    assert np.all(1.0 - ow.v(1.0 - t, "inf") < t ** 12)
    # strictly increasing inside (beyond 0.8, 1 - v is below one ulp of 1)
    x = np.linspace(0.2, 0.8, 61)
    assert np.all(np.diff(ow.v(x, "inf")) > 0)


@pytest.mark.parametrize("aux", [1, 5, "inf"])
def test_partitions_of_unity(aux):
    # Lemma (propertySumbj) for |w| >= 1, and Theorem (PropertyPsi2).
    w = np.linspace(1.0, 3000.0, 20001)
    total = sum(ow.b(2.0 ** (-j) * w, aux) ** 2 for j in range(-1, 40))
    assert np.max(np.abs(total - 1.0)) < 1e-13
    om = np.linspace(-1.0, 1.0, 2001)
    for j in range(3):
        s = sum(ow.psi2(k + 2.0**j * om, aux) ** 2 for k in range(-2**j - 2, 2**j + 3))
        assert np.max(np.abs(s - 1.0)) < 1e-13
    # psi1^2 + varphi^2 = 1 on (1/2, 1), eq. (overlapPsi1Phi)
    u = np.linspace(0.51, 0.99, 49)
    assert np.max(np.abs(ow.psi1(u, aux) ** 2 + ow.varphi(u, aux) ** 2 - 1.0)) < 1e-14


@pytest.mark.parametrize("aux", [1, 5, "inf"])
@pytest.mark.parametrize("shearlet", ["meyer", "smooth"])
@pytest.mark.parametrize("M,N", [(64, 64), (48, 64)])
def test_frame_identity_and_reconstruction(aux, shearlet, M, N):
    psi = spectra(M, N, 2, shearlet=shearlet, aux=aux)
    assert np.max(np.abs((psi ** 2).sum(0) - 1.0)) < 1e-13
    f = np.random.default_rng(3).standard_normal((M, N))
    assert np.max(np.abs(adjoint(forward(f, psi), psi) - f)) < 1e-12
    pp = one_sided_spectra(M, N, 2, shearlet=shearlet, aux=aux)
    mir = pp[:, (-np.arange(M)) % M][:, :, (-np.arange(N)) % N]
    assert np.max(np.abs((pp ** 2 + mir ** 2).sum(0) - 2.0)) < 1e-13


def test_other_choices_change_the_spectra():
    base = spectra(64, 64, 2)
    for aux in (1, 5, "inf"):
        assert np.max(np.abs(spectra(64, 64, 2, aux=aux) - base)) > 1e-3
