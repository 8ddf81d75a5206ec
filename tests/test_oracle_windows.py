"""Pins for the oracle's window functions (Sec. 2.1, Sec. 2.4, Sec. 3.4).

Each check is a value or identity the paper states (or plain calculus), not a
re-typing of the oracle's own formula."""

import numpy as np
import pytest

from oracle.windows import b, psi1, psi2, v, varphi

S2 = np.sqrt(2.0) / 2.0


def test_v_values_and_clamping():
    assert v(0.0) == 0.0 and v(1.0) == pytest.approx(1.0, abs=1e-15)
    assert v(0.5) == pytest.approx(0.5, abs=1e-15)
    assert np.all(v(np.array([-3.0, -1e-9])) == 0.0)
    assert np.all(v(np.array([1.0 + 1e-9, 7.0])) == 1.0)


def test_v_point_symmetry():
    # Lemma in Sec. 2.1: v(x) + v(1 - x) = 1 for all real x.
    x = np.linspace(-2.0, 3.0, 20001)
    # the expanded polynomial has coefficients up to 84, so allow ~100 ulp
    assert np.max(np.abs(v(x) + v(1.0 - x) - 1.0)) < 5e-14


def test_v_derivative():
    # Remark on the construction of v: v'(x) = -140 x^3 (x - 1)^3 on [0, 1],
    # so v' vanishes to third order at both ends.
    x = np.linspace(0.01, 0.99, 99)
    h = 1e-6
    fd = (v(x + h) - v(x - h)) / (2 * h)
    assert np.max(np.abs(fd - (-140.0 * x**3 * (x - 1.0) ** 3))) < 1e-7
    # Flat to third order at the ends: v(e +- t) - v(e) = O(t^4).
    t = 1e-3
    assert abs(v(t) - v(0.0)) < 1e-10 and abs(v(1.0) - v(1.0 - t)) < 1e-10


def test_b_support_and_peak():
    # Sec. 2.1: b is even, nonnegative, supported on [-4,-1] u [1,4], b(+-2) = 1.
    assert b(2.0) == pytest.approx(1.0) and b(-2.0) == pytest.approx(1.0)
    w = np.linspace(-6, 6, 12001)
    vals = b(w)
    assert np.all(vals >= 0)
    assert np.all(vals[(np.abs(w) < 1.0) | (np.abs(w) > 4.0)] == 0.0)
    assert np.all(vals[(np.abs(w) > 1.001) & (np.abs(w) < 3.999)] > 0)
    assert np.array_equal(vals, b(-w))


def test_b_squares_partition():
    # Lemma (propertySumbj): sum_{j >= -1} b^2(2^-j w) = 1 for |w| >= 1,
    # with the stated ramp sin^2(pi/2 v(2w - 1)) on (1/2, 1) and 0 below 1/2.
    w = np.concatenate([np.linspace(0.0, 1.0, 4001), np.linspace(1.0, 5000.0, 20001)])
    total = sum(b(2.0 ** (-j) * w) ** 2 for j in range(-1, 40))
    ramp = np.where(w <= 0.5, 0.0,
                    np.where(w < 1.0, np.sin(np.pi / 2 * v(2 * w - 1)) ** 2, 1.0))
    assert np.max(np.abs(total - ramp)) < 1e-14


def test_psi1_closed_form():
    # Sec. 3.4 prints psi1-hat piecewise: 0, sin(pi/2 v(2|w| - 1)), 1,
    # cos(pi/2 v(|w|/2 - 1)), 0 on the breakpoints 1/2, 1, 2, 4.
    w = np.linspace(-6, 6, 24001)
    a = np.abs(w)
    closed = np.select(
        [a <= 0.5, a < 1.0, a <= 2.0, a < 4.0],
        [0.0, np.sin(np.pi / 2 * v(2 * a - 1)), 1.0, np.cos(np.pi / 2 * v(a / 2 - 1))],
        default=0.0)
    assert np.max(np.abs(psi1(w) - closed)) < 1e-15


def test_psi1_special_values_and_scale_partition():
    assert psi1(0.75) == pytest.approx(S2, abs=1e-15)
    assert psi1(3.0) == pytest.approx(S2, abs=1e-15)
    # at |w| = 4 eq. (b) gives cos(pi/2), which is zero up to rounding
    assert psi1(1.5) == 1.0 and psi1(0.5) == 0.0 and abs(psi1(4.0)) < 1e-16
    # Theorem (PropertyPsi1) and eq. (OverlapPsi1_2).
    w = np.concatenate([np.linspace(0.0, 1.0, 2001), np.linspace(1.0, 1e5, 20001)])
    total = sum(psi1(4.0 ** (-j) * w) ** 2 for j in range(0, 20))
    ramp = np.where(w <= 0.5, 0.0,
                    np.where(w < 1.0, np.sin(np.pi / 2 * v(2 * w - 1)) ** 2, 1.0))
    assert np.max(np.abs(total - ramp)) < 1e-14


def test_psi1_finite_scale_sum():
    # eq. (sum_over_finite_scales) with j0 scales, read with the exponent
    # 2^(-2 j0 + 1) in the cosine (the only one giving 1 at w = 2^(2 j0 - 1)
    # and 0 at 2^(2 j0)).
    for j0 in (1, 2, 3, 4):
        w = np.linspace(0.0, 2.0 ** (2 * j0 + 1), 40001)
        total = sum(psi1(4.0 ** (-j) * w) ** 2 for j in range(j0))
        lo, hi = 2.0 ** (2 * j0 - 1), 2.0 ** (2 * j0)
        expect = np.select(
            [w <= 0.5, w < 1.0, w <= lo, w < hi],
            [0.0, np.sin(np.pi / 2 * v(2 * w - 1)) ** 2, 1.0,
             np.cos(np.pi / 2 * v(2.0 ** (-2 * j0 + 1) * w - 1)) ** 2],
            default=0.0)
        assert np.max(np.abs(total - expect)) < 1e-14


def test_psi2_values_and_partitions():
    assert psi2(0.0) == 1.0 and psi2(1.0) == 0.0 and psi2(-1.0) == 0.0
    assert psi2(0.5) == pytest.approx(S2, abs=1e-15) and psi2(-0.5) == pytest.approx(S2, abs=1e-15)
    w = np.linspace(-3, 3, 6001)
    assert np.all(psi2(w)[np.abs(w) >= 1.0] == 0.0)
    assert np.array_equal(psi2(w), psi2(-w))
    # Lemma (PropertyPsi2): three shifted squares sum to 1 on |w| <= 1.
    x = np.linspace(-1, 1, 4001)
    s3 = psi2(x - 1) ** 2 + psi2(x) ** 2 + psi2(x + 1) ** 2
    assert np.max(np.abs(s3 - 1)) < 5e-14
    # Theorem (PropertyPsi2): sum_{k=-2^j}^{2^j} psi2(k + 2^j w)^2 = 1, |w| <= 1.
    for j in range(0, 6):
        tot = sum(psi2(k + 2.0 ** j * x) ** 2 for k in range(-2 ** j, 2 ** j + 1))
        assert np.max(np.abs(tot - 1)) < 5e-14


def test_scaling_function():
    # Sec. 2.4: varphi = 1 on [0, 1/2], 0 from 1 on, and eq. (overlapPsi1Phi):
    # psi1^2 + varphi^2 = 1 on [1/2, 1].
    assert varphi(0.0) == 1.0 and varphi(0.5) == 1.0 and varphi(1.0) == 0.0
    assert varphi(0.75) == pytest.approx(S2, abs=1e-15)
    w = np.linspace(0.5, 1.0, 5001)
    assert np.max(np.abs(psi1(w) ** 2 + varphi(w) ** 2 - 1)) < 5e-15
    w = np.linspace(-3, 3, 6001)
    assert np.array_equal(varphi(w), varphi(-w))
