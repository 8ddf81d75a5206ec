"""Pins for the oracle's spectra, index order and Nyquist fix (Sec. 3.1-3.2,
Sec. 3.5.1-3.5.2, Sec. 3.6, Sec. 3.8.1)."""

import numpy as np
import pytest

from oracle.grid import grid_spacing, signed_index
from oracle.spectra import (index_table, num_spectra, spectra, symmetrize_line,
                            symmetrize_nyquist, spectrum_plane)


def test_counts(golden):
    tab = golden("paper_tables.txt")
    for entry in tab["eta"].split():
        J, eta = (int(x) for x in entry.split(":"))
        assert num_spectra(J) == eta == len(index_table(J))
    for entry in tab["per_scale"].split():
        j, n = (int(x) for x in entry.split(":"))
        assert sum(1 for (_, jj, _) in index_table(3) if jj == j) == n


def test_index_order_text():
    # Sec. 3.5.2: per scale h k=0, h k=-1..-2^j+1, seam k=-2^j, v k=-2^j+1..2^j-1,
    # seam k=2^j, h k=2^j-1..1; low-pass first.
    assert index_table(1) == [("lowpass", -1, 0), ("h", 0, 0), ("hv", 0, -1),
                              ("v", 0, 0), ("hv", 0, 1)]
    assert index_table(2)[5:] == [("h", 1, 0), ("h", 1, -1), ("hv", 1, -2),
                                  ("v", 1, -1), ("v", 1, 0), ("v", 1, 1),
                                  ("hv", 1, 2), ("h", 1, 1)]


PARSEVAL_CASES = [(8, 8, 1, "max"), (64, 64, 2, "max"), (63, 65, 2, "max"),
                  (256, 512, 3, "max"), (512, 256, 3, "max"), (384, 512, 3, "max"),
                  (512, 512, 3, "max"), (128, 128, 3, "min"), (96, 64, 2, "max")]


@pytest.mark.parametrize("M,N,J,ms", PARSEVAL_CASES)
def test_parseval_identity(M, N, J, ms, golden):
    # Theorem of Sec. 3.2 on the grid; the paper measures 8e-15 (Sec. 3.6).
    psi = spectra(M, N, J, max_scale=ms)
    dev = np.max(np.abs((psi ** 2).sum(axis=0) - 1.0))
    assert dev < 1e-13
    assert float(golden("paper_tables.txt")["frame_tightness"]) < 1e-13
    assert np.all(psi >= 0) and np.all(psi <= 1 + 1e-15)


def _direction_pins(M, N, J):
    """Grid points on the centre ray of each shearlet, inside the flat band
    4^j <= |t| <= 2 4^j of psi1(4^-j t) and off the Nyquist lines. There the
    shearlet's psi2 factor is psi2(0) = 1, every other shear of the scale sees
    psi2(+-1) = 0 or less, and psi1 vanishes at every other scale, so exactly
    one spectrum is 1 and all others are 0. The centre ray of (h, j, k) and of
    the seam elements is w2 / w1 = -k / 2^j; that of (v, j, k) is
    w1 / w2 = -k / 2^j."""
    d = grid_spacing(M, N, J)
    pins = []
    for i, (kind, j, k) in enumerate(index_table(J)):
        if kind == "lowpass":
            continue
        P = 2 ** j
        for s in (1, -1):
            for q in range(int(np.ceil(4 ** j / d)), int(np.floor(2 * 4 ** j / d)) + 1):
                if (q * k) % P:
                    continue
                along, across = s * q, s * (-k * q // P)
                q1, q2 = (across, along) if kind == "v" else (along, across)
                if -(N // 2) < q1 < (N + 1) // 2 and -(M // 2) < q2 < (M + 1) // 2:
                    pins.append((i, (q2 % M, q1 % N)))
                    break
    return pins


@pytest.mark.parametrize("M,N,J", [(512, 512, 3), (64, 64, 2), (256, 512, 3),
                                   (128, 128, 3), (1024, 1024, 5)])
def test_direction_pins(M, N, J):
    pins = _direction_pins(M, N, J)
    eta = num_spectra(J)
    if M == N and M >= 128:
        # square grids reach the flat band of every scale along both axes
        assert {i for i, _ in pins} == set(range(1, eta))
    for i, (r, c) in pins:
        col = _column_at(M, N, J, r, c)
        assert col[i] == pytest.approx(1.0, abs=1e-15), (i, r, c)
        # zero up to cos(pi/2) = 6e-17 where a band edge falls on the point
        assert np.all(np.abs(np.delete(col, i)) < 1e-16), (i, r, c)


def _column_at(M, N, J, r, c):
    # Evaluate all spectra at one grid point on a tiny sub-grid: the
    # spectra depend only on (w1, w2), so a 1x1 evaluation is enough.
    from oracle.spectra import spectrum
    d = grid_spacing(M, N, J)
    w1 = np.array([[signed_index(N)[c] * d]])
    w2 = np.array([[signed_index(M)[r] * d]])
    return np.array([spectrum(kind, j, k, w1, w2)[0, 0] for (kind, j, k) in index_table(J)])


@pytest.mark.parametrize("M,N,J", [(64, 64, 2), (256, 256, 3), (128, 256, 3), (63, 65, 2)])
def test_point_symmetry(M, N, J):
    # The spectra are real and even on the grid after the Nyquist fix, which is
    # what makes the coefficients real (Sec. 3.8.1).
    psi = spectra(M, N, J)
    flipped = psi[:, (-np.arange(M)) % M][:, :, (-np.arange(N)) % N]
    assert np.array_equal(psi, flipped)


@pytest.mark.parametrize("M,J", [(64, 2), (256, 3)])
def test_transpose_and_mirror(M, J):
    psi = spectra(M, M, J)
    tab = index_table(J)
    where = {t: i for i, t in enumerate(tab)}
    mirror = (-np.arange(M)) % M
    for i, (kind, j, k) in enumerate(tab):
        # transposition swaps the cones (eq. verticalShearlet)
        twin = {"h": "v", "v": "h"}.get(kind, kind)
        np.testing.assert_allclose(psi[i].T, psi[where[(twin, j, k)]], rtol=0, atol=1e-15)
        # omega_2 -> -omega_2 reverses the shear: psi2 is even. The corner
        # (-X, -X) is its own mirror on the grid while (-X, +X) is not a grid
        # point, so the two diagonal seam elements differ there; skip it.
        a = psi[i][mirror, :].copy()
        b = psi[where[(kind, j, -k)]].copy()
        a[M // 2, M // 2] = b[M // 2, M // 2] = 0.0
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


def test_realreal_toy_row(golden):
    # Toy row of Sec. 3.8.1: centred order, frequencies -4..4.
    tab = golden("realreal_toy.txt")
    before = np.array([float(x) for x in tab["before"].split()])
    after = np.array([float(x) for x in tab["after_times_sqrt2"].split()]) / np.sqrt(2.0)
    centred = np.arange(-4, 5)
    natural = np.empty(9)
    natural[centred % 9] = before
    fixed = symmetrize_line(natural)
    np.testing.assert_allclose(fixed[centred % 9], after, rtol=0, atol=1e-15)


def test_fix_touches_only_nyquist_and_keeps_axis_shearlets():
    M = N = 256
    J = 3
    raw = spectra(M, N, J, real_real=False)
    fixed = symmetrize_nyquist(raw)
    diff = np.abs(raw - fixed) > 0
    inner = diff.copy()
    inner[:, M // 2, :] = False
    inner[:, :, N // 2] = False
    assert not inner.any()
    tab = index_table(J)
    changed = {tab[i] for i in range(len(tab)) if diff[i].any()}
    # Sec. 3.8.1: only finest-scale spectra change; the shear-0 horizontal and
    # vertical ones are kept.
    assert changed and all(j == J - 1 for (_, j, _) in changed)
    assert ("h", J - 1, 0) not in changed and ("v", J - 1, 0) not in changed
    # the fix keeps the sum of squares
    np.testing.assert_allclose((fixed ** 2).sum(0), (raw ** 2).sum(0), rtol=0, atol=1e-14)


def test_support_in_scale_band():
    # supp psi1 = [1/2, 4] in |w| (Theorem PropertyPsi1) dilated by 4^j.
    M = N = 256
    J = 3
    d = grid_spacing(M, N, J)
    q = np.abs(signed_index(N)) * d
    for i, (kind, j, k) in enumerate(index_table(J)):
        if kind != "h":
            continue
        plane = spectrum_plane(M, N, J, i)
        # (values of 6e-17 = cos(pi/2) at the outer band edge count as zero)
        cols = (plane > 1e-15).any(axis=0)
        assert np.all(q[cols] > 4 ** j / 2) and np.all(q[cols] < 4 ** (j + 1))
