"""Pins for the oracle's scale count and frequency grid (Sec. 3.1, Sec. 3.5.1)."""

import numpy as np
import pytest

from oracle.grid import (default_scales, frequencies, grid_extent, grid_spacing,
                         signed_index)


def test_scale_table(golden):
    table = golden("paper_tables.txt")["scales"].split()
    for entry in table:
        rng, j0 = entry.split(":")
        lo, hi = (int(x) for x in rng.split("-"))
        for n in range(lo, hi + 1):
            assert default_scales(n, 1) == int(j0)
            assert default_scales(1, n) == int(j0)


def test_extent_and_spacing():
    # X = 2^(2 j0 - 1) and Delta = 1 exactly when N = 2^(2 j0) + 1 (Sec. 3.5.1).
    for j0 in range(1, 6):
        N = 2 ** (2 * j0) + 1
        assert default_scales(N, N) == j0
        assert grid_spacing(N, N, j0) == 1.0
    # For the default number of scales 1/4 < Delta <= 1 (Sec. 3.5.1).
    for N in range(4, 1025):
        d = grid_spacing(N, N, default_scales(N, N))
        assert 0.25 < d <= 1.0
    assert grid_extent(3, "max") == 32.0 and grid_extent(3, "min") == 16.0


@pytest.mark.parametrize("D", [1, 2, 3, 4, 7, 8, 9, 16, 31, 64, 511, 512])
def test_signed_index_is_omega(D):
    q = signed_index(D)
    # Omega = {-floor(D/2), ..., ceil(D/2) - 1} (Sec. 3.1), natural DFT order.
    assert sorted(q.tolist()) == list(range(-(D // 2), (D + 1) // 2))
    assert np.array_equal(q, np.round(np.fft.fftfreq(D) * D).astype(int))


def test_grid_range_matches_odd_extension():
    # Odd extension to 2n+1 points on [-X, X], drop the last one (Sec. 3.5.1):
    # an even axis of the larger side runs over [-X, X - Delta].
    for (M, N, J) in [(512, 512, 3), (64, 64, 2), (256, 512, 3), (513, 513, 4)]:
        w1, w2 = frequencies(M, N, J)
        X = grid_extent(J)
        d = grid_spacing(M, N, J)
        L = max(M, N)
        axis = w1[0] if N == L else w2[:, 0]
        assert axis.min() == -X
        assert axis.max() == (X - d if L % 2 == 0 else X)
        # rows carry omega_2, columns omega_1
        assert np.all(w1 == w1[0:1, :]) and np.all(w2 == w2[:, 0:1])
