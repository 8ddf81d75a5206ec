"""Scales and the discrete frequency grid (Sec. 3.1, Sec. 3.5.1).

Test infrastructure only (see the package header).

Layout reading: the first array axis (rows, length M) carries omega_2 and the
second axis (columns, length N) carries omega_1, as in the stack description
of Sec. 3.5.2. Arrays are in natural DFT order (index 0 = zero frequency,
negative frequencies in the upper half), so no fftshift is ever needed.

Pinned by tests/test_oracle_grid.py: the scale table and the rule
X = 2^(2 j0 - 1) of Sec. 3.5.1, Delta = 1 exactly when N = 2^(2 j0) + 1,
and the index set Omega of Sec. 3.1.
"""

import numpy as np


def default_scales(M, N):
    """Number of scales j0 = floor(1/2 log2 max(M, N)) (Sec. 3.1, Sec. 3.5.1).

    Computed on integers so that exact powers of two never round down."""
    L = int(max(M, N))
    if L < 1:
        raise ValueError("image size must be positive")
    return (L.bit_length() - 1) // 2


def grid_extent(J, max_scale="max"):
    """Largest grid frequency X (Sec. 3.5.1): X3 = 2^(2J-1) for 'max' and the
    alternative X2 = 2^(2J-2) for 'min' (option maxScale, Sec. 3.5.3)."""
    if max_scale == "max":
        return 2.0 ** (2 * J - 1)
    if max_scale == "min":
        return 2.0 ** (2 * J - 2)
    raise ValueError("max_scale must be 'max' or 'min'")


def grid_spacing(M, N, J, max_scale="max"):
    """Spacing Delta = 2X / (L_odd - 1) of Sec. 3.5.1, with L the larger side
    extended to the next odd length. One spacing serves both axes."""
    L = int(max(M, N))
    L_odd = L + 1 if L % 2 == 0 else L
    return 2.0 * grid_extent(J, max_scale) / (L_odd - 1)


def signed_index(D):
    """Signed frequency of each natural DFT index of an axis of length D:
    p for p <= ceil(D/2) - 1, otherwise p - D. This enumerates the index set
    Omega of Sec. 3.1 (-floor(D/2) .. ceil(D/2) - 1); it is also what the
    odd-extend-then-drop-the-last-entry rule of Sec. 3.5.1 yields."""
    p = np.arange(D)
    top = (D + 1) // 2 - 1
    return np.where(p <= top, p, p - D)


def frequencies(M, N, J, max_scale="max"):
    """Grid points (omega_1, omega_2) as two (M, N) float64 arrays."""
    delta = grid_spacing(M, N, J, max_scale)
    q1 = signed_index(N).astype(np.float64) * delta
    q2 = signed_index(M).astype(np.float64) * delta
    w1 = np.broadcast_to(q1[None, :], (M, N)).copy()
    w2 = np.broadcast_to(q2[:, None], (M, N)).copy()
    return w1, w2
